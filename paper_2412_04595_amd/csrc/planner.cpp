// Parameter selection and host-side tables (float64).
//
// The choices follow the paper's parameter-selection procedure (Sec. 4.3) with the
// error estimates of Sec. 2.3 (Thm thm:SOG, Table 1), Sec. 4.1 (Thms thm::trunFour,
// thm::scal, thm::pad) and Sec. 4.2 (Thm thm::Fcheb, with Thm thm::Che), and a cost
// model for this GPU in place of eq. optimiz's CPU cost ratio.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>
#include <cstring>

#include "internal.hpp"

namespace sog {

// Gauss-Legendre rule of n points on [-1, 1]: the roots of P_n by Newton's method from
// the Chebyshev-like initial guesses cos(pi (i + 3/4) / (n + 1/2)), weights
// 2 / ((1 - x^2) P_n'(x)^2).  Cached per n.
const std::vector<double>& gauss_legendre(int n) {
    static std::mutex mu;
    static std::map<int, std::vector<double>> cache;  // n nodes, then n weights
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(n);
    if (it != cache.end()) return it->second;
    std::vector<double> xw(2 * (size_t)n);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double x = std::cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it2 = 0; it2 < 100; ++it2) {
            double p0 = 1.0, p1 = x;  // P_0, P_1, then the three-term recurrence up to P_n
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p0 = 1.0; p1 = x; }
            dp = n * (x * p1 - p0) / (x * x - 1.0);  // P_n'(x)
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        const double w = 2.0 / ((1.0 - x * x) * dp * dp);
        xw[i] = -x;
        xw[n - 1 - i] = x;
        xw[n + i] = w;
        xw[2 * n - 1 - i] = w;
    }
    return cache.emplace(n, std::move(xw)).first->second;
}

// The ES window psi(d) = exp(beta (sqrt(1 - (d/a)^2) - 1)), |d| < a = P_w/2 (grid units).
// Its transform by x = a sin(theta): 2 a int_0^{pi/2} exp(beta (cos theta - 1))
// cos(kappa a sin theta) cos theta dtheta, an entire function of theta; Gauss-Legendre on
// [0, pi/2] with enough points for the oscillation converges geometrically (a composite
// Simpson rule of 96 panels had left 2e-11 of the transform at P_w = 5).
double es_hat_grid(double kappa, int Pw, double beta) {
    const double a = 0.5 * Pw;
    const int n = 64 + (int)std::ceil(2.0 * std::fabs(kappa) * a);
    const std::vector<double>& xw = gauss_legendre(n);
    const double hp = 0.25 * 3.14159265358979323846;  // [0, pi/2] = hp (t + 1)
    double sum = 0;
    for (int i = 0; i < n; ++i) {
        const double th = hp * (xw[i] + 1.0);
        sum += xw[n + i] * std::exp(beta * (std::cos(th) - 1.0)) * std::cos(kappa * a * std::sin(th)) * std::cos(th);
    }
    return 2.0 * a * hp * sum;
}

// The Kaiser-Bessel window W(d) = I_0(beta sqrt(1 - (d/a)^2)) / I_0(beta), |d| <= a = P_w/2
// (grid units; one of the windows of Remark rmk::PWindow, no formula printed), and its
// transform: the truncated window's standard closed form
//   What_g(kappa) = (2 a / I_0(beta)) sinh(z) / z,  z = sqrt(beta^2 - (kappa a)^2),
// continued as sin(z') / z', z' = sqrt((kappa a)^2 - beta^2), beyond kappa a = beta.
// I_0 and I_1 by their power series, summed in long double: every term is positive, so
// the sum keeps its relative accuracy for any argument (the window's beta stays below 60).
long double bessel_i0_ld(long double x) {
    const long double t = 0.25L * x * x;
    long double term = 1.0L, sum = 1.0L;
    for (int k = 1; k < 400; ++k) {
        term *= t / ((long double)k * k);
        sum += term;
        if (term < 1e-21L * sum) break;
    }
    return sum;
}

double bessel_i0(double x) { return (double)bessel_i0_ld(x); }

double bessel_i1(double x) {
    const long double t = 0.25L * (long double)x * x;
    long double term = 0.5L * x, sum = term;
    for (int k = 1; k < 400; ++k) {
        term *= t / ((long double)k * (k + 1));
        sum += term;
        if (std::fabs(term) < 1e-21L * std::fabs(sum)) break;
    }
    return (double)sum;
}

// the window in long double: the polynomial fit interpolates these samples, and the
// derivative of an interpolant of degree nu magnifies sample errors up to 2 nu^2-fold at
// the ends of its interval (Markov's inequality), 4e-13 from samples rounded to double
long double kb_value_ld(long double d, int Pw, long double beta) {
    const long double a = 0.5L * Pw;
    const long double t = d / a;
    if (!(std::fabs(t) <= 1.0L)) return 0.0L;
    return bessel_i0_ld(beta * std::sqrt((1.0L - t) * (1.0L + t))) / bessel_i0_ld(beta);
}

double kb_value_grid(double d, int Pw, double beta) { return (double)kb_value_ld(d, Pw, beta); }

double kb_hat_grid(double kappa, int Pw, double beta) {
    const double a = 0.5 * Pw;
    const double z2 = beta * beta - kappa * kappa * a * a;
    double f = 1.0;
    if (z2 > 1e-12) {
        const double z = std::sqrt(z2);
        f = std::sinh(z) / z;
    } else if (z2 < -1e-12) {
        const double z = std::sqrt(-z2);
        f = std::sin(z) / z;
    }
    return 2.0 * a * f / bessel_i0(beta);
}

// Remark rmk::PWindow: the weight a particle at offset u in [-1/2, 1/2] (grid units) from
// its nearest node puts on node o (o = 0 .. P_w - 1, at o - (P_w-1)/2 from that node),
// W(o - (P_w-1)/2 - u), replaced by its Chebyshev interpolant of degree nu on that
// interval (the nu + 1 first-kind points), written in monomials of u, highest degree first
// (the order Horner's rule takes): coef[o (nu + 1) + j] multiplies u^(nu - j).
void window_poly_fit(int Pw, double beta, int nu, std::vector<double>& coef) {
    const long double pi = 3.14159265358979323846264338327950288L;
    coef.assign((size_t)Pw * (nu + 1), 0.0);
    const int hw = (Pw - 1) / 2;
    const int np = nu + 1;
    // T_k(2u) in monomials of u: T_0 = 1, T_1 = 2u, T_{k+1} = 4u T_k - T_{k-1}
    std::vector<std::vector<long double>> T(np, std::vector<long double>(np, 0.0L));
    T[0][0] = 1.0L;
    if (np > 1) T[1][1] = 2.0L;
    for (int k = 1; k + 1 < np; ++k)
        for (int j = 0; j < np; ++j)
            T[k + 1][j] = (j > 0 ? 4.0L * T[k][j - 1] : 0.0L) - T[k - 1][j];
    std::vector<long double> f(np);
    for (int o = 0; o < Pw; ++o) {
        for (int j = 0; j < np; ++j) {
            const long double t = std::cos((j + 0.5L) * pi / np);
            f[j] = kb_value_ld((long double)(o - hw) - 0.5L * t, Pw, beta);
        }
        std::vector<long double> mono(np, 0.0L);
        for (int k = 0; k < np; ++k) {
            long double c = 0.0L;
            for (int j = 0; j < np; ++j) c += f[j] * std::cos((long double)k * (j + 0.5L) * pi / np);
            c *= 2.0L / np;
            if (k == 0) c *= 0.5L;
            for (int j = 0; j < np; ++j) mono[j] += c * T[k][j];
        }
        for (int j = 0; j <= nu; ++j) coef[(size_t)o * np + j] = (double)mono[nu - j];
    }
}

// Largest deviation of the fitted weights from the window, and (derr) of their derivative
// in u from the window's, over 201 offsets per node; the derivative relative to its
// largest value.
double window_poly_error(int Pw, double beta, int nu, const std::vector<double>& coef, double* derr) {
    const int hw = (Pw - 1) / 2;
    double ew = 0, ed = 0, dmax = 0;
    const double inv_i0 = 1.0 / bessel_i0(beta);
    for (int o = 0; o < Pw; ++o)
        for (int i = 0; i <= 200; ++i) {
            const double u = -0.5 + i / 200.0;
            const double* c = coef.data() + (size_t)o * (nu + 1);
            double w = c[0], dw = 0;
            for (int j = 1; j <= nu; ++j) {
                dw = dw * u + w;
                w = w * u + c[j];
            }
            const double d = (double)(o - hw) - u;
            const double t = std::min(1.0, std::fabs(d) / (0.5 * Pw));
            const double r = std::sqrt((1.0 - t) * (1.0 + t));
            ew = std::max(ew, std::fabs(w - bessel_i0(beta * r) * inv_i0));
            if (derr) {
                // d/du W(d(u)) = -W'(d) = beta (d / a^2) I_1(beta r) / (r I_0(beta)), -> beta^2 d / (2 a^2 I_0) at r = 0
                const double a2 = 0.25 * Pw * Pw;
                const double ex = r > 1e-12 ? beta * d / a2 * bessel_i1(beta * r) / r * inv_i0
                                            : 0.5 * beta * beta * d / a2 * inv_i0;
                ed = std::max(ed, std::fabs(dw - ex));
                dmax = std::max(dmax, std::fabs(ex));
            }
        }
    if (derr) *derr = dmax > 0 ? ed / dmax : ed;
    return ew;
}

// The polynomial degree (Sec. 4: chosen adaptively): the smallest nu in [4, kMaxWinPoly]
// whose weights are within eps / 20 of the window (the window's own aliasing is held to
// eps / 4), or kMaxWinPoly.
int window_poly_degree(int Pw, double beta, double eps) {
    std::vector<double> c;
    for (int nu = 4; nu < kMaxWinPoly; ++nu) {
        window_poly_fit(Pw, beta, nu, c);
        if (window_poly_error(Pw, beta, nu, c, nullptr) <= eps / 20.0) return nu;
    }
    return kMaxWinPoly;
}

namespace {

struct Row {
    double b, r0, omega, eE;
    int ME;
    double eF;
    int MF;
};
// Table 1 (tabl:parameter).
const Row kTable1[6] = {
    {2.0, 1.9892536839080267, 0.9944464927622323, 3.12e-2, 16, 9.93e-3, 11},
    {1.62976708826776469, 2.7520026668023417, 1.0078069793438068, 2.33e-3, 31, 6.21e-4, 16},
    {1.48783512395703226, 3.7554672283554990, 0.9919117057598183, 2.29e-4, 46, 7.98e-5, 26},
    {1.32070036405934420, 4.3914554711638349, 1.0018891411481198, 1.18e-6, 76, 5.76e-7, 41},
    {1.21812525709410644, 5.6355288151271085, 1.0009014615603334, 7.14e-10, 166, 5.14e-10, 71},
    {1.14878150173321925, 7.2956245490719404, 1.0000368348358225, 1.30e-15, 271, 1.98e-14, 116},
};

// GPU cost model: seconds per unit of work of the float32 kernels on MI355X, fitted to
// the kernels' event times at N = 10^6 on the cube for two windows and grid sizes (float64
// takes about twice as long in every term, the near field's included since its candidate
// test runs on the matrix cores in float32 for both forms: the same ranking serves both).
// It only ranks candidate discretisations, all of which meet the error model.
constexpr double kCostNearPair = 5.6e-12;   // per neighbour pair within r_c
constexpr double kCostSpreadSlot = 1.0e-10; // per particle per gridding lane update (x planes of a wave x 64-node passes)
constexpr double kCostGatherPt = 1.7e-13;   // per particle per window point of the gathering
constexpr double kCostFFTPt = 1.4e-11;      // per real grid point: FFT chain, tile halo loads and adds
constexpr double kCostLongDirect = 1.0e-12; // per particle per (half-plane mode x Chebyshev term)
constexpr double kCostWindow2Pt = 9.0e-13;  // per particle per 2D window point per Chebyshev term
constexpr double kCostFFT2Pt = 3.6e-11;     // per 2D grid point per Chebyshev term

const double kPi = 3.14159265358979323846;

bool is_smooth(int n) {
    if (n <= 0) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Exponent E of the Gaussian-window error exp(-E) for P_w points at spacing h for the
// narrowest Gaussian s: the larger of erfc(sqrt(S)) ~ exp(-S) and the aliasing term
// exp(-pi^2 mu (P_w-1)^2 / (4 s^2 S)), mu = s^2 - H^2/S (Thm thm::scal), balanced over S.
// Returns E and the balancing S.
double window_exponent(int Pw, double h, double s, double* S_out) {
    double u = Pw - 1;
    double a = kPi * kPi * u * u / 4.0;
    double c = (u * h / 2.0) * (u * h / 2.0) / (s * s);  // H^2 / s^2
    if (8.0 * c * c >= a) {
        // the aliasing exponent a/S - a c/S^2 peaks below S: best S is its peak
        if (S_out) *S_out = 2.0 * c;
        return a / (4.0 * c);
    }
    double lo = 2.0 * c, hi = std::sqrt(a);  // root of S^3 - a S + a c in (2c, sqrt(a))
    for (int it = 0; it < 100; ++it) {
        double mid = 0.5 * (lo + hi);
        double f = mid * mid * mid - a * mid + a * c;
        if (f < 0) lo = mid; else hi = mid;
    }
    double S = 0.5 * (lo + hi);
    if (S_out) *S_out = S;
    return S;
}

int tile_edge(int prec, int Pw) {
    // LDS of the gridding kernel (tile, halo and staging; the gathering kernel needs less)
    // within tile_lds_budget(P_w)
    const size_t rs = (prec == SOG_PREC_FP64) ? 8 : 4;
    for (int B = 16; B >= 1; --B)
        if (spread_lds_bytes(rs, Pw, B, B, B) <= tile_lds_budget(Pw, rs)) return B;
    return 1;
}

// The gridding kernel's lanes take the (y, z) nodes of a window, 64 per pass; node
// (oy, oz) of a window whose corner is at LDS word c sits at c + oy HZ + oz.  When every
// residue of oy HZ + oz modulo 64 occurs at most once per pass, lane (oy HZ + oz) mod 64
// can take it and the 64 lanes of a pass hit 64 distinct banks for any corner.
bool spread_pitch_conflict_free(int Pw, int HZ) {
    const int npass = (Pw * Pw + 63) / 64;
    int cnt[64] = {0};
    for (int oy = 0; oy < Pw; ++oy)
        for (int oz = 0; oz < Pw; ++oz)
            if (++cnt[(oy * HZ + oz) % 64] > npass) return false;
    return true;
}

// Tile of the gridding and gathering kernels.  float32: among z extents whose halo pitch
// is conflict-free, the tile with the largest share of owned nodes in its halo block that
// fits tile_lds_budget(P_w) of LDS; float64 (two banks per value anyway), or no such extent: the
// largest cube.
void spread_tile(int prec, int Pw, int B[3]) {
    const int c = tile_edge(prec, Pw);
    B[0] = B[1] = B[2] = c;
    if (prec == SOG_PREC_FP64) return;
    double best = (double)c * c * c / std::pow((double)(c + Pw - 1), 3);
    for (int bz = std::max(1, Pw - 1); bz <= 40; ++bz) {
        const int HZ = bz + Pw - 1;
        if (!spread_pitch_conflict_free(Pw, HZ)) continue;
        int bxy = 32;
        while (bxy > 1 && spread_lds_bytes(4, Pw, bxy, bxy, bz) > tile_lds_budget(Pw, 4)) --bxy;
        if (spread_lds_bytes(4, Pw, bxy, bxy, bz) > tile_lds_budget(Pw, 4)) continue;
        const double eff = (double)bxy * bxy * bz / ((double)(bxy + Pw - 1) * (bxy + Pw - 1) * HZ);
        if (eff >= 0.97 * best) {
            best = std::max(best, eff);
            B[0] = B[1] = bxy;
            B[2] = bz;
        }
    }
}

// Deterministic gridding (see tile_colour): per direction, m = 1 + ceil((P_w - 1) / B)
// colours repeat so that two tiles of one colour have m - 1 full tiles between them; in x
// and y (periodic) the tiles after the last whole run of m, the short last tile among
// them, get colours of their own, so no run of m crosses the short tile or the wrap.  A
// block must not wrap onto itself either: B + P_w - 1 <= I (the edge shrinks until it
// holds).  z is not periodic: t mod m with m at most the tile count.  False if a periodic
// direction has fewer than two tiles' room.
bool deterministic_tiles(int Pw, const int gI[3], int B[3], int nt[3], int m[3], int q[3], int ncol[3]) {
    for (int d = 0; d < 3; ++d) {
        const bool periodic = d < 2;
        if (periodic)
            while (B[d] > 1 && B[d] + Pw - 1 > gI[d]) --B[d];
        if (periodic && B[d] + Pw - 1 > gI[d]) return false;
        nt[d] = (gI[d] + B[d] - 1) / B[d];
        m[d] = 1 + (Pw - 1 + B[d] - 1) / B[d];
        if (!periodic) {
            m[d] = std::min(m[d], nt[d]);
            q[d] = 0;
            ncol[d] = m[d];
            continue;
        }
        const int full = gI[d] % B[d] == 0 ? nt[d] : nt[d] - 1;
        q[d] = full / m[d];
        ncol[d] = m[d] + (nt[d] - q[d] * m[d]);
    }
    return true;
}

// Lane of each window node per pass (see spread_pitch_conflict_free); when the pitch is
// not conflict-free, nodes in row order.  A lane left without a node in a pass gets, where
// possible, a dummy node that the kernel updates with zero weight: an offset from the
// window corner that no window node has, that stays in the corner's x plane for every
// corner in the tile (offset <= P_w H_Z - B_z), that no other dummy uses, and preferably
// one in the lane's own bank.  Returns false, leaving such lanes at -1, when there are
// not enough of them.
bool spread_lane_nodes(int Pw, int HZ, int Bz, signed char* noy, signed char* noz) {
    for (int i = 0; i < 4 * 64; ++i) noy[i] = noz[i] = -1;
    if (Pw < 1 || Pw > kMaxPw) return false;  // the table holds 4 passes of 64 nodes
    if (spread_pitch_conflict_free(Pw, HZ)) {
        int used[64] = {0};
        for (int oy = 0; oy < Pw; ++oy)
            for (int oz = 0; oz < Pw; ++oz) {
                const int lane = (oy * HZ + oz) % 64;
                const int ps = used[lane]++;
                noy[ps * 64 + lane] = (signed char)oy;
                noz[ps * 64 + lane] = (signed char)oz;
            }
    } else {
        for (int k = 0; k < Pw * Pw && k < 4 * 64; ++k) {
            noy[k] = (signed char)(k / Pw);
            noz[k] = (signed char)(k % Pw);
        }
    }
    const int npass = (Pw * Pw + 63) / 64;
    std::vector<int> cand;
    for (int oy = 0; oy < Pw; ++oy)
        for (int oz = Pw; oz < HZ; ++oz)
            if (oy * HZ + oz <= Pw * HZ - Bz) cand.push_back(oy * HZ + oz);
    std::vector<char> taken(cand.size(), 0);
    std::vector<int> open;
    for (int k = 0; k < npass * 64; ++k)
        if (noy[k] < 0) open.push_back(k);
    std::vector<int> pick(open.size(), -1);
    for (int round = 0; round < 2; ++round)
        for (size_t i = 0; i < open.size(); ++i) {
            if (pick[i] >= 0) continue;
            for (size_t c = 0; c < cand.size(); ++c)
                if (!taken[c] && (round == 1 || cand[c] % 64 == open[i] % 64)) {
                    taken[c] = 1;
                    pick[i] = (int)c;
                    break;
                }
        }
    for (size_t i = 0; i < open.size(); ++i)
        if (pick[i] < 0) return false;
    for (size_t i = 0; i < open.size(); ++i) {
        noy[open[i]] = (signed char)(cand[pick[i]] / HZ);
        noz[open[i]] = (signed char)(cand[pick[i]] % HZ);
    }
    return true;
}

struct MidChoice {
    bool ok = false;
    int I[3] = {0, 0, 0};
    int Izs = 0, Pw = 0;
    double S = 0, cost = 1e300;
    int window = SOG_WINDOW_GAUSSIAN;
    double beta = 0;
    int nu = 0;
};

// Aliasing estimate of the ES and KB windows.  Gridding and gathering each fold the spectrum of
// the spread charge onto the grid's band; for the narrowest mid-range Gaussian s (1D,
// normalised to G(0) = 1) the error is about
//   (1/pi) int_0^pi sqrt(pi) (s/h) exp(-(s/h)^2 kappa^2 / 4) R(kappa) dkappa,
//   R(kappa) = sum_{n=1,2} (|What_g(2 pi n - kappa)| + |What_g(2 pi n + kappa)|) / What_g(kappa),
// in grid units.  R depends only on (P_w, beta), so it is tabulated once per pair.  Against
// a 1D simulation of gridding, FFT, deconvolution and gathering the estimate is within a
// factor 2 of the measured error.
constexpr int kEsK = 65;                                   // kappa points on [0, pi]
constexpr double kEsShape[] = {1.6, 1.8, 2.0, 2.2, 2.4, 2.6};  // beta / P_w candidates
constexpr int kEsNShape = sizeof(kEsShape) / sizeof(kEsShape[0]);

// Per (window, P_w, beta): R(kappa_i) in [0, kEsK) and What_g(kappa_i) / What_g(0) in
// [kEsK, 2 kEsK).
const std::vector<double>& es_ratio(int window, int Pw, double beta) {
    static std::mutex mu;
    static std::map<std::pair<int, long long>, std::vector<double>> cache;
    const std::pair<int, long long> key(Pw * 4 + window, std::llround(beta * 1e9));
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    // a composite Simpson rule in theta with the panels the largest argument (5 pi) needs,
    // the nodes shared by every argument (an estimate: its accuracy is ample)
    const double a = 0.5 * Pw;
    const int nq = 2 * (48 + (int)std::ceil(2.0 * 5.0 * kPi * a));
    const double dth = 0.5 * kPi / nq;
    std::vector<double> f(nq + 1), x(nq + 1);
    for (int i = 0; i <= nq; ++i) {
        const double th = i * dth;
        f[i] = std::exp(beta * (std::cos(th) - 1.0)) * std::cos(th) * ((i == 0 || i == nq) ? 1.0 : ((i & 1) ? 4.0 : 2.0));
        x[i] = a * std::sin(th);
    }
    auto hat = [&](double kappa) {
        if (window == SOG_WINDOW_KB) return kb_hat_grid(kappa, Pw, beta);
        double sum = 0;
        for (int i = 0; i <= nq; ++i) sum += f[i] * std::cos(kappa * x[i]);
        return 2.0 * a * sum * dth / 3.0;
    };
    std::vector<double> R(2 * kEsK);
    const double wzero = hat(0.0);
    for (int i = 0; i < kEsK; ++i) {
        const double k = kPi * i / (kEsK - 1);
        double al = 0;
        for (int nn = 1; nn <= 2; ++nn) al += std::fabs(hat(2 * kPi * nn - k)) + std::fabs(hat(2 * kPi * nn + k));
        const double w0 = hat(k);
        R[i] = w0 > 0 ? al / w0 : 1e300;
        R[kEsK + i] = w0 / wzero;
    }
    return cache.emplace(key, std::move(R)).first->second;
}

// The deconvolution multiplies each direction's spectrum by Ghat(k) / What(k)^2; where that
// grows above its value at k = 0 it amplifies the rounding of the spread grid (float32: a
// window with What(pi) / What(0) ~ 1e-5, a flat ES window on a coarse grid, amplified it
// 1.5e5-fold and cost 1e-4 in the potential).  ES windows are accepted only where the
// growth stays below kEsAmpMax in every direction, as the Gaussian's does (it never grows).
constexpr double kEsAmpMax = 4.0;

double es_alias_estimate(int window, int Pw, double beta, double s_over_h) {
    const std::vector<double>& R = es_ratio(window, Pw, beta);
    double acc = 0;
    for (int i = 0; i < kEsK; ++i) {
        const double k = kPi * i / (kEsK - 1);
        const double e = std::exp(-s_over_h * s_over_h * k * k / 4.0);
        const double wn = R[kEsK + i];
        if (!(wn > 0) || e / (wn * wn) > kEsAmpMax) return 1e300;
        acc += std::sqrt(kPi) * s_over_h * e * R[i] * ((i == 0 || i == kEsK - 1) ? 0.5 : 1.0);
    }
    return acc * (kPi / (kEsK - 1)) / kPi;
}

// The ES or KB window for spacing h: the smallest P_w (odd, at most kMaxPw) whose estimate
// meets eps / kEsMargin with the best beta of kEsShape (or the given P_w / beta); false if
// none.  The margin covers the estimate's shortfall on coarse grids (up to 2.5x against the
// 1D simulation at s/h = 2) and the forces, whose error is about 8x the potential's in the
// same simulation for either window.
constexpr double kEsMargin = 4.0;
bool es_window(int window, double h, double s0, double eps, const sog_params& ov, int* Pw_out, double* beta_out) {
    eps /= kEsMargin;
    for (int p = 3; p <= kMaxPw; p += 2) {
        if (ov.mid_Pw[0] > 0 && p != ov.mid_Pw[0]) continue;
        double best = 1e300, bbest = 0;
        for (int ci = 0; ci < kEsNShape; ++ci) {
            const double beta = ov.mid_beta > 0 ? ov.mid_beta : kEsShape[ci] * p;
            const double e = es_alias_estimate(window, p, beta, s0 / h);
            if (bbest == 0 || e < best) { best = e; bbest = beta; }
            if (ov.mid_beta > 0) break;
        }
        if (best <= eps || ov.mid_Pw[0] > 0) {
            *Pw_out = p;
            *beta_out = bbest;
            return true;
        }
    }
    return false;
}

MidChoice plan_mid(const double L[3], int64_t n, double s0, double sm, int nl, double eps, int prec,
                   const sog_params& ov) {
    MidChoice best;
    const double eps_t = eps, eps_w = eps, eps_p = eps;
    double hmax = kPi * s0 / (2.0 * std::sqrt(std::log(0.1 / eps_t)));
    // grid spacings as fractions of the coarsest that resolves s_0; the finer ones let the
    // widest window the kernels take (P_w = 15) reach tight tolerances
    const double fr[] = {1.0, 0.92, 0.85, 0.78, 0.7, 0.62, 0.55, 0.48, 0.42, 0.36};
    for (double f : fr) {
        MidChoice c;
        double h = f * hmax;
        for (int d = 0; d < 2; ++d) c.I[d] = next_smooth((int)std::ceil(L[d] / h - 1e-9), true);
        c.I[2] = std::max(1, (int)std::ceil(L[2] / h - 1e-9));
        if (ov.mid_I[0] > 0) for (int d = 0; d < 3; ++d) c.I[d] = ov.mid_I[d];
        double hd[3] = {L[0] / c.I[0], L[1] / c.I[1], L[2] / c.I[2]};
        double hw = std::max(hd[0], std::max(hd[1], hd[2]));
        const MidChoice grid = c;
        // the Gaussian window (eq. GS), the ES and the KB window, each where allowed
        const bool auto_shaped = ov.mid_window == SOG_WINDOW_AUTO && !(ov.mid_S > 0);
        const bool try_win[3] = {ov.mid_window == SOG_WINDOW_AUTO || ov.mid_window == SOG_WINDOW_GAUSSIAN,
                                 ov.mid_window == SOG_WINDOW_ES || auto_shaped,
                                 ov.mid_window == SOG_WINDOW_KB || auto_shaped};
        for (int win = 0; win < 3; ++win) {
            c = grid;
            int Pw = 0, nu = 0;
            double S = 0, beta = 0;
            if (!try_win[win]) continue;
            if (win == 0) {
                if (ov.mid_Pw[0] > 0) {
                    Pw = ov.mid_Pw[0];
                    window_exponent(Pw, hw, s0, &S);
                } else {
                    for (int p = 5; p <= kMaxPw; p += 2) {
                        double Sp;
                        double E = window_exponent(p, hw, s0, &Sp);
                        if (std::exp(-E) <= eps_w) { Pw = p; S = Sp; break; }
                    }
                    if (Pw == 0) continue;
                }
                if (ov.mid_S > 0) S = ov.mid_S;
            } else {
                const int kind = win == 1 ? SOG_WINDOW_ES : SOG_WINDOW_KB;
                if (!es_window(kind, hw, s0, eps_w, ov, &Pw, &beta)) continue;
                if (kind == SOG_WINDOW_KB) nu = ov.mid_nu;  // 0: chosen once the plan is (below)
            }
            for (int d = 0; d < 2; ++d)
                if (c.I[d] < 2 * Pw) c.I[d] = next_smooth(2 * Pw, true);
            // the x and y passes hold at least one complex line (and pitch) per block in LDS
            if (fft_x_lds_min_bytes(prec, c.I[0], nl, 1) > 65536 || fft_x_lds_min_bytes(prec, c.I[1], 0, 1) > 65536)
                continue;
            hd[0] = L[0] / c.I[0];
            hd[1] = L[1] / c.I[1];
            // the window's reach in z: (P_w - 1)/2 nodes (Gaussian), its support P_w/2 (ES)
            double Hz = (win == 0 ? 0.5 * (Pw - 1) : 0.5 * Pw) * hd[2];
            // padding (Thm thm::pad): the widest mid-range Gaussian must decay to eps over
            // the extension beyond the window's reach.  (Decay to sqrt(eps) was too little
            // for a cell with a large z dipole, whose image errors add up coherently: the
            // 2e5-particle layered electrolyte missed 1e-4 in the forces at m = 10.)
            double delta = sm * std::sqrt(std::log(1.0 / eps_p));
            double Lzs = L[2] + 2.0 * Hz + delta;
            int half = next_smooth((int)std::ceil(Lzs / hd[2] / 2.0 - 1e-9), false);
            c.Izs = 2 * half;
            while (c.Izs < c.I[2] + Pw + 2) c.Izs = 2 * next_smooth(c.Izs / 2 + 1, false);
            if (ov.mid_Izs > 0) c.Izs = ov.mid_Izs;
            c.Pw = Pw;
            c.S = S;
            c.window = win == 0 ? SOG_WINDOW_GAUSSIAN : (win == 1 ? SOG_WINDOW_ES : SOG_WINDOW_KB);
            c.beta = beta;
            c.nu = nu;
            double Ng = (double)c.I[0] * c.I[1] * c.Izs;
            // gridding: each wave updates ceil(P_w / 4) x planes times ceil(P_w^2 / 64)
            // passes of 64 (y, z) nodes per particle; gathering: P_w^3 points per particle
            const double slots = (double)((Pw + 3) / 4) * ((Pw * Pw + 63) / 64);
            // the x and y passes move batches of W lines (W n <= the line kernels' element
            // cap, W <= 16); below 8 lines a batch reads row segments of under 64 bytes, and
            // the passes slow down (8e6-particle cube: the y pass 1.7x per point at W = 4)
            const int wmin = std::min(fft_lines_per_batch(prec, c.I[0]), fft_lines_per_batch(prec, c.I[1]));
            const double fft_pen = wmin >= 8 ? 1.0 : 1.0 + 0.5 * std::log2(8.0 / wmin);
            c.cost = (double)n * (kCostSpreadSlot * slots + kCostGatherPt * Pw * Pw * Pw) + kCostFFTPt * Ng * fft_pen;
            // ES is charged 1% so that KB takes the ties: the ES window's derivative is
            // infinite at the edge of its support, and in float32 its gradients near the
            // edge lost up to 5e-3 of the mid range's largest (10^6 and 8e6 cubes; KB's
            // polynomials 2e-6, the same support and cost within 4%)
            if (win == 1) c.cost *= 1.01;
            c.ok = true;
            if (c.cost < best.cost) best = c;
        }
        if (ov.mid_I[0] > 0) break;
    }
    return best;
}

}  // namespace

namespace {

struct LongChoice {
    bool ok = false;
    int form = SOG_LONG_DIRECT, P = 0, nk[2] = {0, 0}, I2[2] = {0, 0}, Pw2 = 0, Q = 0, Ps = 0;
    double S2 = 0, cost = 1e300;
    std::string why;  // when not ok: the limit that ruled the form out
};

// Costs of the long range's FFT form (seconds, float32 kernels on MI355X; float64 about
// twice), fitted to the kernels' event times on the 10^6-particle confined box, slab and
// layered cell.  Gridding: every node of a 16 x 16 tile tests every particle of the (at
// most 3 x 3) tiles its windows can come from and stages those that reach it, 8 planes
// per pass, about 2048 tiles at once on the GPU: per candidate particle and pass.  Gathering: 64 particles of a tile at a
// time, about 1280 tiles at once: per batch, window node and pass.  Transforms per grid
// point and plane (each direction), scaling per mode and multiply-add of its z kernel.
constexpr double kCostL2Cand = 1.05e-7;
constexpr double kCostL2GatherNode = 1.3e-7;
constexpr double kCostL2FFTPt = 1.2e-11;
constexpr double kCostL2ScaleTable = 1.3e-12;
constexpr double kCostL2ScaleTaylor = 3.0e-13;

// The Taylor form of the z kernel (App. C, Lemma lemma::Taylor): Q terms of
// e^{-x} = sum_{p<Q} (-x)^p/p!, x = dz^2/s^2 <= (L_z/s_{m+1})^2 = xi, leave at most
// xi^Q/Q! of each Gaussian (the lemma's bound with the variable z - z' on [-L_z, L_z]).
int taylor_terms(double xi, double eps) {
    double t = 1.0;  // xi^Q / Q!
    for (int Q = 1; Q <= 16; ++Q) {
        t *= xi / Q;
        if (t <= eps) return Q;
    }
    return 0;
}

LongChoice plan_long(const double L[3], int64_t n, double sl, int nl, double eps, int prec, const sog_options& opt) {
    const sog_params& ov = opt.params;
    LongChoice best;
    const double pf = prec == SOG_PREC_FP64 ? 2.0 : 1.0;
    double eta = sl / L[2];
    int P = ov.long_P;
    if (P <= 0) {
        // Thm thm::Che with the constants its proof drops (2 x 1.0865), doubled for
        // interpolation in both the source and the target z
        for (P = 2; P <= 64; ++P) {
            double lg = 0.5 * std::lgamma(P + 1.0) + P * std::log(2.0 * std::sqrt(2.0) * eta);
            if (std::log(4.0 * 1.0865) - lg <= std::log(eps)) break;
        }
        if (P > 64) {
            best.why = "long range: more than 64 Chebyshev terms in z";
            return best;
        }
    }
    // direct form (App. B): |k| <= 2 sqrt(log(1/eps)) / s_{m+1} (Thm thm::Fcheb)
    LongChoice d;
    d.form = SOG_LONG_DIRECT;
    d.P = P;
    double K = 2.0 * std::sqrt(std::log(1.0 / eps)) / sl;
    for (int a = 0; a < 2; ++a) d.nk[a] = (int)std::floor(K * L[a] / (2.0 * kPi));
    if (ov.long_nk[0] > 0 || ov.long_nk[1] > 0) { d.nk[0] = ov.long_nk[0]; d.nk[1] = ov.long_nk[1]; }
    double nh = (d.nk[0] + 1.0) + d.nk[1] * (2.0 * d.nk[0] + 1.0);
    d.cost = kCostLongDirect * (double)n * nh * P;
    d.ok = nh * P <= 65536.0;
    if (!d.ok)
        d.why = "long range, direct form: " + std::to_string((long long)nh) + " modes x " + std::to_string(P) +
                " Chebyshev terms exceed the kernel's 65536";
    else if (long_moments_lds(prec == SOG_PREC_FP64 ? 8 : 4, P, d.nk[0], d.nk[1], kMomMinChunk, 0) > kMomMaxLds) {
        d.ok = false;
        d.why = "long range, direct form: " + std::to_string(2 * d.nk[0] + 1) + " + " + std::to_string(d.nk[1] + 1) +
                " plane-wave rows exceed the moments kernel's LDS";
    }
    // FFT form (Alg. al::long): 2D Gaussian window on an I^long grid, the mid range's error
    // rules; the z kernel exact (a table per mode) or in App. C's Taylor form (none)
    LongChoice f;
    f.form = SOG_LONG_FFT;
    f.why = "long range, FFT form: no Gaussian window of at most 15 points meets the tolerance on grids with lines "
            "the FFT kernels take";
    const double hmax = kPi * sl / (2.0 * std::sqrt(std::log(0.1 / eps)));
    const int Qt = taylor_terms((L[2] / sl) * (L[2] / sl), eps);
    const double fr[] = {1.0, 0.92, 0.85, 0.78, 0.7, 0.62, 0.55, 0.48, 0.42, 0.36};
    for (double fc : fr) {
        int I2[2];
        for (int a = 0; a < 2; ++a) I2[a] = next_smooth((int)std::ceil(L[a] / (fc * hmax) - 1e-9), true);
        if (ov.long_I[0] > 0) { I2[0] = ov.long_I[0]; I2[1] = ov.long_I[1]; }
        double hw = std::max(L[0] / I2[0], L[1] / I2[1]);
        int Pw2 = 0;
        double S2 = 0;
        if (ov.long_Pw[0] > 0) {
            Pw2 = ov.long_Pw[0];
            window_exponent(Pw2, hw, sl, &S2);
        } else {
            for (int pw = 5; pw <= kMaxPw; pw += 2) {
                double Sp;
                if (std::exp(-window_exponent(pw, hw, sl, &Sp)) <= eps) { Pw2 = pw; S2 = Sp; break; }
            }
        }
        if (ov.long_S > 0) S2 = ov.long_S;
        if (Pw2 > 0) {
            for (int a = 0; a < 2; ++a)
                if (I2[a] < 2 * Pw2) I2[a] = next_smooth(2 * Pw2, true);
            if (I2[0] <= fft_max_line(prec) && I2[1] / 2 <= fft_max_line(prec)) {
                const double npts = (double)I2[0] * I2[1];
                const double modes = (double)I2[0] * (I2[1] / 2 + 1);
                // the two z kernels: exact (Q = 0, P_s = P) or Taylor (P_s = 2Q - 1)
                for (int taylor = 0; taylor < 2; ++taylor) {
                    if (taylor && (ov.long_Q < 0 || (Qt == 0 && ov.long_Q == 0))) continue;
                    if (!taylor && ov.long_Q > 0) continue;
                    LongChoice c;
                    c.form = SOG_LONG_FFT;
                    c.P = P;
                    c.Q = taylor ? (ov.long_Q > 0 ? ov.long_Q : Qt) : 0;
                    c.Ps = taylor ? 2 * c.Q - 1 : P;
                    if (taylor && ov.long_P <= 0) c.P = std::min(P, c.Ps);  // exact in z beyond 2Q - 1 terms
                    if (c.Ps > kLong2MaxPlanes || c.P > kLong2MaxPlanes || c.Q > 16) continue;
                    c.I2[0] = I2[0];
                    c.I2[1] = I2[1];
                    c.Pw2 = Pw2;
                    c.S2 = S2;
                    const double ch_s = std::ceil(c.Ps / 8.0), ch_t = std::ceil(c.P / 8.0);
                    const double ntx = std::ceil(I2[0] / (double)kLong2Tile), nty = std::ceil(I2[1] / (double)kLong2Tile);
                    const double ntl = ntx * nty;
                    const double cand = (double)n / ntl * std::min(ntx, 3.0) * std::min(nty, 3.0);
                    const double t_spread = std::max(1.0, ntl / 2048.0) * cand * ch_s * kCostL2Cand;
                    const double t_gather =
                        std::max(1.0, ntl / 1280.0) * std::ceil((double)n / ntl / 64.0) * Pw2 * Pw2 * ch_t * kCostL2GatherNode;
                    const double t_scale = taylor ? kCostL2ScaleTaylor * modes * ((double)nl * c.Q + (double)c.Q * c.P * c.Ps)
                                                  : kCostL2ScaleTable * modes * c.P * c.Ps;
                    c.cost = pf * (t_spread + t_gather + kCostL2FFTPt * npts * (c.Ps + c.P) + t_scale);
                    c.ok = true;
                    if (c.cost < f.cost || !f.ok) f = c;
                }
            } else {
                f.why = "long range, FFT form: grid lines above the FFT kernels' " + std::to_string(fft_max_line(prec)) +
                        " points";
            }
        }
        if (ov.long_I[0] > 0) break;
    }
    if (ov.long_form == SOG_LONG_DIRECT) return d;
    if (ov.long_form == SOG_LONG_FFT) return f;
    if (f.ok && (!d.ok || f.cost < d.cost)) return f;
    if (d.ok) return d;
    best.why = d.why + "; " + f.why;
    return best;
}

void sog_weights(double b, double sigma, double omega, int M, std::vector<double>& w, std::vector<double>& s) {
    // Sec. 2.2: w_l = (pi/2)^{-1/2} b^{-l} log(b) / sigma, w_0 scaled by omega, s_l = sqrt(2) b^l sigma
    w.resize(M + 1);
    s.resize(M + 1);
    for (int l = 0; l <= M; ++l) {
        w[l] = std::sqrt(2.0 / kPi) * std::log(b) / sigma * std::pow(b, -(double)l);
        s[l] = std::sqrt(2.0) * std::pow(b, (double)l) * sigma;
    }
    w[0] *= omega;
}

}  // namespace

int next_smooth(int n, bool even) {
    if (n < 1) n = 1;
    for (int m = n;; ++m) {
        if (even && (m % 2)) continue;
        if (is_smooth(m)) return m;
    }
}

// Radix sequence of a length-n transform with the fewest stages (each stage is one pass
// over the batch in LDS); the radices are those the line kernels have butterflies for,
// composite ones (6, 8, 9, 10, 16) computed in registers.  Ties: the larger first radix.
bool factor_fft(int n, FFTFactors& f) {
    static const int kRadices[] = {16, 10, 9, 8, 7, 6, 5, 4, 3, 2};
    f.n = n;
    f.nstages = 0;
    if (n < 1) return false;
    std::vector<int> best(n + 1, 1 << 20), pick(n + 1, 0);
    best[1] = 0;
    for (int m = 2; m <= n; ++m) {
        if (n % m) continue;  // only divisors of n are reached
        for (int R : kRadices)
            if (m % R == 0 && best[m / R] + 1 < best[m]) {
                best[m] = best[m / R] + 1;
                pick[m] = R;
            }
    }
    if (best[n] >= (1 << 20) || best[n] > kMaxStages) return false;
    for (int m = n; m > 1; m /= pick[m]) f.radix[f.nstages++] = pick[m];
    return true;
}

// C[c][n] = (2 - delta_{n0}) / P * T_n(t_c): L_c(t) = sum_n C[c][n] T_n(t) (App. A.2, V^{-1}).
void cheb_V_inverse(int P, double* C) {
    std::vector<double> T(P);
    for (int c = 0; c < P; ++c) {
        double tc = std::cos((c + 0.5) * kPi / P);
        T[0] = 1.0;
        if (P > 1) T[1] = tc;
        for (int k = 2; k < P; ++k) T[k] = 2.0 * tc * T[k - 1] - T[k - 2];
        for (int k = 0; k < P; ++k) C[c * P + k] = (k == 0 ? 1.0 : 2.0) / P * T[k];
    }
}

// Long-range kernel K(k; c, c') = pi sum_{l>m} w_l s_l^2 e^{-s_l^2 k^2/4} e^{-(z_c - z_c')^2/s_l^2}
// (from eq. trun2; the k = 0 constant, which multiplies sum_j q_j = 0, is dropped via
// expm1), moved to the Chebyshev coefficient basis: Kt = C^T K C.  out: nk x P x P.
void long_kernel_cheb_basis(const Resolved& r, const double* k2, int nk, double* out) {
    const int P = r.P;
    std::vector<double> C(P * P), K(P * P), T(P * P), zc(P);
    cheb_V_inverse(P, C.data());
    for (int c = 0; c < P; ++c) zc[c] = 0.5 * r.L[2] * std::cos((c + 0.5) * kPi / P);
    for (int ik = 0; ik < nk; ++ik) {
        std::fill(K.begin(), K.end(), 0.0);
        for (int l = r.m + 1; l <= r.M; ++l) {
            double s2 = r.s[l] * r.s[l];
            double coef = kPi * r.w[l] * s2;
            if (k2[ik] == 0.0) {
                for (int c = 0; c < P; ++c)
                    for (int e = 0; e < P; ++e) {
                        double dz = zc[c] - zc[e];
                        K[c * P + e] += coef * std::expm1(-dz * dz / s2);
                    }
            } else {
                double ek = std::exp(-s2 * k2[ik] / 4.0);
                if (ek == 0.0) continue;
                for (int c = 0; c < P; ++c)
                    for (int e = 0; e < P; ++e) {
                        double dz = zc[c] - zc[e];
                        K[c * P + e] += coef * ek * std::exp(-dz * dz / s2);
                    }
            }
        }
        // T = K C, out = C^T T
        for (int c = 0; c < P; ++c)
            for (int nn = 0; nn < P; ++nn) {
                double acc = 0;
                for (int e = 0; e < P; ++e) acc += K[c * P + e] * C[e * P + nn];
                T[c * P + nn] = acc;
            }
        double* o = out + (size_t)ik * P * P;
        for (int a = 0; a < P; ++a)
            for (int nn = 0; nn < P; ++nn) {
                double acc = 0;
                for (int c = 0; c < P; ++c) acc += C[c * P + a] * T[c * P + nn];
                o[a * P + nn] = acc;
            }
    }
}

// Chebyshev series of F(r) and F'(r)/r in x = 2 r^2 / r_c^2 - 1 on r in [0, r_c]
// (the near-field kernel N(r) = 1/r - F(r) of eq. SOGDEcomp, made independent of M as
// Remark rmk::sum asks; polynomial in r^2 is this library's choice).
void near_chebyshev(Resolved& r) {
    const int Np = kMaxNearDeg + 1;
    std::vector<double> fF(Np), fG(Np), xs(Np);
    for (int j = 0; j < Np; ++j) {
        double x = std::cos(kPi * (j + 0.5) / Np);
        xs[j] = x;
        double rr2 = 0.5 * (x + 1.0) * r.rc * r.rc;
        double F = 0, G = 0;
        for (int l = 0; l <= r.M; ++l) {
            double e = std::exp(-rr2 / (r.s[l] * r.s[l]));
            F += r.w[l] * e;
            G += -2.0 * r.w[l] / (r.s[l] * r.s[l]) * e;
        }
        fF[j] = F;
        fG[j] = G;
    }
    double cmaxF = 0, cmaxG = 0;
    for (int k = 0; k < Np; ++k) {
        double aF = 0, aG = 0;
        for (int j = 0; j < Np; ++j) {
            double Tk = std::cos(k * kPi * (j + 0.5) / Np);
            aF += fF[j] * Tk;
            aG += fG[j] * Tk;
        }
        aF *= 2.0 / Np;
        aG *= 2.0 / Np;
        if (k == 0) { aF *= 0.5; aG *= 0.5; }
        r.near_cF[k] = aF;
        r.near_cG[k] = aG;
        cmaxF = std::max(cmaxF, std::fabs(aF));
        cmaxG = std::max(cmaxG, std::fabs(aG));
    }
    // coefficients below thr x the largest are dropped: far below float32 rounding of the
    // pair terms in the float32 form, near float64 rounding in the float64 form
    double thr = (r.prec == SOG_PREC_FP64) ? 1e-14 : 1e-7;
    int deg = kMaxNearDeg;
    while (deg > 1 && std::fabs(r.near_cF[deg]) < thr * cmaxF && std::fabs(r.near_cG[deg]) < thr * cmaxG) --deg;
    r.near_deg = deg;
    for (int k = deg + 1; k <= kMaxNearDeg; ++k) r.near_cF[k] = r.near_cG[k] = 0.0;
    // monomial coefficients: T_{k+1} = 2 x T_k - T_{k-1} on coefficient vectors (float64;
    // the float32 fits stay below degree 24, where the coefficients of T_k are below 2^23)
    for (int k = 0; k <= kMaxNearDeg; ++k) r.near_mF[k] = r.near_mG[k] = 0.0;
    if (deg <= 24) {
        std::vector<double> t0(deg + 2, 0.0), t1(deg + 2, 0.0), t2(deg + 2, 0.0);
        t0[0] = 1.0;
        t1[1] = 1.0;
        for (int k = 0; k <= deg; ++k) {
            const std::vector<double>& tk = (k == 0) ? t0 : t1;
            for (int j = 0; j <= k; ++j) {
                r.near_mF[j] += r.near_cF[k] * tk[j];
                r.near_mG[j] += r.near_cG[k] * tk[j];
            }
            if (k >= 1) {
                for (int j = 0; j <= deg + 1; ++j) t2[j] = (j > 0 ? 2.0 * t1[j - 1] : 0.0) - t0[j];
                t0 = t1;
                t1 = t2;
            }
        }
    }
}

namespace {

// Near-field work per particle and unit density: the ball of radius rc, or, in a slab
// thinner than 2 rc (where the near field becomes two-dimensional), the ball scaled by the
// mean z extent of the candidate ranges [z - rc, z + rc] cut to [0, L_z] over 2 rc (the
// pair kernel tests every candidate of the 3 x 3 cell columns within that z range).
// Thicker boxes keep the ball, to which the kernel cost constants were fitted.
double neighbour_volume(double rc, double Lz) {
    const double ball = (4.0 * kPi / 3.0) * rc * rc * rc;
    if (Lz >= 2.0 * rc) return ball;
    const int nz = 64;
    double acc = 0;
    for (int i = 0; i < nz; ++i) {
        const double z0 = (i + 0.5) * Lz / nz;
        acc += std::min(Lz, z0 + rc) - std::max(0.0, z0 - rc);
    }
    return ball * (acc / nz) / (2.0 * rc);
}

}  // namespace

sog_status resolve(const double box[3], int64_t n, double tol, const sog_options& opt, Resolved& r,
                   std::string& err, std::vector<PlanCandidate>* cands) {
    const sog_params& ov = opt.params;
    for (int d = 0; d < 3; ++d) {
        if (!(box[d] > 0) || !std::isfinite(box[d])) { err = "box lengths must be finite and > 0"; return SOG_ERR_INVALID_ARG; }
        r.L[d] = box[d];
    }
    if (n <= 1 || n > (int64_t)1 << 26) { err = "n must be in [2, 2^26]"; return SOG_ERR_INVALID_ARG; }
    r.n = n;
    r.prec = opt.precision;
    r.deterministic = opt.deterministic != 0;
    r.eta = opt.params.set_m ? 0.0 : opt.params.eta;
    if (r.prec != SOG_PREC_FP64 && r.prec != SOG_PREC_FP32_BULK) { err = "unknown precision"; return SOG_ERR_INVALID_ARG; }
    double tmin = (r.prec == SOG_PREC_FP64) ? 1e-12 : 1e-5;
    if (!(tol >= tmin && tol <= 1e-2)) { err = "tol outside the reachable range for this precision"; return SOG_ERR_TOL_UNREACHABLE; }
    r.tol = tol;
    if (ov.mid_Pw[0] != ov.mid_Pw[1] || ov.mid_Pw[0] != ov.mid_Pw[2]) { err = "mid_Pw must be equal in x, y, z"; return SOG_ERR_INVALID_ARG; }
    if (ov.mid_window < SOG_WINDOW_AUTO || ov.mid_window > SOG_WINDOW_KB) { err = "mid_window must be 0, 1, 2 or 3"; return SOG_ERR_INVALID_ARG; }
    if (ov.mid_beta < 0 || !std::isfinite(ov.mid_beta)) { err = "mid_beta must be finite and >= 0"; return SOG_ERR_INVALID_ARG; }
    if ((ov.mid_window == SOG_WINDOW_ES || ov.mid_window == SOG_WINDOW_KB) && ov.mid_S > 0) { err = "mid_S is the Gaussian window's shape; use mid_beta with the ES and KB windows"; return SOG_ERR_INVALID_ARG; }
    if (ov.mid_nu != 0 && (ov.mid_window != SOG_WINDOW_KB || ov.mid_nu < 2 || ov.mid_nu > kMaxWinPoly)) { err = "mid_nu is the KB window's polynomial degree, in [2, 16]"; return SOG_ERR_INVALID_ARG; }
    if (ov.mid_Pw[0] < 0 || (ov.mid_Pw[0] > 0 && (ov.mid_Pw[0] % 2 == 0 || ov.mid_Pw[0] < 3 || ov.mid_Pw[0] > kMaxPw))) { err = "mid_Pw must be odd in [3, 15]"; return SOG_ERR_INVALID_ARG; }
    if (ov.long_Pw[0] != ov.long_Pw[1] || (ov.long_Pw[0] > 0 && (ov.long_Pw[0] % 2 == 0 || ov.long_Pw[0] < 3 || ov.long_Pw[0] > kMaxPw))) { err = "long_Pw must be odd in [3, 15] and equal in x, y"; return SOG_ERR_INVALID_ARG; }
    if (ov.long_P < 0 || ov.long_P > 64) { err = "long_P must be in [1, 64]"; return SOG_ERR_INVALID_ARG; }
    if (ov.long_Q < -1 || ov.long_Q > 16) { err = "long_Q must be -1 (exact z kernel), 0 (chosen) or in [1, 16]"; return SOG_ERR_INVALID_ARG; }
    if (ov.mid_Izs % 2) { err = "mid_Izs must be even"; return SOG_ERR_INVALID_ARG; }
    if (!(ov.eta >= 0) || !std::isfinite(ov.eta)) { err = "eta must be finite and >= 0"; return SOG_ERR_INVALID_ARG; }
    if (opt.deterministic != 0 && opt.deterministic != 1) { err = "deterministic must be 0 or 1"; return SOG_ERR_INVALID_ARG; }

    // decomposition parameters
    bool custom = ov.b > 0 || ov.r0 > 0 || ov.omega > 0;
    int ME = 0;
    if (custom) {
        if (!(ov.b > 1 && ov.r0 > std::sqrt(2.0) && ov.omega > 0)) { err = "b, r0, omega must be given together (b > 1, r0 > sqrt 2)"; return SOG_ERR_INVALID_ARG; }
        r.b = ov.b; r.r0 = ov.r0; r.omega = ov.omega;
    } else {
        const Row* row = &kTable1[5];
        for (const Row& t : kTable1)
            if (t.eE <= 0.5 * tol && t.eF <= 0.5 * tol) { row = &t; break; }
        r.b = row->b; r.r0 = row->r0; r.omega = row->omega; ME = row->ME;
    }
    const double V = r.L[0] * r.L[1] * r.L[2];
    const double A = r.L[0] * r.L[1];
    const double rho = (double)n / V;
    const double rc_max = 0.5 * std::min(r.L[0], r.L[1]);
    std::vector<double> rcs;
    if (ov.rc > 0) {
        if (ov.rc > rc_max * (1 + 1e-12)) { err = "rc must be <= min(Lx, Ly)/2 (Assumption ass:SOG)"; return SOG_ERR_INVALID_ARG; }
        rcs.push_back(ov.rc);
    } else {
        for (double c : {2.0, 2.5, 2.75, 3.0, 3.25, 3.5, 4.0, 5.0}) rcs.push_back(std::min(c * std::cbrt(1.0 / rho), rc_max));
        // flat boxes: cutoffs on the scale of the area per particle too (the near field is
        // two-dimensional once r_c exceeds L_z)
        if (r.L[2] < 0.25 * std::min(r.L[0], r.L[1]))
            for (double c : {2.0, 3.0, 4.0, 5.0, 6.0, 8.0}) rcs.push_back(std::min(c * std::sqrt(A / (double)n), rc_max));
    }
    const double eps = tol / 20.0;
    std::string why;  // the last limit that ruled a candidate out
    double best_cost = 1e300;
    Resolved best = r;
    bool found = false;
    for (double rc : rcs) {
        Resolved c = r;
        c.rc = rc;
        c.sigma = rc / c.r0;
        // M: the omitted wide Gaussians leave -(pi/A) sum_{l>M} w_l sum_j q_j z_ij^2 in Phi;
        // bound sum_j |q_j| z_ij^2 by n Lz^2 and keep it below 1e-2 eps
        double wl1 = std::sqrt(2.0 / kPi) * std::log(c.b) / c.sigma;
        double rhs = 1e-2 * eps * A / (kPi * (double)n * r.L[2] * r.L[2]) * (1.0 - 1.0 / c.b) / wl1;
        int M = (int)std::ceil(-std::log(rhs) / std::log(c.b));
        M = std::max(M, ME);
        if (ov.M > 0) M = ov.M;
        M = std::min(M, 4000);
        c.M = M;
        sog_weights(c.b, c.sigma, c.omega, M, c.w, c.s);
        double near_cost = kCostNearPair * (double)n * rho *
                           neighbour_volume(rc, r.L[2]);
        // candidate splits: m = -1 (all long) .. last l with s_l <= 2 Lz
        int mlo = -1, mhi = -1;
        for (int l = 0; l <= M; ++l)
            if (c.s[l] <= 2.0 * r.L[2]) mhi = l;
        mhi = std::min(mhi, std::min(M - 1, kMaxMid - 1));
        if (ov.set_m) { mlo = mhi = ov.m; }
        if (ov.eta > 0 && !ov.set_m) {
            // the range-splitting definition (Sec. 3.1): mid range are the Gaussians with
            // s_l <= eta L_z
            int me = -1;
            for (int l = 0; l <= M; ++l)
                if (c.s[l] <= ov.eta * r.L[2]) me = l;
            if (me >= kMaxMid || me >= M) {
                why = "eta puts more Gaussians in the mid range than the kernels take";
                continue;
            }
            mlo = mhi = me;
        }
        if (ov.set_m && (ov.m < -1 || ov.m > M || ov.m >= kMaxMid)) { err = "m out of range"; return SOG_ERR_INVALID_ARG; }
        for (int m = mlo; m <= mhi; ++m) {
            double cost = near_cost;
            MidChoice mc;
            LongChoice lc;
            if (m >= 0) {
                mc = plan_mid(r.L, n, c.s[0], c.s[m], m + 1, eps, r.prec, ov);
                if (!mc.ok) {
                    why = "mid range: no window of at most 15 points meets the tolerance on grids the kernels take";
                    continue;
                }
                cost += mc.cost;
            }
            if (m < M) {
                lc = plan_long(r.L, n, c.s[m + 1], M - m, eps, r.prec, opt);
                if (!lc.ok) {
                    why = lc.why;
                    continue;
                }
                cost += lc.cost;
            }
            if (cands) cands->push_back(PlanCandidate{cost, rc, m});
            if (cost < best_cost) {
                best_cost = cost;
                best = c;
                best.m = m;
                best.has_mid = m >= 0;
                best.has_long = m < M;
                if (best.has_mid) {
                    for (int d = 0; d < 3; ++d) best.I[d] = mc.I[d];
                    best.Izs = mc.Izs;
                    best.Pw = mc.Pw;
                    best.S = mc.S;
                    best.window = mc.window;
                    best.beta = mc.beta;
                    best.nu = mc.nu;
                }
                if (best.has_long) {
                    best.form = lc.form;
                    best.P = lc.P;
                    best.nk[0] = lc.nk[0]; best.nk[1] = lc.nk[1];
                    best.I2[0] = lc.I2[0]; best.I2[1] = lc.I2[1];
                    best.Pw2 = lc.Pw2;
                    best.S2 = lc.S2;
                    best.Q = lc.Q;
                    best.Ps = lc.Ps;
                }
                found = true;
            }
        }
    }
    if (!found) {
        err = "no feasible discretisation for this box and tolerance" + (why.empty() ? std::string() : ": " + why);
        return SOG_ERR_TOL_UNREACHABLE;
    }
    r = best;
    if (r.has_mid && r.window == SOG_WINDOW_KB && r.nu == 0) r.nu = window_poly_degree(r.Pw, r.beta, eps);
    r.self_coeff = 0;
    for (double v : r.w) r.self_coeff += v;

    // near-field cells
    for (int d = 0; d < 3; ++d) {
        r.nc[d] = std::max(1, (int)std::floor(r.L[d] / r.rc));
        r.ch[d] = r.L[d] / r.nc[d];
    }
    if ((int64_t)r.nc[0] * r.nc[1] * r.nc[2] > (int64_t)1 << 26) { err = "too many near-field cells"; return SOG_ERR_INVALID_ARG; }
    near_chebyshev(r);

    if (r.has_mid) {
        if (r.I[0] < r.Pw || r.I[1] < r.Pw) { err = "mid grid smaller than the window"; return SOG_ERR_INVALID_ARG; }
        if (r.Izs < r.I[2] + r.Pw + 2) { err = "mid_Izs too small for the window support"; return SOG_ERR_INVALID_ARG; }
        for (int d = 0; d < 3; ++d) r.h[d] = r.L[d] / r.I[d];
        r.Lzs = r.Izs * r.h[2];
        for (int d = 0; d < 3; ++d) r.H[d] = 0.5 * (r.Pw - 1) * r.h[d];
        {
            // nearest nodes of z in [0, L_z] lie in [(I_z* - I_z)/2, (I_z* + I_z)/2]; one node
            // of slack on each side, then the window half-width
            const int HWz = (r.Pw - 1) / 2;
            const int lo = (r.Izs - r.I[2]) / 2 - 1 - HWz;
            const int hi = (r.Izs + r.I[2] + 1) / 2 + 2 + HWz;
            r.zband[0] = std::max(0, lo) & ~1;
            r.zband[1] = std::min(r.Izs, (hi + 1) & ~1);
        }
        // tiles: LDS holds the tile plus its (P_w - 1) halo for gridding and gathering;
        // gridding adds each tile's block into the grid with atomics, so any tile count works
        int Bt[3];
        spread_tile(r.prec, r.Pw, Bt);
        const int gI[3] = {r.I[0], r.I[1], r.Izs};
        for (int d = 0; d < 3; ++d) {
            r.B[d] = std::min(Bt[d], gI[d]);
            r.ntile[d] = (gI[d] + r.B[d] - 1) / r.B[d];
        }
        if (r.deterministic && !deterministic_tiles(r.Pw, gI, r.B, r.ntile, r.dcol_m, r.dcol_q, r.dcol_n)) {
            err = "deterministic gridding: the mid grid is too small for the window";
            return SOG_ERR_INVALID_ARG;
        }
        r.spread_dummy = spread_lane_nodes(r.Pw, r.B[2] + r.Pw - 1, r.B[2], r.node_oy, r.node_oz);
        if (!is_smooth(r.I[0]) || !is_smooth(r.I[1]) || !is_smooth(r.Izs / 2)) { err = "mid grid sizes must have only factors 2, 3, 5, 7 (and I_z*/2 as well)"; return SOG_ERR_INVALID_ARG; }
        if (r.I[0] % 2 || r.I[1] % 2) { err = "mid I_x, I_y must be even"; return SOG_ERR_INVALID_ARG; }
        if (r.I[0] > 4096 || r.I[1] > 4096 || r.Izs > 8192) { err = "mid grid too large"; return SOG_ERR_INVALID_ARG; }
        if (std::max(std::max(r.I[0], r.I[1]), r.Izs / 2) > fft_max_line(r.prec)) {
            err = "mid grid line too long for the FFT kernels in this precision";
            return SOG_ERR_INVALID_ARG;
        }
    }
    if (r.has_long) {
        if (r.P < 1 || r.P > 64) { err = "long P out of range"; return SOG_ERR_INVALID_ARG; }
        if (r.form == SOG_LONG_DIRECT) {
            r.nh = (r.nk[0] + 1) + r.nk[1] * (2 * r.nk[0] + 1);
            if ((int64_t)r.nh * r.P > 65536) { err = "too many long-range modes for the direct form"; return SOG_ERR_INVALID_ARG; }
            if (long_moments_lds(r.prec == SOG_PREC_FP64 ? 8 : 4, r.P, r.nk[0], r.nk[1], kMomMinChunk, 0) > kMomMaxLds) {
                err = "too many long-range modes in x and y for the direct form's moments kernel";
                return SOG_ERR_INVALID_ARG;
            }
            r.Q = r.Ps = 0;
        } else {
            if (r.Pw2 < 3 || r.Pw2 > kMaxPw || (r.Pw2 % 2) == 0) { err = "long-range window must have an odd number of points in [3, 15]"; return SOG_ERR_INVALID_ARG; }
            if (r.I2[0] < 2 * r.Pw2 || r.I2[1] < 2 * r.Pw2) { err = "long-range FFT grid smaller than twice its window"; return SOG_ERR_INVALID_ARG; }
            if (!is_smooth(r.I2[0]) || !is_smooth(r.I2[1] / 2) || (r.I2[1] & 1)) { err = "long-range grid sizes must be even with only factors 2, 3, 5, 7 (I^long_y / 2 as well)"; return SOG_ERR_INVALID_ARG; }
            if (r.I2[0] > fft_max_line(r.prec) || r.I2[1] / 2 > fft_max_line(r.prec)) { err = "long-range grid line too long for the FFT kernels in this precision"; return SOG_ERR_INVALID_ARG; }
            if (r.Ps < 1 || r.Ps > kLong2MaxPlanes || r.P > kLong2MaxPlanes || r.Q < 0 || r.Q > 16) { err = "long-range FFT form: at most 32 Chebyshev terms (long_P) and 16 Taylor terms (long_Q)"; return SOG_ERR_INVALID_ARG; }
            for (int a = 0; a < 2; ++a) {
                r.h2[a] = r.L[a] / r.I2[a];
                r.H2[a] = 0.5 * (r.Pw2 - 1) * r.h2[a];
                r.ntile2[a] = (r.I2[a] + kLong2Tile - 1) / kLong2Tile;
            }
        }
    }
    return SOG_OK;
}

}  // namespace sog
