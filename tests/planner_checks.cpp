// Host-side invariants of the planner's tables that the GPU kernels rely on for memory
// safety and correctness (compiled with the host compiler by test_planner_invariants.py;
// no GPU needed):
//
//  1. gridding lane nodes: every window node (y, z) is taken by exactly one lane of one
//     pass; a dummy node has z >= P_w, an offset no window node has, stays in the corner's
//     x plane for every corner in the tile, and is used by no other lane;
//     both kernels' LDS within the tile budget;
//  2. the gridding kernel's LDS addressing (a model of k_spread's index arithmetic): for
//     every corner in the tile, wave, plane and pass, the address lies in the padded halo
//     block, in an x plane the wave owns (x = wave mod 4), and the addresses of one
//     particle are distinct;
//  3. FFT factorisation: every length up to the longest line the kernels take factors
//     exactly when it has no prime factor above 7, into compiled radices;
//  4. the z band: for z in [0, L_z] the nearest node is never clamped, so every window
//     lies inside the band of planes the z transforms read and write;
//  5. the near-field chunks of the float32 pair kernel fit their slots (below);
//  6. the float32 near-field polynomials in monomial form (below);
//  7. the ES window transform (Gauss-Legendre) against a fine composite Simpson sum in x
//     itself (no change of variable), and the Gauss-Legendre rule against exact moments;
//  8. the KB window's transform and its polynomial form (below);
//  9. the deterministic gridding's tiling (below).
//
// Prints one line per failure and "bad N"; exit status 0 when N == 0.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <set>
#include <vector>

#include "../paper_2412_04595_amd/csrc/planner.cpp"

using namespace sog;

static long bad = 0;
#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            ++bad;                            \
            if (bad < 20) {                   \
                std::printf(__VA_ARGS__);     \
                std::printf("\n");            \
            }                                 \
        }                                     \
    } while (0)

static void check_lane_nodes_and_addresses() {
    for (int prec : {SOG_PREC_FP32_BULK, SOG_PREC_FP64})
        for (int Pw = 3; Pw <= 15; Pw += 2) {
            int B[3];
            spread_tile(prec, Pw, B);
            CHECK(spread_lds_bytes(prec == SOG_PREC_FP64 ? 8 : 4, Pw, B[0], B[1], B[2]) <= tile_lds_budget(Pw, prec == SOG_PREC_FP64 ? 8 : 4),
                  "tile LDS over budget Pw %d", Pw);
            // the gathering kernel: the halo block plus its residue-sort scratch (128 + 256 ints)
            CHECK((size_t)(B[0] + Pw - 1) * (B[1] + Pw - 1) * (B[2] + Pw - 1) * (prec == SOG_PREC_FP64 ? 8 : 4) +
                          (128 + 256) * 4 <= tile_lds_budget(Pw, prec == SOG_PREC_FP64 ? 8 : 4),
                  "gather LDS over budget Pw %d", Pw);
            for (int bz : {B[2], 2, 3, 5, 8}) {
                if (bz > B[2]) continue;  // tiles are clipped to small grids, never grown
                const int HX = B[0] + Pw - 1, HY = B[1] + Pw - 1, HZ = bz + Pw - 1, HYZ = HY * HZ;
                const int NPL = (Pw + 3) / 4, NPAD = 4 * NPL - Pw, NPASS = (Pw * Pw + 63) / 64;
                signed char noy[256], noz[256];
                const bool dummy = spread_lane_nodes(Pw, HZ, bz, noy, noz);
                // 1. the node table
                std::set<int> window, seen;
                for (int oy = 0; oy < Pw; ++oy)
                    for (int oz = 0; oz < Pw; ++oz) window.insert(oy * HZ + oz);
                int nreal = 0, none = 0;
                for (int k = 0; k < NPASS * 64; ++k) {
                    if (noy[k] < 0) {
                        ++none;
                        continue;
                    }
                    const int d = noy[k] * HZ + noz[k];
                    CHECK(!seen.count(d), "Pw %d bz %d: offset %d used twice", Pw, bz, d);
                    seen.insert(d);
                    CHECK(noz[k] < HZ, "Pw %d bz %d: node z beyond the pitch", Pw, bz);
                    if (noz[k] < Pw) {
                        ++nreal;
                        CHECK(window.count(d), "Pw %d bz %d: real node outside the window", Pw, bz);
                    } else {
                        CHECK(!window.count(d), "Pw %d bz %d: dummy on a window node", Pw, bz);
                        CHECK(d <= Pw * HZ - bz, "Pw %d bz %d: dummy leaves the plane", Pw, bz);
                    }
                }
                CHECK(nreal == Pw * Pw, "Pw %d bz %d: %d of %d window nodes", Pw, bz, nreal, Pw * Pw);
                CHECK(!dummy || none == 0, "Pw %d bz %d: dummy table with empty lanes", Pw, bz);
                // 2. the addresses of k_spread for every corner of the tile
                const int totp = (HX + NPAD) * HYZ;
                std::vector<int> mark(totp, -1);
                int stamp = 0;
                for (int lx = 0; lx < B[0]; ++lx)
                    for (int ly = 0; ly < B[1]; ++ly)
                        for (int lz = 0; lz < bz; ++lz) {
                            ++stamp;
                            const int corner = lx * HYZ + ly * HZ + lz;
                            for (int g = 0; g < 4; ++g) {
                                const int first = corner + ((g - lx) & 3) * HYZ;
                                for (int pl = 0; pl < NPL; ++pl)
                                    for (int k = 0; k < NPASS * 64; ++k) {
                                        if (noy[k] < 0) continue;  // the lane's private sink
                                        const int at = first + pl * 4 * HYZ + noy[k] * HZ + noz[k];
                                        if (at < 0 || at >= totp) {
                                            CHECK(false, "Pw %d bz %d: address %d outside [0, %d)", Pw, bz, at, totp);
                                            continue;
                                        }
                                        CHECK((at / HYZ) % 4 == g, "Pw %d bz %d: plane not owned by wave %d", Pw, bz, g);
                                        CHECK(mark[at] != stamp, "Pw %d bz %d: address reused in one particle", Pw, bz);
                                        mark[at] = stamp;
                                    }
                            }
                        }
            }
        }
}

static void check_fft_factors() {
    const int compiled[] = {2, 3, 4, 5, 6, 7, 8, 9, 10, 16};
    for (int n = 1; n <= fft_max_line(SOG_PREC_FP32_BULK); ++n) {
        int m = n;
        for (int p : {2, 3, 5, 7})
            while (m % p == 0) m /= p;
        FFTFactors f;
        const bool ok = factor_fft(n, f);
        CHECK(ok == (m == 1), "factor_fft(%d) = %d", n, (int)ok);
        if (!ok) continue;
        long prod = 1;
        for (int i = 0; i < f.nstages; ++i) {
            bool known = false;
            for (int R : compiled) known |= (R == f.radix[i]);
            CHECK(known, "factor_fft(%d): radix %d has no kernel", n, f.radix[i]);
            prod *= f.radix[i];
        }
        CHECK(prod == n && f.nstages <= kMaxStages, "factor_fft(%d): product %ld", n, prod);
    }
}

static void check_z_band() {
    const double boxes[][3] = {{100, 100, 100}, {400, 400, 25}, {50, 50, 800}, {150, 150, 60},
                               {20, 20, 20},    {30, 40, 7.3},  {12, 12, 95}};
    const int64_t ns[] = {1000000, 1000000, 1000000, 200000, 1000, 5000, 3000};
    for (int prec : {SOG_PREC_FP32_BULK, SOG_PREC_FP64})
        for (int b = 0; b < 7; ++b) {
            sog_options opt;
            std::memset(&opt, 0, sizeof(opt));
            opt.precision = prec;
            Resolved r;
            std::string err;
            if (resolve(boxes[b], ns[b], 1e-4, opt, r, err) != SOG_OK || !r.has_mid) continue;
            const int HW = (r.Pw - 1) / 2;
            CHECK(r.zband[0] >= 0 && r.zband[1] <= r.Izs && r.zband[0] % 2 == 0 && r.zband[1] % 2 == 0,
                  "box %d: band [%d, %d) of %d", b, r.zband[0], r.zband[1], r.Izs);
            for (int i = 0; i <= 20000; ++i) {
                const double z = r.L[2] * i / 20000.0;
                const double v = (z - 0.5 * r.L[2] + 0.5 * r.Lzs) / r.h[2];
                const int k = (int)std::rint(v);
                CHECK(k - HW >= r.zband[0] && k + HW < r.zband[1], "box %d: z %g window [%d, %d] leaves the band",
                      b, z, k - HW, k + HW);
            }
        }
}

// 5. near-field chunks (float32 pair kernel): for random columns (empty cells, dense
//    cells, one crowded cell, long sparse columns) the chunks tile the column's particles
//    in order, hold 1..kNearChunk targets within at most kNearUnitCells cells, name the
//    cells of their first and last targets, and fit the column's slots
//    [floor(first / kNearChunk) + c * extra, floor(end / kNearChunk) + (c + 1) * extra).
static void check_near_chunks() {
    unsigned long long st = 12345;
    auto rnd = [&]() {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        return (unsigned)(st >> 33);
    };
    for (int trial = 0; trial < 4000; ++trial) {
        const int ncz = 1 + (int)(rnd() % (trial < 2000 ? 40 : 400));
        const int mode = trial % 5;
        std::vector<int> cs(ncz + 1);
        cs[0] = (int)(rnd() % 1000);
        for (int z = 0; z < ncz; ++z) {
            int c = 0;
            if (mode == 0) c = (int)(rnd() % 43);                  // about 21 per cell
            if (mode == 1) c = (rnd() % 4 == 0) ? (int)(rnd() % 9) : 0;  // sparse
            if (mode == 2) c = (int)(rnd() % 200);                 // dense
            if (mode == 3) c = (z == ncz / 2) ? 1000 : (int)(rnd() % 3);  // one crowded cell
            if (mode == 4) c = (int)(rnd() % 2);                   // long, nearly empty
            cs[z + 1] = cs[z] + c;
        }
        const int extra = near_chunk_extra(ncz);
        const long col = rnd() % 1000;
        const long s0 = cs[0] / kNearChunk + col * extra, s1 = cs[ncz] / kNearChunk + (col + 1) * extra;
        int expect = cs[0];
        const int nu = near_chunk_walk(cs.data(), ncz, [&](int za, int p, int e, int z1) {
            CHECK(p == expect && e > p && e - p <= kNearChunk, "chunks: trial %d [%d, %d) after %d", trial, p, e, expect);
            CHECK(za >= 0 && z1 <= ncz && z1 - za <= kNearUnitCells && z1 > za, "chunks: trial %d cells [%d, %d)", trial,
                  za, z1);
            CHECK(cs[za] <= p && p < cs[za + 1], "chunks: trial %d first target not in cell %d", trial, za);
            CHECK(cs[z1 - 1] <= e - 1 && e - 1 < cs[z1], "chunks: trial %d last target not in cell %d", trial, z1 - 1);
            expect = e;
        });
        CHECK(expect == cs[ncz], "chunks: trial %d ends at %d of %d", trial, expect, cs[ncz]);
        CHECK(s0 + nu <= s1, "chunks: trial %d: %d chunks in %ld slots", trial, nu, s1 - s0);
    }
}

// 6. the float32 near-field polynomials in monomial form (evaluated by Horner in float32)
//    agree with their Chebyshev form (float64) on [-1, 1] no worse than the float32 Chebyshev
//    recurrence does, or within 2.5e-7 of the largest value, for the benchmark workloads' plans
static void check_near_monomials() {
    // the float32 fits stay within the degree the conversion takes, at every tolerance
    for (double tol : {1e-3, 1e-4, 1e-5, 1e-6, 1e-8, 1e-10}) {
        sog_options opt;
        std::memset(&opt, 0, sizeof(opt));
        opt.precision = SOG_PREC_FP32_BULK;
        Resolved r;
        std::string err;
        const double box[3] = {50, 50, 50};
        if (resolve(box, 100000, tol, opt, r, err) != SOG_OK) continue;
        CHECK(r.near_deg <= 24, "monomials: tol %g float32 degree %d above 24", tol, r.near_deg);
        std::printf("float32 near degree at tol %g: %d\n", tol, r.near_deg);
    }
    const double boxes[][3] = {{100, 100, 100}, {400, 400, 25}, {50, 50, 800}, {150, 150, 60}, {20, 20, 20}};
    const int64_t ns[] = {1000000, 1000000, 1000000, 200000, 1000};
    for (int b = 0; b < 5; ++b) {
        sog_options opt;
        std::memset(&opt, 0, sizeof(opt));
        opt.precision = SOG_PREC_FP32_BULK;
        Resolved r;
        std::string err;
        if (resolve(boxes[b], ns[b], 1e-4, opt, r, err) != SOG_OK) {
            CHECK(false, "monomials: box %d does not plan: %s", b, err.c_str());
            continue;
        }
        const int D = r.near_deg;
        for (int which = 0; which < 2; ++which) {
            const double* c = which ? r.near_cG : r.near_cF;
            const double* m = which ? r.near_mG : r.near_mF;
            double vmax = 0, ehorner = 0, erec = 0;
            for (int i = 0; i <= 4000; ++i) {
                const double x = -1.0 + 2.0 * i / 4000.0;
                double ref = 0;
                for (int k = 0; k <= D; ++k) ref += c[k] * std::cos(k * std::acos(x));
                vmax = std::max(vmax, std::fabs(ref));
                float h = (float)m[D];
                for (int k = D - 1; k >= 0; --k) h = std::fmaf(h, (float)x, (float)m[k]);
                ehorner = std::max(ehorner, std::fabs((double)h - ref));
                const float xf = (float)x, x2 = xf + xf;
                float t0 = 1.f, t1 = xf, acc = (float)c[0] + (float)c[1] * xf;
                for (int k = 2; k <= D; ++k) {
                    const float t2 = std::fmaf(x2, t1, -t0);
                    acc = std::fmaf((float)c[k], t2, acc);
                    t0 = t1;
                    t1 = t2;
                }
                erec = std::max(erec, std::fabs((double)acc - ref));
            }
            CHECK(ehorner <= std::max(erec, 2.5e-7 * vmax), "monomials: box %d %s: Horner error %.2e of %.2e (recurrence %.2e)", b,
                  which ? "G" : "F", ehorner, vmax, erec);
            if (b == 0) std::printf("near polynomial %s degree %d: float32 Horner %.2e, recurrence %.2e of max %.3g\n",
                                    which ? "G" : "F", D, ehorner / vmax, erec / vmax, vmax);
        }
    }
}

// 7. es_hat_grid: the transform of psi(d) = exp(beta (sqrt(1 - (d/a)^2) - 1)) on |d| < a.
//    Reference: composite Simpson directly in d with 2e5 panels on [0, a) (the integrand's
//    square-root edge limits it to ~1e-10 relative; below the parity gates, above rounding).
//    The rule itself: n-point Gauss-Legendre integrates x^k exactly for k < 2n.
static void check_es_transform() {
    for (int n : {1, 2, 5, 64, 97}) {
        const std::vector<double>& xw = gauss_legendre(n);
        for (int k = 0; k < 2 * n && k < 40; ++k) {
            double s = 0;
            for (int i = 0; i < n; ++i) s += xw[n + i] * std::pow(xw[i], k);
            const double exact = (k % 2) ? 0.0 : 2.0 / (k + 1);
            CHECK(std::fabs(s - exact) < 1e-14, "gauss-legendre n %d moment %d: %.17g vs %.17g", n, k, s, exact);
        }
    }
    double emax = 0;
    for (int Pw : {3, 5, 9, 15})
        for (double bf : {1.6, 2.3, 2.6})
            for (double kappa : {0.0, 0.7, 2.0, 3.14159, 6.0, 12.0}) {
                const double beta = bf * Pw, a = 0.5 * Pw;
                const int np = 200000;
                const double dd = a / np;
                double s = 0;
                for (int i = 0; i <= np; ++i) {
                    const double d = i * dd;
                    const double u = 1.0 - (d / a) * (d / a);
                    const double f = std::exp(beta * (std::sqrt(u > 0 ? u : 0.0) - 1.0)) * std::cos(kappa * d);
                    s += f * ((i == 0 || i == np) ? 1.0 : ((i & 1) ? 4.0 : 2.0));
                }
                const double ref = 2.0 * s * dd / 3.0;
                const double g = es_hat_grid(kappa, Pw, beta);
                const double e = std::fabs(g - ref) / es_hat_grid(0.0, Pw, beta);
                emax = std::max(emax, e);
                CHECK(e < 1e-9, "es transform Pw %d beta %g kappa %g: %.17g vs %.17g", Pw, beta, kappa, g, ref);
            }
    std::printf("es transform: max relative difference to the direct Simpson sum %.2e\n", emax);
}

// 8. The KB window: kb_hat_grid (closed form) against a composite Simpson sum of
//    kb_value_grid in d (the same edge limit as 7); kb_value_grid is 1 at the centre and
//    1 / I_0(beta) at the support's edge.  The polynomial window (window_poly_fit): every
//    node's polynomial reproduces the window at its nu + 1 interpolation points to
//    rounding (its defining property, checked by Horner on the monomials), the deviation
//    falls geometrically with nu, the degree window_poly_degree picks meets eps / 20, and
//    the polynomials of neighbouring nodes join: node o at u = +1/2 and node o - 1 at
//    u = -1/2 (the same particle seen from the next nearest node) are the same point of
//    the window.
static void check_kb_window() {
    for (int Pw : {3, 7, 9, 15})
        for (double bf : {1.6, 2.3, 2.6}) {
            const double beta = bf * Pw, a = 0.5 * Pw;
            const int np = 200000;
            const double dd = a / np;
            std::vector<double> fw(np + 1);
            for (int i = 0; i <= np; ++i)
                fw[i] = kb_value_grid(i * dd, Pw, beta) * ((i == 0 || i == np) ? 1.0 : ((i & 1) ? 4.0 : 2.0));
            for (double kappa : {0.0, 0.7, 2.0, 3.14159, 6.0, 12.0}) {
                double s = 0;
                for (int i = 0; i <= np; ++i) s += fw[i] * std::cos(kappa * i * dd);
                const double ref = 2.0 * s * dd / 3.0;
                const double g = kb_hat_grid(kappa, Pw, beta);
                CHECK(std::fabs(g - ref) < 1e-9 * kb_hat_grid(0.0, Pw, beta), "kb transform Pw %d beta %g kappa %g: %.17g vs %.17g",
                      Pw, beta, kappa, g, ref);
            }
        }
    CHECK(std::fabs(kb_value_grid(0.0, 9, 20.0) - 1.0) < 1e-15, "kb centre");
    CHECK(std::fabs(kb_value_grid(4.5, 9, 20.0) * std::cyl_bessel_i(0.0, 20.0) - 1.0) < 1e-14, "kb edge");
    CHECK(kb_value_grid(4.5 + 1e-9, 9, 20.0) == 0.0, "kb outside");
    const double pi = 3.14159265358979323846;
    for (int Pw : {3, 9, 15}) {
        const double beta = 2.3 * Pw;
        double prev = 1.0;
        for (int nu : {4, 6, 8, 10, 12}) {
            std::vector<double> c;
            window_poly_fit(Pw, beta, nu, c);
            const int hw = (Pw - 1) / 2;
            auto horner = [&](int o, double u) {
                double w = c[(size_t)o * (nu + 1)];
                for (int j = 1; j <= nu; ++j) w = w * u + c[(size_t)o * (nu + 1) + j];
                return w;
            };
            const double e = window_poly_error(Pw, beta, nu, c, nullptr);
            for (int o = 0; o < Pw; ++o) {
                for (int j = 0; j <= nu; ++j) {
                    const double u = 0.5 * std::cos((j + 0.5) * pi / (nu + 1));
                    const double ex = kb_value_grid((double)(o - hw) - u, Pw, beta);
                    CHECK(std::fabs(horner(o, u) - ex) < 1e-13, "poly window Pw %d nu %d node %d point %d: %.17g vs %.17g",
                          Pw, nu, o, j, horner(o, u), ex);
                }
                if (o > 0)
                    CHECK(std::fabs(horner(o, 0.5) - horner(o - 1, -0.5)) <= 2.0 * e + 1e-13,
                          "poly window Pw %d nu %d: nodes %d and %d do not join", Pw, nu, o - 1, o);
            }
            if (nu > 4) CHECK(e < 0.1 * prev || e < 1e-13, "poly window Pw %d nu %d: error %.3e after %.3e", Pw, nu, e, prev);
            prev = e;
        }
        for (double eps : {1e-4, 1e-8, 1e-12}) {
            const int nu = window_poly_degree(Pw, beta, eps);
            std::vector<double> c;
            window_poly_fit(Pw, beta, nu, c);
            const double e = window_poly_error(Pw, beta, nu, c, nullptr);
            CHECK(e <= eps / 20.0 || nu == kMaxWinPoly, "poly window degree Pw %d eps %g: nu %d error %.3e", Pw, eps, nu, e);
            std::printf("kb window Pw %d eps %g: nu %d, weights within %.2e\n", Pw, eps, nu, e);
        }
    }
}

// 9. Deterministic gridding: for grids of every size class, every window and the tile
//    edges the planner uses (and smaller), the tiling deterministic_tiles returns puts no
//    two blocks (tile plus (P_w - 1)/2 nodes each side, wrapped in x and y, clipped in z)
//    of one tile_colour on a common node, and no block on a node twice (no self-wrap);
//    the colour count matches, and the colour lists the spread launcher forms
//    (first + m j, j < q or the tail tile) are exactly the tiles of that colour.  Checked
//    per direction, which suffices: two tiles of one 3D colour have the same colour in
//    every direction, and blocks that are apart in one direction do not meet.
static void check_deterministic_tiles() {
    long tried = 0;
    for (int Pw = 3; Pw <= 15; Pw += 2)
        for (int I = 2 * Pw; I <= 700; I += (I < 80 ? 1 : 7))
            for (int B0 : {4, 6, 7, 10, 11, 14, 16, 24, 37}) {
                ++tried;
                const int gI[3] = {I, I, I + 6};
                int B[3] = {B0, B0, B0}, nt[3], m[3], q[3], nc[3];
                if (!deterministic_tiles(Pw, gI, B, nt, m, q, nc)) {
                    CHECK(false, "deterministic tiles: none for P_w %d I %d B %d", Pw, I, B0);
                    continue;
                }
                const int hw = (Pw - 1) / 2;
                for (int d = 0; d < 3; ++d) {
                    const bool periodic = d < 2;
                    const int n = gI[d];
                    CHECK(B[d] <= B0 && nt[d] == (n + B[d] - 1) / B[d], "tile count");
                    std::vector<int> owner(n);
                    int maxcol = 0;
                    for (int t = 0; t < nt[d]; ++t) maxcol = std::max(maxcol, tile_colour(t, periodic, m[d], q[d]));
                    CHECK(maxcol + 1 == nc[d], "deterministic tiles: P_w %d I %d dir %d: %d colours used, %d counted",
                          Pw, n, d, maxcol + 1, nc[d]);
                    for (int col = 0; col < nc[d]; ++col) {
                        // the launcher's list of this colour's tiles
                        std::vector<int> listed;
                        if (periodic && col >= m[d]) listed.push_back(q[d] * m[d] + (col - m[d]));
                        else {
                            const int cnt = periodic ? q[d] : (nt[d] - col + m[d] - 1) / m[d];
                            for (int j = 0; j < cnt; ++j) listed.push_back(col + m[d] * j);
                        }
                        std::vector<int> expect;
                        for (int t = 0; t < nt[d]; ++t)
                            if (tile_colour(t, periodic, m[d], q[d]) == col) expect.push_back(t);
                        CHECK(listed == expect, "deterministic tiles: P_w %d I %d dir %d colour %d: launcher lists "
                              "%zu tiles, %zu have the colour", Pw, n, d, col, listed.size(), expect.size());
                        std::fill(owner.begin(), owner.end(), -1);
                        for (int t : expect) {
                            const int lo = t * B[d] - hw, hi = std::min(n, (t + 1) * B[d]) + hw;
                            for (int g = lo; g < hi; ++g) {
                                int gg = g;
                                if (periodic) gg = ((g % n) + n) % n;
                                else if (g < 0 || g >= n) continue;
                                CHECK(owner[gg] == -1, "deterministic tiles: P_w %d I %d B %d dir %d: tiles %d and %d "
                                      "of colour %d share node %d", Pw, n, B[d], d, owner[gg], t, col, gg);
                                owner[gg] = t;
                            }
                        }
                    }
                }
            }
    std::printf("deterministic tiles: %ld grids\n", tried);
}

int main() {
    check_es_transform();
    check_deterministic_tiles();
    check_kb_window();
    check_near_monomials();
    check_near_chunks();
    check_lane_nodes_and_addresses();
    check_fft_factors();
    check_z_band();
    std::printf("bad %ld\n", bad);
    return bad == 0 ? 0 : 1;
}
