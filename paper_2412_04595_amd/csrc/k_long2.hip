// Long range, Fourier-Chebyshev solver with FFTs (Alg. al::long, Sec. 3.3), for boxes
// where the direct form's O(A / s_{m+1}^2) modes per particle are too many (flat and
// strongly confined boxes).  The x,y Fourier sums go through a 2D Gaussian-window grid
// (eq. Chebygrid) and 2D FFTs, z stays polynomial:
//   S2(g, a)  = sum_j q_j W2(g - r_j) T_a(t_j),  a < P_s               (gridding)
//   Shat2     = fft2(S2(., a))                  (real-to-complex along y, then along x)
//   uhat(k,n) = sum_a K(k)[n][a] Shat2(k, a),  n < P                  (scaling)
//   u(., n)   = ifft2(uhat(., n))               (along x, then complex-to-real along y)
//   Phi^long_i = h_x h_y sum_g W2(r_i - g) sum_n T_n(t_i) u(g, n)      (gathering)
// with t = 2 z / L_z on the centred box.  Two forms of the z kernel K (both divided by
// What2(k)^2 and by I2x I2y, the unnormalised inverse):
//   * exact: P_s = P, K = C^T Kz C with Kz(k; c, c') = pi sum_{l>m} w_l s_l^2
//     e^{-s_l^2 |k|^2/4} e^{-(z_c - z_c')^2/s_l^2} at the Chebyshev nodes (eq. trun2,
//     interpolation in the target and anterpolation in the source z); a table per mode;
//   * Taylor (App. C, Lemma lemma::Taylor): e^{-dz^2/s^2} = sum_{p<Q} (-dz^2/s^2)^p/p! + ...,
//     so Kz(k; z, z') = sum_{p<Q} A_p(k) ((z - z')/L_z)^{2p} with
//     A_p(k) = pi ((-1)^p/p!) sum_{l>m} w_l L_z^{2p} s_l^{2-2p} e^{-s_l^2 |k|^2/4}.  In the
//     source z the polynomial is exact with P_s = 2Q - 1 Chebyshev terms, in the target z it
//     is interpolated at the P Chebyshev nodes: K(k) = sum_p A_p(k) B_p with fixed matrices
//     B_p (host, float64).  A_p is formed on the fly per mode (no table), so the scaling
//     reads and writes only the grid.  This is the paper's Taylor form with its sum over the
//     nodes' moments ((z_c - z_j)/L_z)^{2p} reordered through the Chebyshev basis of z_j
//     (equal up to rounding).
// At k = 0 the constant term (p = 0, or the expm1 of the exact form) multiplies
// sum_j q_j and is left out.
//
// Batches do not run this form (its launches are not recorded; a batch whose system needs it
// is refused).
//
// Gridding is output-stationary: a workgroup owns a 16 x 16 tile of nodes, one node per
// thread, and sums in registers the windows of the particles that reach the tile: it reads
// the particles of the (at most three per direction) tiles around its own (particles
// counting-sorted by tile), keeps those whose windows reach it, and stages their weights in
// LDS 128 at a time; 8 planes per pass.  No atomics: each node is written once.  Gathering: one particle per lane,
// the tile's halo of the u planes staged in LDS 8 planes at a time.
#include "launch.hpp"

namespace sog {

hipError_t launch_fft_long2(Plan& p, int sign, int planes);  // k_fft.hip

namespace {

constexpr int kL2Tile = kLong2Tile;  // tile edge (nodes) in x and y
constexpr int kL2Chunk = 8;          // planes per pass of the gridding and gathering
constexpr int kL2Batch = 128;        // particles staged at a time by the gridding

struct L2Geom {
    double L[3];
    double h[2];
    int I[2];
    int nt[2];
};

__device__ __forceinline__ void grid_point2(const L2Geom& g, double x, double y, int a[2], double u[2]) {
    double v[2] = {wrap_periodic(x, g.L[0]) / g.h[0], wrap_periodic(y, g.L[1]) / g.h[1]};
    for (int d = 0; d < 2; ++d) {
        if (!isfinite(v[d])) v[d] = 0;
        double r = rint(v[d]);
        u[d] = v[d] - r;
        a[d] = imod((int)r, g.I[d]);
    }
}

struct L2KeyK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, const double* __restrict__ x, int n, L2Geom g, int* __restrict__ key, int* __restrict__ count) {
    for (int i = gpos.bid * kThreads + threadIdx.x; i < n; i += gpos.nb * kThreads) {
        int a[2];
        double u[2];
        grid_point2(g, x[3 * i], x[3 * i + 1], a, u);
        const int t = (a[0] / kL2Tile) * g.nt[1] + a[1] / kL2Tile;
        key[i] = t;
        atomicAdd(&count[t], 1);
    }
}
};

template <typename real>
struct L2PackK {
    static constexpr int kThreads = 256;
    // rank: the canonical ranks of the deterministic mode, or null (ranks from the cursors)
    __device__ static void run(GridPos gpos, const double* __restrict__ x, const double* __restrict__ q, int n, L2Geom g, const int* __restrict__ key, const int* __restrict__ start, int* __restrict__ cursor, const int* __restrict__ rank, int4* __restrict__ gp, vec4<real>* __restrict__ up) {
    for (int i = gpos.bid * kThreads + threadIdx.x; i < n; i += gpos.nb * kThreads) {
        int a[2];
        double u[2];
        grid_point2(g, x[3 * i], x[3 * i + 1], a, u);
        double zz = x[3 * i + 2], qq = q[i];
        if (!isfinite(zz)) zz = 0;
        if (!isfinite(qq)) qq = 0;
        double t = 2.0 * (zz - 0.5 * g.L[2]) / g.L[2];
        t = fmin(1.0, fmax(-1.0, t));
        const int k = key[i];
        const int p = start[k] + (rank ? rank[i] : atomicAdd(&cursor[k], 1));
        gp[p] = make_int4(a[0], a[1], 0, i);
        vec4<real> v;
        v.x = (real)u[0];
        v.y = (real)u[1];
        v.z = (real)t;
        v.w = (real)qq;
        up[p] = v;
    }
}
};

// The Gaussian window of eq. GS at node o of a P_w-point window, for a particle at offset
// u in [-1/2, 1/2] (grid units) from its nearest node: exp(-S d^2 / HW^2), d = o - HW - u.
template <typename real, int PW>
__device__ __forceinline__ real win2(int o, real u, real S, real inv_hw2) {
    constexpr int HW = (PW - 1) / 2;
    const real d = (real)(o - HW) - u;
    const real r2 = d * d * inv_hw2;
    return (r2 <= (real)1) ? dexp(-S * r2) : (real)0;
}

// The tiles (cyclic, first tile and count) holding the nearest nodes of particles whose
// windows of half-width HW reach nodes [x0, x0 + e) of a periodic line of I nodes in
// tiles of B.
__device__ __forceinline__ int l2_tile_span(int x0, int e, int HW, int I, int nt, int* first) {
    if (e + 2 * HW >= I) {
        *first = 0;
        return nt;
    }
    const int lo = imod(x0 - HW, I), hi = imod(x0 + e - 1 + HW, I);
    const int tlo = lo / kL2Tile, thi = hi / kL2Tile;
    int cnt = (lo <= hi) ? thi - tlo + 1 : (nt - tlo) + thi + 1;
    *first = tlo;
    return cnt < nt ? cnt : nt;
}

template <typename real>
struct L2SpreadArgs {
    const int4* gp;
    const vec4<real>* up;
    const int* tstart;  // ntiles + 1
    real* grid;         // P_s planes of I0 x I1 reals (y fastest)
    int I[2], nt[2], ntiles, Ps;
    real S, inv_hw2;
};

// Whether a window starting at node c (of PW nodes, periodic line of I nodes) reaches
// nodes [x0, x0 + e): the offset of x0 from c, taken mod I, is below PW, or c lies inside.
__device__ __forceinline__ bool l2_reaches(int c, int PW, int x0, int e, int I) {
    const int d = imod(x0 - c, I);      // nodes from the window's first node to x0
    const int d2 = imod(c - x0, I);     // nodes from x0 to the window's first node
    return d < PW || d2 < e;
}

template <typename real, int PW>
struct L2SpreadK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, const L2SpreadArgs<real>& a) {
    constexpr int HW = (PW - 1) / 2;
    __shared__ int2 cs[kL2Batch];
    __shared__ real wxs[kL2Batch * PW], wys[kL2Batch * PW];
    __shared__ __align__(16) real ts[kL2Batch * kL2Chunk];
    __shared__ int wcount[4];
    const int t = xcd_logical(a.ntiles, gpos);
    if (t < 0) return;
    const int tx = t / a.nt[1], ty = t % a.nt[1];
    const int x0 = tx * kL2Tile, y0 = ty * kL2Tile;
    const int ex = min(kL2Tile, a.I[0] - x0), ey = min(kL2Tile, a.I[1] - y0);
    const int lx = threadIdx.x / kL2Tile, ly = threadIdx.x % kL2Tile;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const bool valid = lx < ex && ly < ey;
    // a node outside the grid takes a far-away index that no window reaches
    const int nx = valid ? x0 + lx : -(1 << 29), ny = valid ? y0 + ly : -(1 << 29);
    int fx, fy;
    const int cntx = l2_tile_span(x0, ex, HW, a.I[0], a.nt[0], &fx);
    const int cnty = l2_tile_span(y0, ey, HW, a.I[1], a.nt[1], &fy);
    // the y tiles as at most two runs of consecutive tiles
    const int r1 = min(cnty, a.nt[1] - fy), r2 = cnty - r1;
    for (int c0 = 0; c0 < a.Ps; c0 += kL2Chunk) {
        real acc[kL2Chunk];
#pragma unroll
        for (int k = 0; k < kL2Chunk; ++k) acc[k] = 0;
        for (int ix = 0; ix < cntx; ++ix) {
            const int txx = (fx + ix) % a.nt[0];
            for (int run = 0; run < 2; ++run) {
                const int ty0 = run == 0 ? fy : 0, tn = run == 0 ? r1 : r2;
                if (tn <= 0) continue;
                const int beg = a.tstart[txx * a.nt[1] + ty0], end = a.tstart[txx * a.nt[1] + ty0 + tn];
                for (int base = beg; base < end; base += kL2Batch) {
                    // the next kL2Batch particles of the range; those whose windows reach the
                    // tile are compacted into the staging arrays
                    const int pi = base + (int)threadIdx.x;
                    bool keep = false;
                    int4 g = make_int4(0, 0, 0, 0);
                    if ((int)threadIdx.x < kL2Batch && pi < end) {
                        g = a.gp[pi];
                        keep = l2_reaches(g.x - HW, PW, x0, ex, a.I[0]) && l2_reaches(g.y - HW, PW, y0, ey, a.I[1]);
                    }
                    const unsigned long long m = __ballot(keep);
                    __syncthreads();  // the previous batch's staging is no longer read
                    if (lane == 0) wcount[wid] = __popcll(m);
                    __syncthreads();
                    int off = 0, nb = 0;
                    for (int w = 0; w < 4; ++w) {
                        off += w < wid ? wcount[w] : 0;
                        nb += wcount[w];
                    }
                    if (keep) {
                        const int j = off + __popcll(m & ((1ull << lane) - 1ull));
                        const vec4<real> u = a.up[pi];
                        cs[j] = make_int2(g.x - HW, g.y - HW);
#pragma unroll
                        for (int o = 0; o < PW; ++o) {
                            wxs[j * PW + o] = u.w * win2<real, PW>(o, u.x, a.S, a.inv_hw2);
                            wys[j * PW + o] = win2<real, PW>(o, u.y, a.S, a.inv_hw2);
                        }
                        // T_k(t) for k in [c0, c0 + 8)
                        real T0 = 1, T1 = u.z;
                        for (int k = 0; k < c0 + kL2Chunk; ++k) {
                            const real Tk = k == 0 ? (real)1 : (k == 1 ? u.z : (real)2 * u.z * T1 - T0);
                            if (k >= 2) {
                                T0 = T1;
                                T1 = Tk;
                            }
                            if (k >= c0) ts[j * kL2Chunk + (k - c0)] = Tk;
                        }
                    }
                    __syncthreads();
                    for (int j = 0; j < nb; ++j) {
                        const int2 c = cs[j];
                        int dx = nx - c.x, dy = ny - c.y;
                        dx += dx < 0 ? a.I[0] : 0;
                        dx -= dx >= a.I[0] ? a.I[0] : 0;
                        dy += dy < 0 ? a.I[1] : 0;
                        dy -= dy >= a.I[1] ? a.I[1] : 0;
                        if ((unsigned)dx < (unsigned)PW && (unsigned)dy < (unsigned)PW) {
                            const real w = wxs[j * PW + dx] * wys[j * PW + dy];
#pragma unroll
                            for (int k = 0; k < kL2Chunk; ++k) acc[k] += w * ts[j * kL2Chunk + k];
                        }
                    }
                }
            }
        }
        if (valid) {
            const size_t plane = (size_t)a.I[0] * a.I[1];
            const size_t node = (size_t)nx * a.I[1] + ny;
#pragma unroll
            for (int k = 0; k < kL2Chunk; ++k)
                if (c0 + k < a.Ps) a.grid[(size_t)(c0 + k) * plane + node] = acc[k];
        }
    }
}
};

// Scaling of every mode of the half spectrum: uhat(k, n) = sum_a K(k)[n][a] Shat2(k, a),
// n < P, a < P_s, in place (a thread reads all P_s planes of its mode before it writes).
template <typename real>
struct L2ScaleArgs {
    cpx<real>* cg;        // planes of I0 rows of Kys complex (k_y fastest)
    int I0, Ky, Kys, P, Ps, Q;
    // exact form: K per (n, a) as planes over the modes (j_x = min(i_x, I0 - i_x), k_y):
    // kt[((n P_s + a) (I0/2 + 1) + j_x) Ky + k_y], scaled
    const real* kt;
    // Taylor form: per long-range Gaussian l, e_l = s_l^2/4 and coef[l][p] (p < Q), with
    // A_p(k) = sum_l e^{-e_l |k|^2} coef[l][p]; B_p (Q x P x P_s); 1/What2^2 per direction
    // (the 1/(I0 I1) and pi folded into coef)
    const real* el;
    const real* coef;
    int nl;
    const real* bp;
    const real* winv_x;  // I0
    const real* winv_y;  // Ky
    real dkx, dky;       // 2 pi / L_x, 2 pi / L_y
    int tables_in_lds;   // Taylor: e_l, coef and B_p staged in LDS
};

constexpr int kL2ScaleThreads = 128;
constexpr int kL2MaxQ = 16;

// LDS of the scaling kernel: the modes' P_s source values per thread, then (Taylor, when
// they fit) e_l, coef and B_p.
inline size_t l2_scale_lds(int Ps, int nl, int Q, int P, size_t rs, bool tables) {
    size_t b = (size_t)kL2ScaleThreads * Ps * 2 * rs;
    if (tables) b += ((size_t)nl * (1 + Q) + (size_t)Q * P * Ps) * rs;
    return b;
}

template <typename real>
struct L2ScaleK {
    static constexpr int kThreads = kL2ScaleThreads;
    __device__ static void run(GridPos gpos, const L2ScaleArgs<real>& a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<real>* rho = reinterpret_cast<cpx<real>*>(smem_raw);  // Ps x kL2ScaleThreads
    real* tl = reinterpret_cast<real*>(rho + (size_t)a.Ps * kL2ScaleThreads);
    const real* el = a.el;
    const real* coef = a.coef;
    const real* bp = a.bp;
    if (a.Q > 0 && a.tables_in_lds) {
        real* lel = tl;
        real* lco = lel + a.nl;
        real* lbp = lco + a.nl * a.Q;
        for (int i = threadIdx.x; i < a.nl; i += kL2ScaleThreads) lel[i] = a.el[i];
        for (int i = threadIdx.x; i < a.nl * a.Q; i += kL2ScaleThreads) lco[i] = a.coef[i];
        for (int i = threadIdx.x; i < a.Q * a.P * a.Ps; i += kL2ScaleThreads) lbp[i] = a.bp[i];
        __syncthreads();
        el = lel;
        coef = lco;
        bp = lbp;
    }
    const int mode = gpos.bid * kL2ScaleThreads + threadIdx.x;
    if (mode >= a.I0 * a.Ky) return;  // no barrier below
    const int ix = mode / a.Ky, ky = mode - ix * a.Ky;
    const size_t plane = (size_t)a.I0 * a.Kys;
    cpx<real>* cell = a.cg + (size_t)ix * a.Kys + ky;
    for (int s = 0; s < a.Ps; ++s) rho[s * kL2ScaleThreads + threadIdx.x] = cell[(size_t)s * plane];
    if (a.Q > 0) {
        const int fx = ix < (a.I0 + 1) / 2 ? ix : ix - a.I0;
        const real kx = a.dkx * (real)fx, kyv = a.dky * (real)ky;
        const real k2 = kx * kx + kyv * kyv;
        real A[kL2MaxQ];
#pragma unroll
        for (int p = 0; p < kL2MaxQ; ++p) A[p] = 0;
        for (int l = 0; l < a.nl; ++l) {
            const real e = dexp(-el[l] * k2);
            const real* c = coef + l * a.Q;
#pragma unroll
            for (int p = 0; p < kL2MaxQ; ++p)
                if (p < a.Q) A[p] += e * c[p];
        }
        if (ix == 0 && ky == 0) A[0] = 0;  // the k = 0 constant multiplies sum_j q_j
        const real wv = a.winv_x[ix] * a.winv_y[ky];
        for (int n = 0; n < a.P; ++n) {
            real sr = 0, si = 0;
            for (int s = 0; s < a.Ps; ++s) {
                real kk = 0;
#pragma unroll
                for (int p = 0; p < kL2MaxQ; ++p)
                    if (p < a.Q) kk += A[p] * bp[(p * a.P + n) * a.Ps + s];
                const cpx<real> v = rho[s * kL2ScaleThreads + threadIdx.x];
                sr += kk * v.x;
                si += kk * v.y;
            }
            cell[(size_t)n * plane] = cpx<real>{wv * sr, wv * si};
        }
    } else {
        const int jx = min(ix, a.I0 - ix);
        const size_t kplane = (size_t)(a.I0 / 2 + 1) * a.Ky;
        const real* K = a.kt + (size_t)jx * a.Ky + ky;
        for (int n = 0; n < a.P; ++n) {
            real sr = 0, si = 0;
            for (int s = 0; s < a.Ps; ++s) {
                const real kk = K[(size_t)(n * a.Ps + s) * kplane];
                const cpx<real> v = rho[s * kL2ScaleThreads + threadIdx.x];
                sr += kk * v.x;
                si += kk * v.y;
            }
            cell[(size_t)n * plane] = cpx<real>{sr, si};
        }
    }
}
};

template <typename real>
struct L2GatherArgs {
    const int4* gp;
    const vec4<real>* up;
    const int* tstart;
    const real* grid;  // P planes of I0 x I1 reals
    vec4<real>* part;  // long part of each particle: phi, grad
    int I[2], nt[2], ntiles, P;
    real S, inv_hw2, dcoef[2], area, dzf;
};

constexpr int kL2GatherThreads = 64;

template <typename real, int PW>
struct L2GatherK {
    static constexpr int kThreads = kL2GatherThreads;
    __device__ static void run(GridPos gpos, const L2GatherArgs<real>& a) {
    constexpr int HW = (PW - 1) / 2;
    constexpr int HX = kL2Tile + PW - 1;
    __shared__ real halo[HX * HX * kL2Chunk];  // (lx, ly, k), k fastest
    const int t = xcd_logical(a.ntiles, gpos);
    if (t < 0) return;
    const int beg = a.tstart[t], end = a.tstart[t + 1];
    if (beg == end) return;
    const int tx = t / a.nt[1], ty = t % a.nt[1];
    const int x0 = tx * kL2Tile, y0 = ty * kL2Tile;
    const size_t plane = (size_t)a.I[0] * a.I[1];
    const int nchunks = (a.P + kL2Chunk - 1) / kL2Chunk;
    for (int pb = beg; pb < end; pb += kL2GatherThreads) {
        const int p = pb + threadIdx.x;
        const bool active = p < end;
        int4 g = make_int4(x0, y0, 0, 0);
        vec4<real> u = {0, 0, 0, 0};
        if (active) {
            g = a.gp[p];
            u = a.up[p];
        }
        real phi = 0, gx = 0, gy = 0, gz = 0;
        for (int ci = 0; ci < nchunks; ++ci) {
            const int c0 = ci * kL2Chunk;
            if (nchunks > 1 || pb == beg) {
                __syncthreads();
                // y fastest in the loads (coalesced rows of the grid)
                for (int idx = threadIdx.x; idx < HX * HX * kL2Chunk; idx += kL2GatherThreads) {
                    const int ly = idx % HX, r = idx / HX, lx = r % HX, k = r / HX;
                    const int gxn = imod(x0 - HW + lx, a.I[0]), gyn = imod(y0 - HW + ly, a.I[1]);
                    halo[(lx * HX + ly) * kL2Chunk + k] =
                        (c0 + k < a.P) ? a.grid[(size_t)(c0 + k) * plane + (size_t)gxn * a.I[1] + gyn] : (real)0;
                }
                __syncthreads();
            }
            if (!active) continue;
            // T_k(t) and T_k'(t) = k U_{k-1}(t) for k in [c0, c0 + 8)
            real Tt[kL2Chunk], Td[kL2Chunk];
            {
                real T0 = 1, T1 = u.z, U0 = 1, U1 = 2 * u.z;
                for (int k = 0; k < c0 + kL2Chunk; ++k) {
                    real Tk, Dk;
                    if (k == 0) {
                        Tk = 1;
                        Dk = 0;
                    } else if (k == 1) {
                        Tk = u.z;
                        Dk = 1;
                    } else {
                        Tk = (real)2 * u.z * T1 - T0;
                        Dk = (real)k * U1;
                        const real U2 = (real)2 * u.z * U1 - U0;
                        T0 = T1;
                        T1 = Tk;
                        U0 = U1;
                        U1 = U2;
                    }
                    if (k >= c0) {
                        Tt[k - c0] = Tk;
                        Td[k - c0] = Dk;
                    }
                }
            }
            real wy[PW], dwy[PW];
#pragma unroll
            for (int o = 0; o < PW; ++o) {
                wy[o] = win2<real, PW>(o, u.y, a.S, a.inv_hw2);
                dwy[o] = a.dcoef[1] * ((real)(o - HW) - u.y) * wy[o];
            }
            const int lx0 = g.x - x0, ly0 = g.y - y0;
            for (int ox = 0; ox < PW; ++ox) {
                const real wx = win2<real, PW>(ox, u.x, a.S, a.inv_hw2);
                const real dwx = a.dcoef[0] * ((real)(ox - HW) - u.x) * wx;
                real s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                for (int oy = 0; oy < PW; ++oy) {
                    const real* cell = halo + ((lx0 + ox) * HX + (ly0 + oy)) * kL2Chunk;
                    real c0s = 0, c1s = 0;
#pragma unroll
                    for (int k = 0; k < kL2Chunk; ++k) {
                        c0s += Tt[k] * cell[k];
                        c1s += Td[k] * cell[k];
                    }
                    s0 += wy[oy] * c0s;
                    s1 += dwy[oy] * c0s;
                    s2 += wy[oy] * c1s;
                }
                phi += wx * s0;
                gx += dwx * s0;
                gy += wx * s1;
                gz += wx * s2;
            }
        }
        if (active) a.part[g.w] = vec4<real>{a.area * phi, a.area * gx, a.area * gy, a.area * a.dzf * gz};
    }
}
};

template <typename real, int PW>
hipError_t l2_spread_gather_pw(Plan& p, bool spread) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int ntiles = r.ntile2[0] * r.ntile2[1];
    constexpr int HW = (PW - 1) / 2;
    const real inv_hw2 = (real)(1.0 / ((double)HW * HW));
    if (spread) {
        L2SpreadArgs<real> a;
        a.gp = (const int4*)ws.l2_g;
        a.up = (const vec4<real>*)ws.l2_u;
        a.tstart = ws.l2_tile_start;
        a.grid = (real*)ws.l2_grid;
        for (int d = 0; d < 2; ++d) {
            a.I[d] = r.I2[d];
            a.nt[d] = r.ntile2[d];
        }
        a.ntiles = ntiles;
        a.Ps = r.Ps;
        a.S = (real)r.S2;
        a.inv_hw2 = inv_hw2;
        return launch<L2SpreadK<real, PW>, false>(p, xcd_grid(ntiles), 0, a);
    } else {
        L2GatherArgs<real> a;
        a.gp = (const int4*)ws.l2_g;
        a.up = (const vec4<real>*)ws.l2_u;
        a.tstart = ws.l2_tile_start;
        a.grid = (const real*)ws.l2_grid;
        a.part = (vec4<real>*)ws.parts + 2 * r.n;
        for (int d = 0; d < 2; ++d) {
            a.I[d] = r.I2[d];
            a.nt[d] = r.ntile2[d];
            a.dcoef[d] = (real)(2.0 * r.S2 / ((double)HW * HW * r.h2[d]));
        }
        a.ntiles = ntiles;
        a.P = r.P;
        a.S = (real)r.S2;
        a.inv_hw2 = inv_hw2;
        a.area = (real)(r.h2[0] * r.h2[1]);
        a.dzf = (real)(2.0 / r.L[2]);
        return launch<L2GatherK<real, PW>, false>(p, xcd_grid(ntiles), 0, a);
    }
}

template <typename real>
hipError_t l2_spread_gather(Plan& p, bool spread) {
    switch (p.r.Pw2) {
        case 3: return l2_spread_gather_pw<real, 3>(p, spread);
        case 5: return l2_spread_gather_pw<real, 5>(p, spread);
        case 7: return l2_spread_gather_pw<real, 7>(p, spread);
        case 9: return l2_spread_gather_pw<real, 9>(p, spread);
        case 11: return l2_spread_gather_pw<real, 11>(p, spread);
        case 13: return l2_spread_gather_pw<real, 13>(p, spread);
        case 15: return l2_spread_gather_pw<real, 15>(p, spread);
        default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t run_long_fft(Plan& p, const double* x, const double* q) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int n = (int)r.n;
    if (r.Ps > kLong2MaxPlanes || r.P > kLong2MaxPlanes || r.Q > kL2MaxQ || r.I2[0] < 2 * r.Pw2 ||
        r.I2[1] < 2 * r.Pw2 || (r.I2[1] & 1))
        return hipErrorInvalidConfiguration;
    L2Geom g;
    for (int d = 0; d < 3; ++d) g.L[d] = r.L[d];
    for (int d = 0; d < 2; ++d) {
        g.h[d] = r.h2[d];
        g.I[d] = r.I2[d];
        g.nt[d] = r.ntile2[d];
    }
    const int ntiles = r.ntile2[0] * r.ntile2[1];
    const int blocks = std::min((n + 255) / 256, 8192);
    int t = timer_id(p, "long2_sort");
    timer_begin(p, t);
    hipError_t e = launch_fill_int(p, ws.l2_tile_start, 0, (int64_t)ntiles + 1);
    if (e == hipSuccess) e = launch_fill_int(p, ws.l2_tile_cursor, 0, ntiles);
    if (e == hipSuccess) e = launch<L2KeyK, false>(p, blocks, 0, x, n, g, ws.key, ws.l2_tile_start);
    if (e == hipSuccess) e = launch_exclusive_scan(p, ws.l2_tile_start, ntiles + 1, ws.scan_tmp);
    if (e == hipSuccess && r.deterministic)
        e = launch_canonical_ranks(p, ws.key, false, n, ws.l2_tile_start, ntiles, ws.l2_tile_cursor, ws.det_idx,
                                   ws.det_rank);
    if (e == hipSuccess)
        e = launch<L2PackK<real>, false>(p, blocks, 0, x, q, n, g, (const int*)ws.key, (const int*)ws.l2_tile_start,
                                         ws.l2_tile_cursor, (const int*)(r.deterministic ? ws.det_rank : nullptr),
                                         (int4*)ws.l2_g, (vec4<real>*)ws.l2_u);
    timer_end(p, t);
    if (e != hipSuccess) return e;
    t = timer_id(p, "long2_spread");
    timer_begin(p, t);
    if ((e = l2_spread_gather<real>(p, true)) != hipSuccess) return e;
    timer_end(p, t);
    if ((e = launch_fft_long2(p, -1, r.Ps)) != hipSuccess) return e;
    {
        const int Ky = r.I2[1] / 2 + 1;
        L2ScaleArgs<real> a;
        a.cg = (cpx<real>*)ws.l2_cgrid;
        a.I0 = r.I2[0];
        a.Ky = Ky;
        a.Kys = cgrid_stride(r.I2[1]);
        a.P = r.P;
        a.Ps = r.Ps;
        a.Q = r.Q;
        a.kt = (const real*)ws.l2_kt_r;
        a.el = (const real*)ws.l2_el;
        a.coef = (const real*)ws.l2_coef;
        a.nl = r.M - r.m;
        a.bp = (const real*)ws.l2_bp;
        a.winv_x = (const real*)ws.l2_winv_x;
        a.winv_y = (const real*)ws.l2_winv_y;
        a.dkx = (real)(2.0 * 3.14159265358979323846 / r.L[0]);
        a.dky = (real)(2.0 * 3.14159265358979323846 / r.L[1]);
        const int nl = r.M - r.m;
        a.tables_in_lds = r.Q > 0 && l2_scale_lds(r.Ps, nl, r.Q, r.P, sizeof(real), true) <= 65536;
        const size_t lds = l2_scale_lds(r.Ps, nl, r.Q, r.P, sizeof(real), a.tables_in_lds);
        if (lds > 65536) return hipErrorInvalidConfiguration;
        const int64_t modes = (int64_t)r.I2[0] * Ky;
        t = timer_id(p, "long2_scale");
        timer_begin(p, t);
        e = launch<L2ScaleK<real>, false>(p, (unsigned)((modes + kL2ScaleThreads - 1) / kL2ScaleThreads), lds, a);
        timer_end(p, t);
        if (e != hipSuccess) return e;
    }
    if ((e = launch_fft_long2(p, +1, r.P)) != hipSuccess) return e;
    t = timer_id(p, "long2_gather");
    timer_begin(p, t);
    e = l2_spread_gather<real>(p, false);
    timer_end(p, t);
    return e;
}

}  // namespace

hipError_t launch_long_fft(Plan& p, const double* x, const double* q) {
    if (p.r.prec == SOG_PREC_FP64) return run_long_fft<double>(p, x, q);
    return run_long_fft<float>(p, x, q);
}

}  // namespace sog
