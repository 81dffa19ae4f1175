// Mid-range Fourier spectral solver, gridding and gathering (Alg. al::mid steps 1 and 5,
// eqs. gridding and Phiconv) with the Gaussian window of eq. GS.
//
// Grid: nodes X_a = -Lx/2 + a h_x (a < I_x), likewise y, Z_c = -L_z*/2 + c h_z (c < I_z*),
// stored z-fastest: grid[(a * I_y + b) * I_z* + c].  Window on P_w nodes around the
// nearest node, W(d) = exp(-S (d/H)^2) for |d| <= H = (P_w - 1) h / 2, else 0.
//
// The grid is cut into tiles of B_x x B_y x B_z nodes and particles are sorted by the tile
// of their nearest node (a counting sort).  Gridding: the workgroup of a tile spreads its
// particles into an LDS copy of the tile plus a (P_w - 1) halo and adds that block into
// the grid with float atomics (one launch for all tiles; measured faster than colouring
// the tiles into launches whose blocks never overlap).  Gathering: the workgroup of a
// tile loads the tile plus halo into LDS and evaluates Phi and grad Phi for its
// particles.
#include "launch.hpp"

namespace sog {

namespace {

struct MidGeom {
    double L[3];
    double h[3];
    double Lzs;
    int I[3];   // I_x, I_y, I_z* (node counts of the stored grid)
    int B[3];
    int nt[3];
    int HW;     // (P_w - 1) / 2
    int zlo, zhi;  // z planes that may carry window mass
};

__device__ __forceinline__ void grid_point(const MidGeom& g, double x, double y, double z, int a[3], double u[3]) {
    double v[3];
    v[0] = wrap_periodic(x, g.L[0]) / g.h[0];
    v[1] = wrap_periodic(y, g.L[1]) / g.h[1];
    v[2] = (z - 0.5 * g.L[2] + 0.5 * g.Lzs) / g.h[2];
    for (int d = 0; d < 3; ++d) {
        if (!isfinite(v[d])) v[d] = (d == 2) ? 0.5 * g.I[2] : 0.0;
        double r = rint(v[d]);
        u[d] = v[d] - r;
        int k = (int)r;
        if (d < 2) {
            a[d] = imod(k, g.I[d]);
        } else {
            a[d] = min(max(k, g.zlo + g.HW), g.zhi - 1 - g.HW);  // only invalid input hits the clamp
            if (k != a[d]) u[d] = 0.0;
        }
    }
}

// tile of every particle's nearest node and its rank within the tile (the counting sort's
// histogram)
struct MidKeyK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, const double* __restrict__ x, int n, MidGeom g, int2* __restrict__ key, int* __restrict__ count) {
    for (int i = gpos.bid * kThreads + threadIdx.x; i < n; i += gpos.nb * kThreads) {
        int a[3];
        double u[3];
        grid_point(g, x[3 * i], x[3 * i + 1], x[3 * i + 2], a, u);
        const int k = ((a[0] / g.B[0]) * g.nt[1] + a[1] / g.B[1]) * g.nt[2] + a[2] / g.B[2];
        // kMidSub counters per tile, taken in turn by consecutive particles: the returning
        // atomics cost less with fewer of them on one address
        const int kb = k * kMidSub + (i & (kMidSub - 1));
        key[i] = make_int2(kb, atomicAdd(&count[kb], 1));
    }
}
};

// Scatter of the counting sort: each particle's grid point and offset record written at
// its place in tile order, tile start plus rank (particles read in their own order, no
// atomics).
template <typename real>
struct MidPackK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, const double* __restrict__ x, const double* __restrict__ q, int n, MidGeom g, const int2* __restrict__ key, const int* __restrict__ start, int4* __restrict__ gp, vec4<real>* __restrict__ up) {
    for (int i = gpos.bid * kThreads + threadIdx.x; i < n; i += gpos.nb * kThreads) {
        const int2 kr = key[i];
        const int p = start[kr.x] + kr.y;
        int a[3];
        double u[3];
        grid_point(g, x[3 * i], x[3 * i + 1], x[3 * i + 2], a, u);
        double qq = q[i];
        if (!isfinite(qq)) qq = 0;
        gp[p] = make_int4(a[0], a[1], a[2], i);
        vec4<real> v;
        v.x = (real)u[0];
        v.y = (real)u[1];
        v.z = (real)u[2];
        v.w = (real)qq;
        up[p] = v;
    }
}
};

// The window on the P_w nodes nearest a particle, at offset d = node - particle (units of
// h): the truncated Gaussian exp(-S d^2 / HW^2), |d| <= HW (eq. GS), the ES window
// exp(beta (sqrt(1 - (d/a)^2) - 1)), |d| < a = P_w / 2, or a polynomial window (Remark
// rmk::PWindow: node o's weight as a polynomial in the particle's offset u from its nearest
// node, |u| <= 1/2; the KB window's, fitted by the planner).  The transforms of the windows
// enter the multiplier tables.
enum { kWinGauss = 0, kWinES = 1, kWinPoly = 2 };
template <typename real>
struct WinShape {
    real S, inv_hw2;     // Gaussian
    real beta, inv_a;    // ES
    const real* poly;    // polynomial: per node nu + 1 monomial coefficients in u, highest first
    int kind, nu;
};

// node o's polynomial weight at offset u, and its derivative in u (Horner).  Each node's
// row holds nu + 1 coefficients, a multiple of 4 (leading zeros, which leave Horner's
// rule exact), taken 4 at a time.  The table (global memory, read-only during a call) is
// read through the constant address space: where the node is the same in every lane (the
// gathering's loops) the reads are scalar loads and the coefficients scalar operands.
template <typename real>
using win_table = const __attribute__((address_space(4))) real*;
template <typename real>
__device__ __forceinline__ real win_poly(int o, real u, const WinShape<real>& s) {
    const win_table<real> c = (win_table<real>)s.poly + o * (s.nu + 1);
    real w = 0;
    for (int j = 0; j <= s.nu; j += 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) w = fma(w, u, c[j + i]);
    }
    return w;
}
template <typename real>
__device__ __forceinline__ void win_poly_d(int o, real u, const WinShape<real>& s, real& w, real& dw) {
    const win_table<real> c = (win_table<real>)s.poly + o * (s.nu + 1);
    real v = 0, d = 0;
    for (int j = 0; j <= s.nu; j += 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            d = fma(d, u, v);
            v = fma(v, u, c[j + i]);
        }
    }
    w = v;
    dw = d;
}
// all P_w nodes' weights and derivatives (dcoef d/du) at once, the nodes' Horner chains
// side by side
template <typename real, int PW>
__device__ __forceinline__ void win_poly_all(real u, const WinShape<real>& s, real dcoef, real* w, real* dw) {
    const int n1 = s.nu + 1;
    // the table is read through the constant address space (as win_poly; a flat pointer
    // taken from the LDS copy of a batched launch's arguments made the compiler emit an
    // invalid aperture test)
    const win_table<real> c = (win_table<real>)s.poly;
#pragma unroll
    for (int o = 0; o < PW; ++o) w[o] = dw[o] = 0;
    for (int j = 0; j < n1; ++j) {
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            dw[o] = fma(dw[o], u, w[o]);
            w[o] = fma(w[o], u, c[o * n1 + j]);
        }
    }
#pragma unroll
    for (int o = 0; o < PW; ++o) dw[o] *= dcoef;
}

template <typename real, int PW>
__device__ __forceinline__ real win(int o, real u, const WinShape<real>& s) {
    constexpr int HW = (PW - 1) / 2;
    if (s.kind == kWinPoly) return win_poly(o, u, s);
    const real d = (real)(o - HW) - u;
    if (s.kind == kWinES) {
        const real t = fabs(d) * s.inv_a;
        const real r1 = ((real)1 - t) * ((real)1 + t);
        return (r1 > (real)0) ? dexp(s.beta * (sqrt(r1) - (real)1)) : (real)0;
    }
    const real r2 = d * d * s.inv_hw2;
    return (r2 <= (real)1) ? dexp(-s.S * r2) : (real)0;
}

// the weight and its derivative in the particle coordinate, dcoef d W (Gaussian, dcoef =
// 2 S / (HW^2 h)), dcoef d W / sqrt(1 - (d/a)^2) (ES, dcoef = beta / (a^2 h)) or
// dcoef p'(u) (polynomial, dcoef = 1 / h)
template <typename real, int PW>
__device__ __forceinline__ void win_d(int o, real u, const WinShape<real>& s, real dcoef, real& w, real& dw) {
    constexpr int HW = (PW - 1) / 2;
    if (s.kind == kWinPoly) {
        real dp;
        win_poly_d(o, u, s, w, dp);
        dw = dcoef * dp;
        return;
    }
    const real d = (real)(o - HW) - u;
    if (s.kind == kWinES) {
        const real t = fabs(d) * s.inv_a;
        const real r1 = ((real)1 - t) * ((real)1 + t);
        const real sq = sqrt(r1 > (real)0 ? r1 : (real)1);
        w = (r1 > (real)0) ? dexp(s.beta * (sq - (real)1)) : (real)0;
        dw = dcoef * d * w / sq;
        return;
    }
    const real r2 = d * d * s.inv_hw2;
    w = (r2 <= (real)1) ? dexp(-s.S * r2) : (real)0;
    dw = dcoef * d * w;
}

constexpr int kSpreadThreads = 256;  // 4 waves, one per group of x planes
constexpr int kHaloILP = 24;  // x planes of a halo column loaded or added in flight together

// a halo node index into [0, n): it lies in [-n, 3n), since the halo half-width is below
// n (I >= 2 P_w) and a tile's first node plus its edge is below 2n
__device__ __forceinline__ int wrap_once(int i, int n) {
    if (i < 0) i += n;
    if (i >= n) i -= n;
    if (i >= n) i -= n;
    return i;
}

template <typename real>
struct SpreadArgs {
    const int4* gp;
    const vec4<real>* up;
    const int* tstart;  // tile t owns particles [tstart[t kMidSub], tstart[(t + 1) kMidSub]) (the gather's lists)
    const signed char* nodes;  // (y, z) window node of each lane per pass: 256 oy, then 256 oz
    real* grid;
    int I[3];
    int B[3];
    int nt[3];
    int ntiles;
    WinShape<real> ws;
    // phase < 0: every tile, blocks added with atomics.  Else (deterministic mode, see
    // tile_colour) only the tiles of one colour, pfirst[d] + pstep[d] j, j < pcount[d] per
    // direction, blocks added with plain read-add-writes.
    int phase;
    int pfirst[3], pstep[3], pcount[3];
};

// Owner-tile gridding: the workgroup of a tile spreads the particles whose nearest node
// lies in the tile into an LDS copy of the tile plus a (P_w - 1) halo -- every window
// fits, nothing is clipped -- and then adds that block into the global grid atomically.
// Inside the tile no LDS atomics are used (float LDS atomics are slow on this GPU): wave w
// owns the x planes of the halo block with x = w mod 4 and its lanes take the window's
// (y, z) nodes, so within a particle the lanes touch distinct nodes and no two waves ever
// touch the same node; each wave walks the staged particles in order without
// synchronising with the others.  Per staged particle the batch holds its y and z
// weights, its x weights already rotated to each wave's planes and each wave's byte
// offset of its first plane, so a wave's reads of the next particle do not depend on each
// other and are issued before the current particle's writes.  Every wave updates
// ceil(P_w / 4) planes x P_w^2-node passes per particle without branching: a plane past
// the window has zero weight (it is one of the wave's own planes, possibly one of the
// padding planes after the block), and a lane without a node in a pass updates, with
// zero weight, a dummy node of the same plane that no window node uses (DUMMY) or its
// private sink slot.
template <typename real, int PW, bool DUMMY>
struct SpreadK {
    static constexpr int kThreads = kSpreadThreads;
    __device__ static void run(GridPos gpos, const SpreadArgs<real>& a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int HW = (PW - 1) / 2;
    constexpr int NPASS = (PW * PW + 63) / 64;   // groups of 64 (y, z) window nodes
    constexpr int NPL = (PW + 3) / 4;            // x planes of a window per wave (at most)
    constexpr int NPAD = 4 * NPL - PW;           // padding planes after the block
    constexpr int NW = 2 * PW + 1;               // staged y, z weights and a zero per particle
    static_assert(NPL <= 4, "window too wide for four plane groups");
    int t, tx, ty, tz;
    if (a.phase < 0) {
        t = xcd_logical(a.ntiles, gpos);
        if (t < 0) return;
        tz = t % a.nt[2], ty = (t / a.nt[2]) % a.nt[1], tx = t / (a.nt[2] * a.nt[1]);
    } else {
        const int l = xcd_logical(a.pcount[0] * a.pcount[1] * a.pcount[2], gpos);
        if (l < 0) return;
        tz = a.pfirst[2] + a.pstep[2] * (l % a.pcount[2]);
        ty = a.pfirst[1] + a.pstep[1] * ((l / a.pcount[2]) % a.pcount[1]);
        tx = a.pfirst[0] + a.pstep[0] * (l / (a.pcount[2] * a.pcount[1]));
        t = (tx * a.nt[1] + ty) * a.nt[2] + tz;
    }
    const int beg = a.tstart[t * kMidSub], end = a.tstart[(t + 1) * kMidSub];
    if (beg == end) return;
    const int x0 = tx * a.B[0], y0 = ty * a.B[1], z0 = tz * a.B[2];
    const int HX = a.B[0] + PW - 1, HY = a.B[1] + PW - 1, HZ = a.B[2] + PW - 1;
    const int HYZ = HY * HZ;
    const int totp = (HX + NPAD) * HYZ;
    real* halo = reinterpret_cast<real*>(smem_raw);
    unsigned char* hb = smem_raw;                  // byte view: node offsets are LDS addresses
    real* wyzs = halo + totp + 64;                 // kSpreadStage x NW: wy, wz, 0
    // kSpreadStage x 16: q wx rotated per wave, on a 32-byte boundary so that a wave reads
    // its four in one vector load
    const size_t wx_off = ((((size_t)totp + 64 + (size_t)kSpreadStage * NW) * sizeof(real)) + 31) & ~(size_t)31;
    real* wxs = reinterpret_cast<real*>(smem_raw + wx_off);
    const size_t rec_off = wx_off + (size_t)kSpreadStage * 16 * sizeof(real);
    vec4<real>* sup = reinterpret_cast<vec4<real>*>(smem_raw + rec_off);  // kSpreadStage: u, q
    int4* meta = reinterpret_cast<int4*>(sup + kSpreadStage);  // per wave: byte offset of its first plane
    int* slx = reinterpret_cast<int*>(meta + kSpreadStage);      // x node of the particle in the block
    for (int k = threadIdx.x; k < totp + 64; k += kSpreadThreads) halo[k] = 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int planestep = 4 * HYZ;
    // this lane's (y, z) node of the window in each pass (chosen by the planner so that
    // the 64 lanes of a pass hit distinct LDS banks for any window corner), as byte
    // offsets per plane; its y and z weight slots (the zero slot for a dummy node)
    int off[NPL][NPASS], oy2[NPASS], oz2[NPASS];
    bool has[NPASS];
#pragma unroll
    for (int ps = 0; ps < NPASS; ++ps) {
        const int oy = a.nodes[ps * 64 + lane], oz = a.nodes[256 + ps * 64 + lane];
        has[ps] = oy >= 0;
        oy2[ps] = has[ps] ? oy : 0;
        oz2[ps] = (has[ps] && oz < PW) ? PW + oz : 2 * PW;
        const int o = has[ps] ? oy * HZ + oz : 0;
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) off[pl][ps] = (pl * planestep + o) * (int)sizeof(real);
    }
    const int sinkb = (totp + lane) * (int)sizeof(real);
    // thread t holds particle g0 + t of the tile's current group of kSpreadThreads
    // particles (one load per group of batches; indices clamped into the tile's list, so
    // every load is valid and unconditional)
    static_assert(kSpreadThreads % kSpreadStage == 0, "a group of particles is whole batches");
    int g0 = beg;
    int4 gq = a.gp[min(beg + (int)threadIdx.x, end - 1)];
    vec4<real> uq = a.up[min(beg + (int)threadIdx.x, end - 1)];
    for (int c0 = beg; c0 < end; c0 += kSpreadStage) {
        const int cnt = min(kSpreadStage, end - c0);
        if (c0 - g0 >= kSpreadThreads) {
            g0 += kSpreadThreads;
            gq = a.gp[min(g0 + (int)threadIdx.x, end - 1)];
            uq = a.up[min(g0 + (int)threadIdx.x, end - 1)];
        }
        __syncthreads();
        // this thread's place in the batch
        const int sidx = (int)threadIdx.x - (c0 - g0);
        if (sidx >= 0 && sidx < cnt) {
            const int lx0 = gq.x - x0;
            const int corner = lx0 * HYZ + (gq.y - y0) * HZ + (gq.z - z0);
            int m[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) m[g] = (corner + ((g - lx0) & 3) * HYZ) * (int)sizeof(real);
            meta[sidx] = int4{m[0], m[1], m[2], m[3]};
            slx[sidx] = lx0;
            sup[sidx] = vec4<real>{uq.x, uq.y, uq.z, uq.w};
        }
        __syncthreads();
        // y, z weights and a zero; per wave g the x weights of its planes (x = g mod 4)
        for (int idx = threadIdx.x; idx < cnt * (NW + 16); idx += kSpreadThreads) {
            if (idx < cnt * NW) {
                const int i = idx / NW, r = idx - i * NW;
                const vec4<real> u = sup[i];
                wyzs[idx] = (r < 2 * PW) ? win<real, PW>(r < PW ? r : r - PW, r < PW ? u.y : u.z, a.ws)
                                         : (real)0;
            } else {
                const int jdx = idx - cnt * NW;
                const int i = jdx >> 4, g = (jdx >> 2) & 3, pl = jdx & 3;
                const vec4<real> u = sup[i];
                const int ox = ((g - slx[i]) & 3) + 4 * pl;
                wxs[jdx] = (ox < PW) ? u.w * win<real, PW>(ox, u.x, a.ws) : (real)0;
            }
        }
        __syncthreads();
        // software pipeline: the next particle's weights and offsets are read before this
        // particle's writes (they are read-only here, so the order is free)
        const int* metaw = reinterpret_cast<const int*>(meta) + wave;
        int mk = metaw[0];
        real wx4[4], wy[NPASS], wz[NPASS];
        {
            const vec4<real> w4 = *reinterpret_cast<const vec4<real>*>(wxs + wave * 4);
            wx4[0] = w4.x;
            wx4[1] = w4.y;
            wx4[2] = w4.z;
            wx4[3] = w4.w;
#pragma unroll
            for (int ps = 0; ps < NPASS; ++ps) {
                wy[ps] = wyzs[oy2[ps]];
                wz[ps] = wyzs[oz2[ps]];
            }
        }
        for (int i = 0; i < cnt; ++i) {
            const int base = mk;
            real wyz[NPASS], wx[NPL];
#pragma unroll
            for (int ps = 0; ps < NPASS; ++ps) wyz[ps] = wy[ps] * wz[ps];
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) wx[pl] = wx4[pl];
            real cur[NPL][NPASS];
            int at[NPL][NPASS];
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
                for (int ps = 0; ps < NPASS; ++ps) {
                    at[pl][ps] = (DUMMY || has[ps]) ? base + off[pl][ps] : sinkb;
                    cur[pl][ps] = *reinterpret_cast<const real*>(hb + at[pl][ps]);
                }
            {
                const int in = min(i + 1, cnt - 1);
                mk = metaw[4 * in];
                const vec4<real> w4 = *reinterpret_cast<const vec4<real>*>(wxs + in * 16 + wave * 4);
                wx4[0] = w4.x;
                wx4[1] = w4.y;
                wx4[2] = w4.z;
                wx4[3] = w4.w;
                const real* wp = wyzs + in * NW;
#pragma unroll
                for (int ps = 0; ps < NPASS; ++ps) {
                    wy[ps] = wp[oy2[ps]];
                    wz[ps] = wp[oz2[ps]];
                }
            }
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
                for (int ps = 0; ps < NPASS; ++ps)
                    *reinterpret_cast<real*>(hb + at[pl][ps]) = cur[pl][ps] + wx[pl] * wyz[ps];
        }
    }
    __syncthreads();
    // add the block into the grid: each item is one (y, z) column of the block and a run of
    // up to kHaloILP x planes, whose atomic adds are in flight together (only nodes some
    // window reached are touched)
    const int nch = (HX + kHaloILP - 1) / kHaloILP;
    const size_t plane = (size_t)a.I[1] * a.I[2];
    for (int it = threadIdx.x; it < HYZ * nch; it += kSpreadThreads) {
        const int c = it / HYZ, k = it - c * HYZ;
        const int ly = k / HZ, lz = k - ly * HZ;
        const int gz = z0 - HW + lz;
        if (gz < 0 || gz >= a.I[2]) continue;
        const size_t colyz = (size_t)wrap_once(y0 - HW + ly, a.I[1]) * a.I[2] + gz;
        real v[kHaloILP];
        size_t at[kHaloILP];
#pragma unroll
        for (int j = 0; j < kHaloILP; ++j) {
            const int lx = c * kHaloILP + j;
            v[j] = (lx < HX) ? halo[lx * HYZ + k] : (real)0;
            at[j] = (size_t)wrap_once(x0 - HW + lx, a.I[0]) * plane + colyz;
        }
        if (a.phase < 0) {
#pragma unroll
            for (int j = 0; j < kHaloILP; ++j)
                if (v[j] != (real)0) atomicAdd(a.grid + at[j], v[j]);
        } else {
            // no other block of this colour touches these nodes, and within the block each
            // node has one (y, z) column and one x plane
            real old[kHaloILP];
#pragma unroll
            for (int j = 0; j < kHaloILP; ++j) old[j] = v[j] != (real)0 ? a.grid[at[j]] : (real)0;
#pragma unroll
            for (int j = 0; j < kHaloILP; ++j)
                if (v[j] != (real)0) a.grid[at[j]] = old[j] + v[j];
        }
    }
}
};

// zero planes [zlo, zlo + 2 span2) of every (x, y) line of the real grid, one wave per
// line (the other planes are never read or written)
template <typename real>
struct ZeroBandK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, real* __restrict__ grid, int nlines, int Izs, int zlo, int span2) {
    struct alignas(2 * sizeof(real)) pair { real a, b; };
    const int lane = threadIdx.x & 63;
    for (int line = gpos.bid * 4 + (threadIdx.x >> 6); line < nlines; line += gpos.nb * 4) {
        pair* row = reinterpret_cast<pair*>(grid + (size_t)line * Izs + zlo);
        for (int c = lane; c < span2; c += 64) row[c] = pair{0, 0};
    }
}
};

template <typename real>
struct GatherArgs {
    const int4* gp;
    const vec4<real>* up;
    const int* tstart;
    const real* grid;
    vec4<real>* part;  // mid part of each particle: phi, grad
    int I[3];
    int B[3];
    int nt[3];
    int ntiles;
    WinShape<real> ws;
    real dcoef[3];  // the derivative factors of win_d per direction
    real vol;       // h_x h_y h_z
};

constexpr int kGatherChunk = 256;  // particles sorted and dealt to the lanes at a time (the block size)

template <typename real, int PW>
struct GatherK {
    static constexpr int kThreads = kGatherChunk;
    __device__ static void run(GridPos gpos, const GatherArgs<real>& a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real* halo = reinterpret_cast<real*>(smem_raw);
    const int t = xcd_logical(a.ntiles, gpos);
    if (t < 0) return;
    const int beg = a.tstart[t * kMidSub], end = a.tstart[(t + 1) * kMidSub];
    if (beg == end) return;
    constexpr int HW = (PW - 1) / 2;
    const int tz = t % a.nt[2], ty = (t / a.nt[2]) % a.nt[1], tx = t / (a.nt[2] * a.nt[1]);
    const int x0 = tx * a.B[0], y0 = ty * a.B[1], z0 = tz * a.B[2];
    const int HX = a.B[0] + PW - 1, HY = a.B[1] + PW - 1, HZ = a.B[2] + PW - 1;
    const int HYZ = HY * HZ;
    // load the tile plus halo: each item is one (y, z) column of the block and a run of
    // up to kHaloILP x planes, whose loads are all in flight together
    const int nch = (HX + kHaloILP - 1) / kHaloILP;
    const size_t plane = (size_t)a.I[1] * a.I[2];
    for (int it = threadIdx.x; it < HYZ * nch; it += kThreads) {
        const int c = it / HYZ, k = it - c * HYZ;
        const int ly = k / HZ, lz = k - ly * HZ;
        const int gz = z0 - HW + lz;
        const bool zin = gz >= 0 && gz < a.I[2];
        const size_t colyz = (size_t)wrap_once(y0 - HW + ly, a.I[1]) * a.I[2] + (zin ? gz : 0);
        real v[kHaloILP];
#pragma unroll
        for (int j = 0; j < kHaloILP; ++j) {
            const int lx = c * kHaloILP + j;
            v[j] = (zin && lx < HX) ? a.grid[(size_t)wrap_once(x0 - HW + lx, a.I[0]) * plane + colyz] : (real)0;
        }
#pragma unroll
        for (int j = 0; j < kHaloILP; ++j) {
            const int lx = c * kHaloILP + j;
            if (lx < HX) halo[lx * HYZ + k] = v[j];
        }
    }
    // Lanes and LDS banks: a lane reads the rows of its particle's window at the window
    // corner plus offsets that are the same in every lane (mostly paired dword reads), so
    // two lanes collide in a bank when their corners are within one of each other mod 64.
    // Each chunk of up to 256 particles is counting-sorted by corner mod 64 and dealt to
    // the lanes so that each half-wave holds increasing residues about two apart.
    __shared__ int rcount[64], rstart[64], order[kGatherChunk];
    for (int c0 = beg; c0 < end; c0 += kGatherChunk) {
        const int cnt = min(kGatherChunk, end - c0);
        if (threadIdx.x < 64) rcount[threadIdx.x] = 0;
        __syncthreads();
        int res = 0, rank = 0;
        if ((int)threadIdx.x < cnt) {
            const int4 g = a.gp[c0 + threadIdx.x];
            res = (((g.x - x0) * HY + (g.y - y0)) * HZ + (g.z - z0)) & 63;
            rank = atomicAdd(&rcount[res], 1);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            int v = rcount[threadIdx.x];
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(v, o, 64);
                if ((int)threadIdx.x >= o) v += u;
            }
            rstart[threadIdx.x] = v - rcount[threadIdx.x];
        }
        __syncthreads();
        if ((int)threadIdx.x < cnt) order[rstart[res] + rank] = threadIdx.x;
        __syncthreads();
        // wave w takes sorted positions w + 4 j; lane l its j = 2 (l mod 32) + l / 32, so the
        // residues in each half-wave are about two apart (paired reads then rarely share a
        // bank in either half-wave)
        const int lane = threadIdx.x & 63;
        const int k = (((lane & 31) << 1) | (lane >> 5)) * 4 + (threadIdx.x >> 6);  // sorted position
        if (k < cnt) {
        const int p = c0 + order[k];
        const int4 g = a.gp[p];
        const vec4<real> u = a.up[p];
        real wy[PW], dwy[PW], wz[PW], dwz[PW];
        if (a.ws.kind == kWinPoly) {
            win_poly_all<real, PW>(u.y, a.ws, a.dcoef[1], wy, dwy);
            win_poly_all<real, PW>(u.z, a.ws, a.dcoef[2], wz, dwz);
        } else {
#pragma unroll
            for (int o = 0; o < PW; ++o) {
                win_d<real, PW>(o, u.y, a.ws, a.dcoef[1], wy[o], dwy[o]);
                win_d<real, PW>(o, u.z, a.ws, a.dcoef[2], wz[o], dwz[o]);
            }
        }
        const int lx0 = g.x - x0, ly0 = g.y - y0, lz0 = g.z - z0;
        real phi = 0, gx = 0, gy = 0, gz = 0;
        for (int ox = 0; ox < PW; ++ox) {
            real wx, dwx;
            win_d<real, PW>(ox, u.x, a.ws, a.dcoef[0], wx, dwx);
            real s0 = 0, s1 = 0, s2 = 0;  // sum_y wy * (sum_z wz u), sum_y dwy * (...), sum_y wy * (sum_z dwz u)
#pragma unroll
            for (int oy = 0; oy < PW; ++oy) {
                const real* row = halo + ((lx0 + ox) * HY + (ly0 + oy)) * HZ + lz0;
                real c0 = 0, c1 = 0;
#pragma unroll
                for (int oz = 0; oz < PW; ++oz) {
                    const real v = row[oz];
                    c0 += wz[oz] * v;
                    c1 += dwz[oz] * v;
                }
                s0 += wy[oy] * c0;
                s1 += dwy[oy] * c0;
                s2 += wy[oy] * c1;
            }
            phi += wx * s0;
            gx += dwx * s0;
            gy += wx * s1;
            gz += wx * s2;
        }
        const int i = g.w;
        a.part[i] = vec4<real>{a.vol * phi, a.vol * gx, a.vol * gy, a.vol * gz};
        }
        __syncthreads();  // the next chunk reuses rcount and order
    }
}
};

template <typename real, int PW>
hipError_t spread_gather_pw(Plan& p, bool spread) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int ntiles = r.ntile[0] * r.ntile[1] * r.ntile[2];
    const int HW = (PW - 1) / 2;
    const bool es = r.window == SOG_WINDOW_ES;
    const bool poly = r.window == SOG_WINDOW_KB;
    WinShape<real> shape;
    shape.S = (real)r.S;
    shape.inv_hw2 = (real)(HW > 0 ? 1.0 / ((double)HW * HW) : 0.0);
    shape.beta = (real)r.beta;
    shape.inv_a = (real)(2.0 / PW);
    shape.poly = (const real*)ws.wpoly;
    shape.kind = poly ? kWinPoly : (es ? kWinES : kWinGauss);
    shape.nu = window_poly_row(r.nu) - 1;  // the padded degree of the table
    if (spread) {
        SpreadArgs<real> a;
        a.gp = (const int4*)ws.mid_g;
        a.up = (const vec4<real>*)ws.mid_u;
        a.tstart = ws.tile_start;
        a.nodes = ws.spread_nodes;
        a.grid = (real*)ws.grid;
        a.I[0] = r.I[0]; a.I[1] = r.I[1]; a.I[2] = r.Izs;
        for (int d = 0; d < 3; ++d) { a.B[d] = r.B[d]; a.nt[d] = r.ntile[d]; }
        a.ntiles = ntiles;
        a.ws = shape;
        const size_t lds = spread_lds_bytes(sizeof(real), PW, r.B[0], r.B[1], r.B[2]);
        if (lds > tile_lds_budget(PW, sizeof(real))) return hipErrorInvalidConfiguration;
        const int nlines = r.I[0] * r.I[1];
        hipError_t e = launch<ZeroBandK<real>>(p, std::min((nlines + 3) / 4, 16384), 0, (real*)ws.grid, nlines, r.Izs,
                                               r.zband[0], (r.zband[1] - r.zband[0]) / 2);
        if (e != hipSuccess) return e;
        a.phase = -1;
        for (int d = 0; d < 3; ++d) a.pfirst[d] = a.pstep[d] = a.pcount[d] = 0;
        if (!r.deterministic)
            return r.spread_dummy ? launch<SpreadK<real, PW, true>>(p, xcd_grid(ntiles), lds, a)
                                  : launch<SpreadK<real, PW, false>>(p, xcd_grid(ntiles), lds, a);
        // colour by colour (tile_colour), in a fixed order; one launch over each colour's tiles
        const int nphase = r.dcol_n[0] * r.dcol_n[1] * r.dcol_n[2];
        for (int ph = 0; ph < nphase; ++ph) {
            const int col[3] = {ph / (r.dcol_n[1] * r.dcol_n[2]), (ph / r.dcol_n[2]) % r.dcol_n[1], ph % r.dcol_n[2]};
            for (int d = 0; d < 3; ++d) {
                const int m = r.dcol_m[d], qq = r.dcol_q[d], c = col[d];
                if (d < 2 && c >= m) {  // a tile after the whole runs: a colour of its own
                    a.pfirst[d] = qq * m + (c - m);
                    a.pstep[d] = 1;
                    a.pcount[d] = 1;
                } else {
                    a.pfirst[d] = c;
                    a.pstep[d] = m;
                    a.pcount[d] = d < 2 ? qq : (r.ntile[d] - c + m - 1) / m;
                }
            }
            const int cnt = a.pcount[0] * a.pcount[1] * a.pcount[2];
            if (cnt == 0) continue;
            a.phase = ph;
            e = r.spread_dummy ? launch<SpreadK<real, PW, true>>(p, xcd_grid(cnt), lds, a)
                               : launch<SpreadK<real, PW, false>>(p, xcd_grid(cnt), lds, a);
            if (e != hipSuccess) return e;
        }
        return e;
    } else {
        GatherArgs<real> a;
        a.gp = (const int4*)ws.mid_g;
        a.up = (const vec4<real>*)ws.mid_u;
        a.tstart = ws.tile_start;
        a.grid = (const real*)ws.grid;
        a.part = (vec4<real>*)ws.parts + r.n;
        a.I[0] = r.I[0]; a.I[1] = r.I[1]; a.I[2] = r.Izs;
        for (int d = 0; d < 3; ++d) {
            a.B[d] = r.B[d];
            a.nt[d] = r.ntile[d];
            a.dcoef[d] = poly ? (real)(1.0 / r.h[d])
                              : es ? (real)(4.0 * r.beta / ((double)PW * PW * r.h[d]))
                                   : (real)(2.0 * r.S / ((double)HW * HW * r.h[d]));
        }
        a.ntiles = ntiles;
        a.ws = shape;
        a.vol = (real)(r.h[0] * r.h[1] * r.h[2]);
        size_t lds = (size_t)(r.B[0] + PW - 1) * (r.B[1] + PW - 1) * (r.B[2] + PW - 1) * sizeof(real);
        // plus the static residue sort: 128 + kGatherChunk ints
        if (lds + (128 + kGatherChunk) * sizeof(int) > tile_lds_budget(PW, sizeof(real))) return hipErrorInvalidConfiguration;
        return launch<GatherK<real, PW>>(p, xcd_grid(ntiles), lds, a);
    }
}

template <typename real>
hipError_t spread_gather(Plan& p, bool spread) {
    switch (p.r.Pw) {
        case 3: return spread_gather_pw<real, 3>(p, spread);
        case 5: return spread_gather_pw<real, 5>(p, spread);
        case 7: return spread_gather_pw<real, 7>(p, spread);
        case 9: return spread_gather_pw<real, 9>(p, spread);
        case 11: return spread_gather_pw<real, 11>(p, spread);
        case 13: return spread_gather_pw<real, 13>(p, spread);
        case 15: return spread_gather_pw<real, 15>(p, spread);
        default: return hipErrorInvalidValue;
    }
}

MidGeom mid_geom(const Resolved& r) {
    MidGeom g;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = r.L[d];
        g.h[d] = r.h[d];
        g.B[d] = r.B[d];
        g.nt[d] = r.ntile[d];
    }
    g.Lzs = r.Lzs;
    g.I[0] = r.I[0];
    g.I[1] = r.I[1];
    g.I[2] = r.Izs;
    g.HW = (r.Pw - 1) / 2;
    g.zlo = r.zband[0];
    g.zhi = r.zband[1];
    return g;
}

template <typename real>
hipError_t run_mid_prepare(Plan& p, const double* x, const double* q) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int n = (int)r.n;
    MidGeom g = mid_geom(r);
    const int ntiles = r.ntile[0] * r.ntile[1] * r.ntile[2];
    const int blocks = std::min((n + 255) / 256, 8192);
    const int nbins = ntiles * kMidSub;
    hipError_t e = launch_fill_int(p, ws.tile_start, 0, (int64_t)nbins + 1);
    if (e == hipSuccess) e = launch<MidKeyK>(p, blocks, 0, x, n, g, (int2*)ws.key2, ws.tile_start);
    if (e == hipSuccess) e = launch_exclusive_scan(p, ws.tile_start, nbins + 1, ws.scan_tmp2);
    if (e == hipSuccess && r.deterministic)
        e = launch_canonical_ranks(p, ws.key2, true, n, ws.tile_start, nbins, nullptr, ws.det_idx2, nullptr);
    if (e == hipSuccess)
        e = launch<MidPackK<real>>(p, blocks, 0, x, q, n, g, (const int2*)ws.key2, (const int*)ws.tile_start,
                                   (int4*)ws.mid_g, (vec4<real>*)ws.mid_u);
    return e;
}

}  // namespace

hipError_t launch_fft_mid(Plan& p);  // k_fft.hip

hipError_t launch_mid(Plan& p, const double* x, const double* q, int stages) {
    const bool f64 = p.r.prec == SOG_PREC_FP64;
    hipError_t e = hipSuccess;
    if (stages & 1) {
        int t = timer_id(p, "mid_sort");
        timer_begin(p, t);
        e = f64 ? run_mid_prepare<double>(p, x, q) : run_mid_prepare<float>(p, x, q);
        timer_end(p, t);
        if (e != hipSuccess) return e;
        t = timer_id(p, "mid_spread");
        timer_begin(p, t);
        e = f64 ? spread_gather<double>(p, true) : spread_gather<float>(p, true);
        timer_end(p, t);
        if (e != hipSuccess) return e;
    }
    if (stages & 2) {
        e = launch_fft_mid(p);
        if (e != hipSuccess) return e;
        const int t = timer_id(p, "mid_gather");
        timer_begin(p, t);
        e = f64 ? spread_gather<double>(p, false) : spread_gather<float>(p, false);
        timer_end(p, t);
    }
    return e;
}

}  // namespace sog
