// Mid-range Fourier spectral solver, gridding and gathering (Alg. al::mid steps 1 and 5,
// eqs. gridding and Phiconv) with the Gaussian window of eq. GS.
//
// Grid: nodes X_a = -Lx/2 + a h_x (a < I_x), likewise y, Z_c = -L_z*/2 + c h_z (c < I_z*),
// stored z-fastest: grid[(a * I_y + b) * I_z* + c].  Window on P_w nodes around the
// nearest node, W(d) = exp(-S (d/H)^2) for |d| <= H = (P_w - 1) h / 2, else 0.
//
// Gridding is output-stationary: the grid is cut into tiles of B_x x B_y x B_z nodes; one
// workgroup owns a tile, accumulates into it in LDS every particle whose window touches
// it (lists built per call by a counting sort), and writes the tile once.  No global
// atomics and no clearing pass: every node is written exactly once.
// Gathering: one workgroup per tile loads the tile plus a (P_w - 1) halo into LDS and
// evaluates Phi and grad Phi for the particles whose nearest node lies in the tile.
#include "device_common.hpp"

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
            a[d] = min(max(k, g.HW), g.I[2] - 1 - g.HW);  // only invalid input hits the clamp
            if (k != a[d]) u[d] = 0.0;
        }
    }
}

__global__ void k_mid_key(const double* __restrict__ x, int n, MidGeom g, int* __restrict__ key) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int a[3];
        double u[3];
        grid_point(g, x[3 * i], x[3 * i + 1], x[3 * i + 2], a, u);
        key[i] = ((a[0] / g.B[0]) * g.nt[1] + a[1] / g.B[1]) * g.nt[2] + a[2] / g.B[2];
    }
}

template <typename real>
__global__ void k_mid_pack(const double* __restrict__ x, const double* __restrict__ q, int n, MidGeom g,
                           const int* __restrict__ perm, int4* __restrict__ gp, vec4<real>* __restrict__ up) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        int i = perm[p];
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

// distinct tiles touched along one direction by the window nodes a0-HW .. a0+HW
__device__ __forceinline__ int touched(int a0, int HW, int I, int B, bool periodic, int* out) {
    int cnt = 0;
    for (int o = -HW; o <= HW; ++o) {
        int gi = a0 + o;
        if (periodic) gi = imod(gi, I);
        else if (gi < 0 || gi >= I) continue;
        int t = gi / B;
        bool seen = false;
        for (int k = 0; k < cnt; ++k) seen |= (out[k] == t);
        if (!seen && cnt < 8) out[cnt++] = t;
    }
    return cnt;
}

__global__ void k_dup(const int4* __restrict__ gp, int n, MidGeom g, int* __restrict__ count, const int* __restrict__ start,
                      int* __restrict__ cursor, int* __restrict__ list, int cap, int fill) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        int4 a = gp[p];
        int tx[8], ty[8], tz[8];
        int nx = touched(a.x, g.HW, g.I[0], g.B[0], true, tx);
        int ny = touched(a.y, g.HW, g.I[1], g.B[1], true, ty);
        int nz = touched(a.z, g.HW, g.I[2], g.B[2], false, tz);
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j)
                for (int k = 0; k < nz; ++k) {
                    int t = (tx[i] * g.nt[1] + ty[j]) * g.nt[2] + tz[k];
                    if (!fill) {
                        atomicAdd(&count[t], 1);
                    } else {
                        int pos = start[t] + atomicAdd(&cursor[t], 1);
                        if (pos < cap) list[pos] = p;
                    }
                }
    }
}

template <typename real>
struct SpreadArgs {
    const int4* gp;
    const vec4<real>* up;
    const int* dstart;
    const int* dlist;
    int cap;  // entries in dlist
    real* grid;
    int I[3];
    int B[3];
    int nt[3];
    int ntiles;
    real S;
    real inv_hw2;  // 1 / HW^2
};

// window weights on the P_w nodes: W((node - particle) h) with node - particle = o - HW - u
template <typename real, int PW>
__device__ __forceinline__ real win(int o, real u, real S, real inv_hw2) {
    constexpr int HW = (PW - 1) / 2;
    const real d = (real)(o - HW) - u;
    const real r2 = d * d * inv_hw2;
    return (r2 <= (real)1) ? dexp(-S * r2) : (real)0;
}

constexpr int kSpreadThreads = 128;

template <typename real, int PW>
__global__ __launch_bounds__(kSpreadThreads) void k_spread(SpreadArgs<real> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real* tile = reinterpret_cast<real*>(smem_raw);
    const int T = a.B[0] * a.B[1] * a.B[2];
    real* wts = tile + T;  // kSpreadThreads x 2 PW
    const int t = xcd_logical_block(a.ntiles);
    if (t < 0) return;
    const int tz = t % a.nt[2], ty = (t / a.nt[2]) % a.nt[1], tx = t / (a.nt[2] * a.nt[1]);
    const int x0 = tx * a.B[0], y0 = ty * a.B[1], z0 = tz * a.B[2];
    const int ex = min(a.B[0], a.I[0] - x0), ey = min(a.B[1], a.I[1] - y0), ez = min(a.B[2], a.I[2] - z0);
    for (int k = threadIdx.x; k < T; k += blockDim.x) tile[k] = 0;
    __syncthreads();
    constexpr int HW = (PW - 1) / 2;
    real* myw = wts + threadIdx.x * 2 * PW;
    const int beg = min(a.dstart[t], a.cap), end = min(a.dstart[t + 1], a.cap);
    for (int e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const int p = a.dlist[e];
        const int4 g = a.gp[p];
        const vec4<real> u = a.up[p];
        real wz[PW];
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            myw[o] = u.w * win<real, PW>(o, u.x, a.S, a.inv_hw2);
            myw[PW + o] = win<real, PW>(o, u.y, a.S, a.inv_hw2);
            wz[o] = win<real, PW>(o, u.z, a.S, a.inv_hw2);
        }
        const int sx0 = g.x - HW, sy0 = g.y - HW, sz = g.z - HW;
        const int zlo = max(sz, z0), zhi = min(sz + PW, z0 + ez);
        if (zlo >= zhi) continue;
        for (int ix = -1; ix <= 1; ++ix) {
            const int sx = sx0 + ix * a.I[0];
            const int xlo = max(sx, x0), xhi = min(sx + PW, x0 + ex);
            if (xlo >= xhi) continue;
            for (int iy = -1; iy <= 1; ++iy) {
                const int sy = sy0 + iy * a.I[1];
                const int ylo = max(sy, y0), yhi = min(sy + PW, y0 + ey);
                if (ylo >= yhi) continue;
                for (int gx = xlo; gx < xhi; ++gx) {
                    const real wx = myw[gx - sx];
                    for (int gy = ylo; gy < yhi; ++gy) {
                        const real wxy = wx * myw[PW + gy - sy];
                        real* row = tile + ((gx - x0) * a.B[1] + (gy - y0)) * a.B[2] - z0;
#pragma unroll
                        for (int o = 0; o < PW; ++o) {
                            const int gz = sz + o;
                            if (gz >= zlo && gz < zhi) atomicAdd(row + gz, wxy * wz[o]);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < T; k += blockDim.x) {
        const int lz = k % a.B[2], ly = (k / a.B[2]) % a.B[1], lx = k / (a.B[2] * a.B[1]);
        if (lx < ex && ly < ey && lz < ez)
            a.grid[((size_t)(x0 + lx) * a.I[1] + (y0 + ly)) * a.I[2] + (z0 + lz)] = tile[k];
    }
}

template <typename real>
struct GatherArgs {
    const int4* gp;
    const vec4<real>* up;
    const int* tstart;
    const real* grid;
    real* pphi;   // part 1 (n)
    real* pgrad;  // part 1 (n x 3)
    int I[3];
    int B[3];
    int nt[3];
    int ntiles;
    real S;
    real inv_hw2;
    real dcoef[3];  // 2 S / (HW^2 h_d): d/dx_particle of W is dcoef * (node - particle in h) * W
    real vol;       // h_x h_y h_z
};

template <typename real, int PW>
__global__ __launch_bounds__(256) void k_gather(GatherArgs<real> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real* halo = reinterpret_cast<real*>(smem_raw);
    const int t = xcd_logical_block(a.ntiles);
    if (t < 0) return;
    const int beg = a.tstart[t], end = a.tstart[t + 1];
    if (beg == end) return;
    constexpr int HW = (PW - 1) / 2;
    const int tz = t % a.nt[2], ty = (t / a.nt[2]) % a.nt[1], tx = t / (a.nt[2] * a.nt[1]);
    const int x0 = tx * a.B[0], y0 = ty * a.B[1], z0 = tz * a.B[2];
    const int HX = a.B[0] + PW - 1, HY = a.B[1] + PW - 1, HZ = a.B[2] + PW - 1;
    const int tot = HX * HY * HZ;
    for (int k = threadIdx.x; k < tot; k += blockDim.x) {
        const int lz = k % HZ, ly = (k / HZ) % HY, lx = k / (HZ * HY);
        const int gx = imod(x0 - HW + lx, a.I[0]);
        const int gy = imod(y0 - HW + ly, a.I[1]);
        const int gz = z0 - HW + lz;
        halo[k] = (gz >= 0 && gz < a.I[2]) ? a.grid[((size_t)gx * a.I[1] + gy) * a.I[2] + gz] : (real)0;
    }
    __syncthreads();
    for (int p = beg + threadIdx.x; p < end; p += blockDim.x) {
        const int4 g = a.gp[p];
        const vec4<real> u = a.up[p];
        real wy[PW], dwy[PW], wz[PW], dwz[PW];
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            wy[o] = win<real, PW>(o, u.y, a.S, a.inv_hw2);
            dwy[o] = a.dcoef[1] * ((real)(o - HW) - u.y) * wy[o];
            wz[o] = win<real, PW>(o, u.z, a.S, a.inv_hw2);
            dwz[o] = a.dcoef[2] * ((real)(o - HW) - u.z) * wz[o];
        }
        const int lx0 = g.x - x0, ly0 = g.y - y0, lz0 = g.z - z0;
        real phi = 0, gx = 0, gy = 0, gz = 0;
        for (int ox = 0; ox < PW; ++ox) {
            const real wx = win<real, PW>(ox, u.x, a.S, a.inv_hw2);
            const real dwx = a.dcoef[0] * ((real)(ox - HW) - u.x) * wx;
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
        a.pphi[i] = a.vol * phi;
        a.pgrad[3 * i] = a.vol * gx;
        a.pgrad[3 * i + 1] = a.vol * gy;
        a.pgrad[3 * i + 2] = a.vol * gz;
    }
}

template <typename real, int PW>
hipError_t spread_gather_pw(Plan& p, bool spread) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int ntiles = r.ntile[0] * r.ntile[1] * r.ntile[2];
    const int HW = (PW - 1) / 2;
    const real S = (real)r.S;
    const real inv_hw2 = (real)(1.0 / ((double)HW * HW));
    if (spread) {
        SpreadArgs<real> a;
        a.gp = (const int4*)ws.mid_g;
        a.up = (const vec4<real>*)ws.mid_u;
        a.dstart = ws.dup_start;
        a.dlist = ws.dup_list;
        a.cap = (int)std::min<int64_t>((int64_t)r.n * r.max_dup, INT32_MAX);
        a.grid = (real*)ws.grid;
        a.I[0] = r.I[0]; a.I[1] = r.I[1]; a.I[2] = r.Izs;
        for (int d = 0; d < 3; ++d) { a.B[d] = r.B[d]; a.nt[d] = r.ntile[d]; }
        a.ntiles = ntiles;
        a.S = S;
        a.inv_hw2 = inv_hw2;
        size_t lds = ((size_t)r.B[0] * r.B[1] * r.B[2] + (size_t)kSpreadThreads * 2 * PW) * sizeof(real);
        if (lds > 65536) return hipErrorInvalidConfiguration;
        k_spread<real, PW><<<xcd_grid(ntiles), kSpreadThreads, lds, p.stream>>>(a);
    } else {
        GatherArgs<real> a;
        a.gp = (const int4*)ws.mid_g;
        a.up = (const vec4<real>*)ws.mid_u;
        a.tstart = ws.tile_start;
        a.grid = (const real*)ws.grid;
        a.pphi = (real*)ws.parts_phi + r.n;
        a.pgrad = (real*)ws.parts_grad + 3 * r.n;
        a.I[0] = r.I[0]; a.I[1] = r.I[1]; a.I[2] = r.Izs;
        for (int d = 0; d < 3; ++d) {
            a.B[d] = r.B[d];
            a.nt[d] = r.ntile[d];
            a.dcoef[d] = (real)(2.0 * r.S / ((double)HW * HW * r.h[d]));
        }
        a.ntiles = ntiles;
        a.S = S;
        a.inv_hw2 = inv_hw2;
        a.vol = (real)(r.h[0] * r.h[1] * r.h[2]);
        size_t lds = (size_t)(r.B[0] + PW - 1) * (r.B[1] + PW - 1) * (r.B[2] + PW - 1) * sizeof(real);
        if (lds > 65536) return hipErrorInvalidConfiguration;
        k_gather<real, PW><<<xcd_grid(ntiles), 256, lds, p.stream>>>(a);
    }
    return hipGetLastError();
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
    k_mid_key<<<blocks, 256, 0, p.stream>>>(x, n, g, ws.key);
    hipError_t e = launch_counting_sort(p, ws.key, n, ntiles, ws.tile_start, ws.tile_cursor, ws.perm);
    if (e != hipSuccess) return e;
    k_mid_pack<real><<<blocks, 256, 0, p.stream>>>(x, q, n, g, ws.perm, (int4*)ws.mid_g, (vec4<real>*)ws.mid_u);
    // window lists: count, scan, fill
    e = launch_fill_int(ws.dup_start, 0, (int64_t)ntiles + 1, p.stream);
    if (e != hipSuccess) return e;
    e = launch_fill_int(ws.dup_cursor, 0, ntiles, p.stream);
    if (e != hipSuccess) return e;
    k_dup<<<blocks, 256, 0, p.stream>>>((const int4*)ws.mid_g, n, g, ws.dup_start, nullptr, nullptr, nullptr, 0, 0);
    e = launch_exclusive_scan(p, ws.dup_start, ntiles + 1);
    if (e != hipSuccess) return e;
    k_dup<<<blocks, 256, 0, p.stream>>>((const int4*)ws.mid_g, n, g, nullptr, ws.dup_start, ws.dup_cursor, ws.dup_list,
                                         (int)std::min<int64_t>((int64_t)n * r.max_dup, INT32_MAX), 1);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fft_mid(Plan& p);  // k_fft.hip

hipError_t launch_mid(Plan& p, const double* x, const double* q) {
    const bool f64 = p.r.prec == SOG_PREC_FP64;
    int t = timer_id(p, "mid_sort");
    timer_begin(p, t);
    hipError_t e = f64 ? run_mid_prepare<double>(p, x, q) : run_mid_prepare<float>(p, x, q);
    timer_end(p, t);
    if (e != hipSuccess) return e;
    t = timer_id(p, "mid_spread");
    timer_begin(p, t);
    e = f64 ? spread_gather<double>(p, true) : spread_gather<float>(p, true);
    timer_end(p, t);
    if (e != hipSuccess) return e;
    e = launch_fft_mid(p);
    if (e != hipSuccess) return e;
    t = timer_id(p, "mid_gather");
    timer_begin(p, t);
    e = f64 ? spread_gather<double>(p, false) : spread_gather<float>(p, false);
    timer_end(p, t);
    return e;
}

}  // namespace sog
