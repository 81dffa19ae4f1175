// Long range, Fourier-Chebyshev solver with FFTs (Alg. al::long, Sec. 3.3): for flat
// boxes the direct form needs O(A / s_{m+1}^2) modes per particle, so the x,y Fourier
// sums go through a 2D Gaussian-window grid (eq. Chebygrid) and 2D FFTs, exactly as the
// mid range does in 3D, while z stays in the Chebyshev basis:
//   S2(g, n)  = sum_j q_j W2(g - r_j) T_n(t_j)                       (gridding)
//   Shat2     = fft2(S2(., n)) for each n
//   uhat(k,n) = sum_n' Kt(k)[n][n'] / What2(k)^2 / (I2x I2y) Shat2(k, n')   (scaling)
//   u(., n)   = ifft2(uhat(., n))                                      (unnormalised)
//   Phi^long_i = h_x h_y sum_g W2(r_i - g) sum_n T_n(t_i) u(g, n)      (gathering)
// Kt = C^T K C is the same Chebyshev-basis z kernel as the direct form.  Gridding is
// output-stationary over 2D tiles that hold all P Chebyshev terms, gathering uses a
// halo tile, as in the mid range.
#include "device_common.hpp"

namespace sog {

hipError_t launch_fft_lines(Plan& p, void* data, const FFTFactors& f, const void* tw, int nlines, int ncols,
                            size_t outer_stride, size_t col_stride, size_t elem_stride, int sign, int W);

namespace {

struct L2Geom {
    double L[3];
    double h[2];
    int I[2];
    int B[2];
    int nt[2];
    int HW;
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

__global__ void k_l2_key(const double* __restrict__ x, int n, L2Geom g, int* __restrict__ key) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int a[2];
        double u[2];
        grid_point2(g, x[3 * i], x[3 * i + 1], a, u);
        key[i] = (a[0] / g.B[0]) * g.nt[1] + a[1] / g.B[1];
    }
}

template <typename real>
__global__ void k_l2_pack(const double* __restrict__ x, const double* __restrict__ q, int n, L2Geom g,
                          const int* __restrict__ perm, int4* __restrict__ gp, vec4<real>* __restrict__ up) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        int i = perm[p];
        int a[2];
        double u[2];
        grid_point2(g, x[3 * i], x[3 * i + 1], a, u);
        double zz = x[3 * i + 2], qq = q[i];
        if (!isfinite(zz)) zz = 0;
        if (!isfinite(qq)) qq = 0;
        double t = 2.0 * (zz - 0.5 * g.L[2]) / g.L[2];
        t = fmin(1.0, fmax(-1.0, t));
        gp[p] = make_int4(a[0], a[1], 0, i);
        vec4<real> v;
        v.x = (real)u[0];
        v.y = (real)u[1];
        v.z = (real)t;
        v.w = (real)qq;
        up[p] = v;
    }
}

__device__ __forceinline__ int touched2(int a0, int HW, int I, int B, int* out) {
    int cnt = 0;
    for (int o = -HW; o <= HW; ++o) {
        int t = imod(a0 + o, I) / B;
        bool seen = false;
        for (int k = 0; k < cnt; ++k) seen |= (out[k] == t);
        if (!seen && cnt < 8) out[cnt++] = t;
    }
    return cnt;
}

__global__ void k_l2_dup(const int4* __restrict__ gp, int n, L2Geom g, int* __restrict__ count,
                         const int* __restrict__ start, int* __restrict__ cursor, int* __restrict__ list, int cap,
                         int fill) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        int4 a = gp[p];
        int tx[8], ty[8];
        int nx = touched2(a.x, g.HW, g.I[0], g.B[0], tx);
        int ny = touched2(a.y, g.HW, g.I[1], g.B[1], ty);
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                int t = tx[i] * g.nt[1] + ty[j];
                if (!fill) {
                    atomicAdd(&count[t], 1);
                } else {
                    int pos = start[t] + atomicAdd(&cursor[t], 1);
                    if (pos < cap) list[pos] = p;
                }
            }
    }
}

template <typename real, int PW>
__device__ __forceinline__ real win2(int o, real u, real S, real inv_hw2) {
    constexpr int HW = (PW - 1) / 2;
    const real d = (real)(o - HW) - u;
    const real r2 = d * d * inv_hw2;
    return (r2 <= (real)1) ? dexp(-S * r2) : (real)0;
}

template <typename real>
struct L2SpreadArgs {
    const int4* gp;
    const vec4<real>* up;
    const int* dstart;
    const int* dlist;
    int cap;
    cpx<real>* grid;  // P x I2x x I2y
    int I[2], B[2], nt[2], ntiles, P;
    real S, inv_hw2;
};

constexpr int kL2Threads = 128;

template <typename real, int PW>
__global__ __launch_bounds__(kL2Threads) void k_l2_spread(L2SpreadArgs<real> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = a.P;
    real* tile = reinterpret_cast<real*>(smem_raw);  // B0 x B1 x P
    const int T = a.B[0] * a.B[1] * P;
    real* tn = tile + T;                              // kL2Threads x P
    const int t = xcd_logical_block(a.ntiles);
    if (t < 0) return;
    const int tx = t / a.nt[1], ty = t % a.nt[1];
    const int x0 = tx * a.B[0], y0 = ty * a.B[1];
    const int ex = min(a.B[0], a.I[0] - x0), ey = min(a.B[1], a.I[1] - y0);
    for (int k = threadIdx.x; k < T; k += blockDim.x) tile[k] = 0;
    __syncthreads();
    constexpr int HW = (PW - 1) / 2;
    real* mt = tn + threadIdx.x * P;
    const int beg = min(a.dstart[t], a.cap), end = min(a.dstart[t + 1], a.cap);
    for (int e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const int p = a.dlist[e];
        const int4 g = a.gp[p];
        const vec4<real> u = a.up[p];
        real wx[PW], wy[PW];
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            wx[o] = u.w * win2<real, PW>(o, u.x, a.S, a.inv_hw2);
            wy[o] = win2<real, PW>(o, u.y, a.S, a.inv_hw2);
        }
        real T0 = 1, T1 = u.z;
        mt[0] = 1;
        if (P > 1) mt[1] = u.z;
        for (int k = 2; k < P; ++k) {
            const real T2 = (real)2 * u.z * T1 - T0;
            mt[k] = T2;
            T0 = T1;
            T1 = T2;
        }
        for (int ix = -1; ix <= 1; ++ix) {
            const int sx = g.x - HW + ix * a.I[0];
            for (int iy = -1; iy <= 1; ++iy) {
                const int sy = g.y - HW + iy * a.I[1];
#pragma unroll
                for (int ox = 0; ox < PW; ++ox) {
                    const int gx = sx + ox;
                    if (gx < x0 || gx >= x0 + ex) continue;
#pragma unroll
                    for (int oy = 0; oy < PW; ++oy) {
                        const int gy = sy + oy;
                        if (gy < y0 || gy >= y0 + ey) continue;
                        const real w = wx[ox] * wy[oy];
                        real* cell = tile + ((gx - x0) * a.B[1] + (gy - y0)) * P;
                        for (int k = 0; k < P; ++k) atomicAdd(cell + k, w * mt[k]);
                    }
                }
            }
        }
    }
    __syncthreads();
    const size_t plane = (size_t)a.I[0] * a.I[1];
    for (int k = threadIdx.x; k < T; k += blockDim.x) {
        const int nn = k % P, ly = (k / P) % a.B[1], lx = k / (P * a.B[1]);
        if (lx < ex && ly < ey)
            a.grid[nn * plane + (size_t)(x0 + lx) * a.I[1] + (y0 + ly)] = cpx<real>{tile[k], 0};
    }
}

template <typename real>
__global__ void k_l2_scale(cpx<real>* __restrict__ grid, int I0, int I1, int P, const real* __restrict__ kt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<real>* v = reinterpret_cast<cpx<real>*>(smem_raw) + threadIdx.x * P;
    const int kp = blockIdx.x * blockDim.x + threadIdx.x;
    if (kp >= I0 * I1) return;
    const int ix = kp / I1, iy = kp % I1;
    const int jx = min(ix, I0 - ix), jy = min(iy, I1 - iy);
    const real* K = kt + ((size_t)jx * (I1 / 2 + 1) + jy) * P * P;
    const size_t plane = (size_t)I0 * I1;
    for (int k = 0; k < P; ++k) v[k] = grid[k * plane + kp];
    for (int nn = 0; nn < P; ++nn) {
        real sr = 0, si = 0;
        for (int e = 0; e < P; ++e) {
            sr += K[nn * P + e] * v[e].x;
            si += K[nn * P + e] * v[e].y;
        }
        grid[nn * plane + kp] = cpx<real>{sr, si};
    }
}

template <typename real>
struct L2GatherArgs {
    const int4* gp;
    const vec4<real>* up;
    const int* tstart;
    const cpx<real>* grid;
    vec4<real>* part;  // long part of each particle: phi, grad
    int I[2], B[2], nt[2], ntiles, P;
    real S, inv_hw2, dcoef[2], area, dzf;
};

template <typename real, int PW>
__global__ __launch_bounds__(64) void k_l2_gather(L2GatherArgs<real> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = a.P;
    constexpr int HW = (PW - 1) / 2;
    const int t = xcd_logical_block(a.ntiles);
    if (t < 0) return;
    const int beg = a.tstart[t], end = a.tstart[t + 1];
    if (beg == end) return;
    const int tx = t / a.nt[1], ty = t % a.nt[1];
    const int x0 = tx * a.B[0], y0 = ty * a.B[1];
    const int HX = a.B[0] + PW - 1, HY = a.B[1] + PW - 1;
    real* halo = reinterpret_cast<real*>(smem_raw);  // HX x HY x P
    real* tt = halo + HX * HY * P;                    // blockDim x 2P
    const size_t plane = (size_t)a.I[0] * a.I[1];
    for (int k = threadIdx.x; k < HX * HY * P; k += blockDim.x) {
        const int nn = k % P, ly = (k / P) % HY, lx = k / (P * HY);
        const int gx = imod(x0 - HW + lx, a.I[0]), gy = imod(y0 - HW + ly, a.I[1]);
        halo[k] = a.grid[nn * plane + (size_t)gx * a.I[1] + gy].x;
    }
    __syncthreads();
    real* Tt = tt + threadIdx.x * 2 * P;
    real* Td = Tt + P;
    for (int p = beg + threadIdx.x; p < end; p += blockDim.x) {
        const int4 g = a.gp[p];
        const vec4<real> u = a.up[p];
        {
            real T0 = 1, T1 = u.z, U0 = 1, U1 = 2 * u.z;
            Tt[0] = 1;
            Td[0] = 0;
            if (P > 1) { Tt[1] = u.z; Td[1] = 1; }
            for (int k = 2; k < P; ++k) {
                const real T2 = (real)2 * u.z * T1 - T0;
                Tt[k] = T2;
                Td[k] = (real)k * U1;
                const real U2 = (real)2 * u.z * U1 - U0;
                T0 = T1; T1 = T2;
                U0 = U1; U1 = U2;
            }
        }
        real wy[PW], dwy[PW];
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            wy[o] = win2<real, PW>(o, u.y, a.S, a.inv_hw2);
            dwy[o] = a.dcoef[1] * ((real)(o - HW) - u.y) * wy[o];
        }
        const int lx0 = g.x - x0, ly0 = g.y - y0;
        real phi = 0, gx = 0, gy = 0, gz = 0;
        for (int ox = 0; ox < PW; ++ox) {
            const real wx = win2<real, PW>(ox, u.x, a.S, a.inv_hw2);
            const real dwx = a.dcoef[0] * ((real)(ox - HW) - u.x) * wx;
            real s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int oy = 0; oy < PW; ++oy) {
                const real* cell = halo + ((lx0 + ox) * HY + (ly0 + oy)) * P;
                real c0 = 0, c1 = 0;
                for (int k = 0; k < P; ++k) {
                    c0 += Tt[k] * cell[k];
                    c1 += Td[k] * cell[k];
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
        a.part[i] = vec4<real>{a.area * phi, a.area * gx, a.area * gy, a.area * a.dzf * gz};
    }
}

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
        a.dstart = ws.l2_dup_start;
        a.dlist = ws.l2_dup_list;
        a.cap = (int)std::min<int64_t>((int64_t)r.n * r.max_dup2, INT32_MAX);
        a.grid = (cpx<real>*)ws.l2_grid;
        for (int d = 0; d < 2; ++d) { a.I[d] = r.I2[d]; a.B[d] = r.B2[d]; a.nt[d] = r.ntile2[d]; }
        a.ntiles = ntiles;
        a.P = r.P;
        a.S = (real)r.S2;
        a.inv_hw2 = inv_hw2;
        size_t lds = ((size_t)r.B2[0] * r.B2[1] * r.P + (size_t)kL2Threads * r.P) * sizeof(real);
        if (lds > 65536) return hipErrorInvalidConfiguration;
        k_l2_spread<real, PW><<<xcd_grid(ntiles), kL2Threads, lds, p.stream>>>(a);
    } else {
        L2GatherArgs<real> a;
        a.gp = (const int4*)ws.l2_g;
        a.up = (const vec4<real>*)ws.l2_u;
        a.tstart = ws.l2_tile_start;
        a.grid = (const cpx<real>*)ws.l2_grid;
        a.part = (vec4<real>*)ws.parts + 2 * r.n;
        for (int d = 0; d < 2; ++d) {
            a.I[d] = r.I2[d];
            a.B[d] = r.B2[d];
            a.nt[d] = r.ntile2[d];
            a.dcoef[d] = (real)(2.0 * r.S2 / ((double)HW * HW * r.h2[d]));
        }
        a.ntiles = ntiles;
        a.P = r.P;
        a.S = (real)r.S2;
        a.inv_hw2 = inv_hw2;
        a.area = (real)(r.h2[0] * r.h2[1]);
        a.dzf = (real)(2.0 / r.L[2]);
        size_t lds = ((size_t)(r.B2[0] + PW - 1) * (r.B2[1] + PW - 1) * r.P + 64 * 2 * (size_t)r.P) * sizeof(real);
        if (lds > 65536) return hipErrorInvalidConfiguration;
        k_l2_gather<real, PW><<<xcd_grid(ntiles), 64, lds, p.stream>>>(a);
    }
    return hipGetLastError();
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
    L2Geom g;
    for (int d = 0; d < 3; ++d) g.L[d] = r.L[d];
    for (int d = 0; d < 2; ++d) {
        g.h[d] = r.h2[d];
        g.I[d] = r.I2[d];
        g.B[d] = r.B2[d];
        g.nt[d] = r.ntile2[d];
    }
    g.HW = (r.Pw2 - 1) / 2;
    const int ntiles = r.ntile2[0] * r.ntile2[1];
    const int blocks = std::min((n + 255) / 256, 8192);
    int t = timer_id(p, "long2_sort");
    timer_begin(p, t);
    k_l2_key<<<blocks, 256, 0, p.stream>>>(x, n, g, ws.key);
    hipError_t e = launch_counting_sort(p, ws.key, n, ntiles, ws.l2_tile_start, ws.l2_tile_cursor, ws.perm);
    if (e != hipSuccess) return e;
    k_l2_pack<real><<<blocks, 256, 0, p.stream>>>(x, q, n, g, ws.perm, (int4*)ws.l2_g, (vec4<real>*)ws.l2_u);
    if ((e = launch_fill_int(ws.l2_dup_start, 0, (int64_t)ntiles + 1, p.stream)) != hipSuccess) return e;
    if ((e = launch_fill_int(ws.l2_dup_cursor, 0, ntiles, p.stream)) != hipSuccess) return e;
    k_l2_dup<<<blocks, 256, 0, p.stream>>>((const int4*)ws.l2_g, n, g, ws.l2_dup_start, nullptr, nullptr, nullptr, 0, 0);
    if ((e = launch_exclusive_scan(p, ws.l2_dup_start, ntiles + 1, ws.scan_tmp)) != hipSuccess) return e;
    k_l2_dup<<<blocks, 256, 0, p.stream>>>((const int4*)ws.l2_g, n, g, nullptr, ws.l2_dup_start, ws.l2_dup_cursor,
                                            ws.l2_dup_list, (int)std::min<int64_t>((int64_t)n * r.max_dup2, INT32_MAX), 1);
    timer_end(p, t);
    t = timer_id(p, "long2_spread");
    timer_begin(p, t);
    if ((e = l2_spread_gather<real>(p, true)) != hipSuccess) return e;
    timer_end(p, t);
    const int I0 = r.I2[0], I1 = r.I2[1], P = r.P;
    const size_t plane = (size_t)I0 * I1;
    t = timer_id(p, "long2_fft");
    timer_begin(p, t);
    // forward: y lines are contiguous (one per block), x lines are strided by I1
    if ((e = launch_fft_lines(p, ws.l2_grid, p.f2y, ws.l2_tw_y, P * I0, 1, I1, 0, 1, -1, 1)) != hipSuccess) return e;
    if ((e = launch_fft_lines(p, ws.l2_grid, p.f2x, ws.l2_tw_x, P * I1, I1, plane, 1, I1, -1, 16)) != hipSuccess) return e;
    {
        const int B = 64;
        size_t lds = (size_t)B * P * sizeof(cpx<real>);
        if (lds > 65536) return hipErrorInvalidConfiguration;
        k_l2_scale<real><<<(int)((plane + B - 1) / B), B, lds, p.stream>>>((cpx<real>*)ws.l2_grid, I0, I1, P,
                                                                           (const real*)ws.l2_kt_r);
    }
    if ((e = launch_fft_lines(p, ws.l2_grid, p.f2x, ws.l2_tw_x, P * I1, I1, plane, 1, I1, +1, 16)) != hipSuccess) return e;
    if ((e = launch_fft_lines(p, ws.l2_grid, p.f2y, ws.l2_tw_y, P * I0, 1, I1, 0, 1, +1, 1)) != hipSuccess) return e;
    timer_end(p, t);
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
