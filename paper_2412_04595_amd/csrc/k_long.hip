// Long range, Fourier-Chebyshev solver in its direct form (App. B, Alg. al::long_nonfft;
// Sec. 3.3), with Chebyshev interpolation in the target z and anterpolation in the
// source z (the "interpolation/anterpolation" of the abstract).
//
// With t = 2 z / Lz, first-kind Chebyshev nodes t_c and L_c(t) = sum_n C[c][n] T_n(t)
// (C = V^{-1}, App. A.2), the kernel of eq. trun2 sampled on the nodes,
//   K(k; c, c') = pi sum_{l>m} w_l s_l^2 exp(-s_l^2 |k|^2 / 4) exp(-(z_c - z_c')^2 / s_l^2),
// gives
//   Phi^long_i = (1/A) Re sum_k e^{i k.r_i} sum_c L_c(t_i) sum_c' K(k;c,c') sum_j q_j e^{-i k.r_j} L_c'(t_j).
// In the Chebyshev coefficient basis this is
//   mu(k, n)  = sum_j q_j e^{-i k.r_j} T_n(t_j)                 (moments: gridding + interpolation)
//   a(k, n)   = (w_k / A) sum_n' Kt(k)[n][n'] mu(k, n'),  Kt = C^T K C   (scaling, built on the host)
//   Phi^long_i = sum_{k in half plane} Re( e^{i k.r_i} sum_n T_n(t_i) a(k, n) )   (gathering)
// with w_k = 1 for k = 0 and 2 otherwise (the output is real, mu(-k) = conj mu(k)).
// The gradient uses i k in x, y and dT_n/dz = (2/Lz) n U_{n-1}(t) in z.
//
// Moments are summed per block in the working precision and across blocks in float64
// in a fixed order.
#include "launch.hpp"

namespace sog {

namespace {

template <typename real>
struct MomArgs {
    const double* x;
    const double* q;
    int n;
    double L[3];
    int nkx, nky, nh, P;
    int per_block;  // particles per block
    int chunk;      // particles per LDS batch (<= kMomThreads)
    int ts, es;     // LDS row strides of the T_n rows and of the exponential rows (elements)
    int nitems;
    double* mu;     // blocks x nh x P complex
};

__device__ __forceinline__ void mode_of(int kk, int nkx, int* nx, int* ny) {
    if (kk <= nkx) {
        *ny = 0;
        *nx = kk;
    } else {
        const int r = kk - (nkx + 1);
        *ny = 1 + r / (2 * nkx + 1);
        *nx = r % (2 * nkx + 1) - nkx;
    }
}

template <typename real>
struct MomentsK {
    static constexpr int kThreads = kMomThreads;
    // every item (mode, 4 degrees) in chunks of kMomThreads items, G = group(chunk) threads per item
    __device__ static void run(GridPos gpos, const MomArgs<real>& a) {
        for (int i0 = 0; i0 < a.nitems; i0 += kMomThreads) {
            const int left = min(kMomThreads, a.nitems - i0);
            __syncthreads();  // the previous chunk's reduction has read its LDS
            chunk(gpos, a, i0, max(1, kMomThreads / left));
        }
    }
    __device__ static void chunk(GridPos gpos, const MomArgs<real>& a, int item0, int G) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int CH = a.chunk, P = a.P;
    const int NX = 2 * a.nkx + 1, NY = a.nky + 1;
    const int TS = a.ts, ES = a.es;
    real* Tn = reinterpret_cast<real*>(smem_raw);                            // P rows of TS
    cpx<real>* ex = reinterpret_cast<cpx<real>*>(Tn + ((P * TS + 3) & ~3));  // NX rows of ES (includes q)
    cpx<real>* ey = ex + NX * ES;                                             // NY rows of ES
    cpx<real>* red = ey + NY * ES;                                            // kMomThreads x 4
    const int PB = (P + 3) / 4;
    const int item_l = threadIdx.x / G, sub = threadIdx.x - item_l * G;
    const int item = item0 + item_l;
    const bool act = item_l * G + G <= kMomThreads && item < a.nitems;
    const int kk = act ? item / PB : 0;
    const int n0 = act ? (item % PB) * 4 : 0;
    int nxs, nys;
    mode_of(kk, a.nkx, &nxs, &nys);
    cpx<real> acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = cpx<real>{0, 0};
    const int pbeg = gpos.bid * a.per_block;
    const int pend = min(a.n, pbeg + a.per_block);
    const double kx0 = 2.0 * 3.14159265358979323846 / a.L[0], ky0 = 2.0 * 3.14159265358979323846 / a.L[1];
    for (int s = pbeg; s < pend; s += CH) {
        const int cnt = min(CH, pend - s);
        if (threadIdx.x < CH) {
            const int t = threadIdx.x;
            if (t < cnt) {
                const int i = s + t;
                double xx = a.x[3 * i], yy = a.x[3 * i + 1], zz = a.x[3 * i + 2], qq = a.q[i];
                if (!(isfinite(xx) && isfinite(yy) && isfinite(zz) && isfinite(qq))) { xx = yy = zz = 0; qq = 0; }
                const double xc = wrap_periodic(xx, a.L[0]) - 0.5 * a.L[0];
                const double yc = wrap_periodic(yy, a.L[1]) - 0.5 * a.L[1];
                double tt = 2.0 * (zz - 0.5 * a.L[2]) / a.L[2];
                tt = fmin(1.0, fmax(-1.0, tt));
                const real tr = (real)tt;
                real T0 = 1, T1 = tr;
                Tn[t] = T0;
                if (P > 1) Tn[TS + t] = T1;
                for (int k = 2; k < P; ++k) {
                    const real T2 = (real)2 * tr * T1 - T0;
                    Tn[k * TS + t] = T2;
                    T0 = T1;
                    T1 = T2;
                }
                real sx, cx, sy, cy;
                dsincos((real)(kx0 * xc), &sx, &cx);
                dsincos((real)(ky0 * yc), &sy, &cy);
                const cpx<real> e1 = {cx, -sx};  // e^{-i kx0 x}
                const cpx<real> e2 = {cy, -sy};
                // e^{-i nx kx0 x} for nx = -nkx..nkx, times q
                cpx<real> pw = {(real)qq, 0};
                ex[a.nkx * ES + t] = pw;
                cpx<real> pp = pw, pm = pw;
                for (int k = 1; k <= a.nkx; ++k) {
                    pp = cmul(pp, e1);
                    pm = cmulc(pm, e1);
                    ex[(a.nkx + k) * ES + t] = pp;
                    ex[(a.nkx - k) * ES + t] = pm;
                }
                cpx<real> py = {1, 0};
                ey[t] = py;
                for (int k = 1; k <= a.nky; ++k) {
                    py = cmul(py, e2);
                    ey[k * ES + t] = py;
                }
            }
        }
        __syncthreads();
        if (act) {
            const cpx<real>* exr = ex + (nxs + a.nkx) * ES;
            const cpx<real>* eyr = ey + nys * ES;
            for (int j = sub; j < cnt; j += G) {
                const cpx<real> e = cmul(exr[j], eyr[j]);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const real tv = Tn[min(n0 + c, P - 1) * TS + j];
                    acc[c].x += e.x * tv;
                    acc[c].y += e.y * tv;
                }
            }
        }
        __syncthreads();
    }
    // sum the G partial results of each item in a fixed order
#pragma unroll
    for (int c = 0; c < 4; ++c) red[threadIdx.x * 4 + c] = acc[c];
    __syncthreads();
    if (act && sub == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int nn = n0 + c;
            if (nn >= P) continue;
            double sr = 0, si = 0;
            for (int g = 0; g < G; ++g) {
                const cpx<real> v = red[(threadIdx.x + g) * 4 + c];
                sr += (double)v.x;
                si += (double)v.y;
            }
            // partial sums as rows (mode, n) over the blocks, so the contraction reads them coalesced
            double* o = a.mu + 2 * (((size_t)kk * P + nn) * gpos.nb + gpos.bid);
            o[0] = sr;
            o[1] = si;
        }
    }
}
};

// one block per mode: for each n (a wave per n) the float64 sum of the blocks' partial
// moments (each lane a strided subset, then a fixed-order butterfly across the wave), then
// a = (w_k/A) Kt mu
constexpr int kContractThreads = 256;
template <typename real>
struct ContractK {
    static constexpr int kThreads = kContractThreads;
    __device__ static void run(GridPos gpos, const double* __restrict__ mu, int nblocks, int nh, int P,
                               const double* __restrict__ kt, double invA, cpx<real>* __restrict__ aout) {
        __shared__ double smu[2 * 64];
        const int k = gpos.bid;
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int nn = wv; nn < P; nn += kContractThreads / 64) {
            const double2* o = reinterpret_cast<const double2*>(mu) + ((size_t)k * P + nn) * nblocks;
            double sr = 0, si = 0;
            for (int b = lane; b < nblocks; b += 64) {
                const double2 v = o[b];
                sr += v.x;
                si += v.y;
            }
            for (int off = 32; off > 0; off >>= 1) {
                sr += __shfl_xor(sr, off, 64);
                si += __shfl_xor(si, off, 64);
            }
            if (lane == 0) {
                smu[2 * nn] = sr;
                smu[2 * nn + 1] = si;
            }
        }
        __syncthreads();
        const double wk = (k == 0 ? 1.0 : 2.0) * invA;
        for (int nn = threadIdx.x; nn < P; nn += kContractThreads) {
            const double* row = kt + ((size_t)k * P + nn) * P;
            double sr = 0, si = 0;
            for (int e = 0; e < P; ++e) {
                sr += row[e] * smu[2 * e];
                si += row[e] * smu[2 * e + 1];
            }
            aout[(size_t)k * P + nn] = cpx<real>{(real)(wk * sr), (real)(wk * si)};
        }
    }
};

template <typename real>
struct EvalArgs {
    const double* x;
    int n;
    double L[3];
    int nkx, nky, nh, P;
    const cpx<real>* acoef;
    vec4<real>* part;  // long part of each particle: phi, grad
};

// Evaluation for more Chebyshev terms than EvalRegK takes: T_n and T_n' per thread in LDS.
// STAGED: the coefficient table (nh x P) is copied to LDS; otherwise (a table larger than
// LDS) it is read where it is, through scalar loads (every thread reads the same entry)
template <typename real, bool STAGED, int B>
struct EvalK {
    static constexpr int kThreads = B;
    __device__ static void run(GridPos gpos, const EvalArgs<real>& a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = a.P, nh = a.nh;
    cpx<real>* sa = reinterpret_cast<cpx<real>*>(smem_raw);  // nh x P when staged
    real* Tt = reinterpret_cast<real*>(sa + (STAGED ? nh * P : 0));  // P x blockDim: T_n(t)
    real* Td = Tt + P * kThreads;                           // P x blockDim: dT_n/dt
    using ctab = const __attribute__((address_space(4))) cpx<real>;
    ctab* ga = (ctab*)a.acoef;
    if (STAGED) {
        for (int idx = threadIdx.x; idx < nh * P; idx += kThreads) sa[idx] = a.acoef[idx];
    }
    __syncthreads();
    const int i = gpos.bid * kThreads + threadIdx.x;
    if (i >= a.n) return;
    const int t = threadIdx.x;
    double xx = a.x[3 * i], yy = a.x[3 * i + 1], zz = a.x[3 * i + 2];
    if (!(isfinite(xx) && isfinite(yy) && isfinite(zz))) xx = yy = zz = 0;
    const double xc = wrap_periodic(xx, a.L[0]) - 0.5 * a.L[0];
    const double yc = wrap_periodic(yy, a.L[1]) - 0.5 * a.L[1];
    double tt = 2.0 * (zz - 0.5 * a.L[2]) / a.L[2];
    tt = fmin(1.0, fmax(-1.0, tt));
    const real tr = (real)tt;
    {
        // T_n and T_n' = n U_{n-1}
        real T0 = 1, T1 = tr, U0 = 1, U1 = 2 * tr;
        Tt[t] = 1;
        Td[t] = 0;
        if (P > 1) {
            Tt[B + t] = tr;
            Td[B + t] = 1;
        }
        for (int k = 2; k < P; ++k) {
            const real T2 = (real)2 * tr * T1 - T0;
            Tt[k * B + t] = T2;
            Td[k * B + t] = (real)k * U1;
            const real U2 = (real)2 * tr * U1 - U0;
            T0 = T1; T1 = T2;
            U0 = U1; U1 = U2;
        }
    }
    const double kx0 = 2.0 * 3.14159265358979323846 / a.L[0], ky0 = 2.0 * 3.14159265358979323846 / a.L[1];
    real sx, cx, sy, cy;
    dsincos((real)(kx0 * xc), &sx, &cx);
    dsincos((real)(ky0 * yc), &sy, &cy);
    const cpx<real> e1 = {cx, sx}, e2 = {cy, sy};
    real phi = 0, gx = 0, gy = 0, gz = 0;
    const real rkx0 = (real)kx0, rky0 = (real)ky0;
    // e^{-i nkx kx0 x}
    cpx<real> eneg = {1, 0};
    for (int k = 0; k < a.nkx; ++k) eneg = cmulc(eneg, e1);
    cpx<real> phy = {1, 0};
    int kk = 0;
    for (int ny = 0; ny <= a.nky; ++ny) {
        cpx<real> ph = (ny == 0) ? phy : cmul(phy, eneg);
        const int nxlo = (ny == 0) ? 0 : -a.nkx;
        for (int nx = nxlo; nx <= a.nkx; ++nx, ++kk) {
            real ur = 0, ui = 0, dr = 0, di = 0;
            for (int k = 0; k < P; ++k) {
                cpx<real> c;
                if (STAGED) {
                    c = sa[(size_t)kk * P + k];
                } else {
                    c.x = ga[(size_t)kk * P + k].x;
                    c.y = ga[(size_t)kk * P + k].y;
                }
                const real tv = Tt[k * B + t], dv = Td[k * B + t];
                ur += tv * c.x;
                ui += tv * c.y;
                dr += dv * c.x;
                di += dv * c.y;
            }
            // e^{i k.r} (U)
            const real re = ph.x * ur - ph.y * ui, im = ph.x * ui + ph.y * ur;
            phi += re;
            gx -= (real)nx * rkx0 * im;
            gy -= (real)ny * rky0 * im;
            gz += ph.x * dr - ph.y * di;
            ph = cmul(ph, e1);
        }
        phy = cmul(phy, e2);
    }
    a.part[i] = vec4<real>{phi, gx, gy, gz * (real)(2.0 / a.L[2])};
}
};

// P <= PR: T_n(t) and T_n'(t) in registers (loops unrolled over PR, guarded by P), the
// coefficient table read through scalar loads (every lane reads the same entry): no LDS.
// PR is 40 in float32 (one kernel for every plan of the batched workloads at tol 1e-4)
// and 16 in float64 (twice the registers per term).  Terms from 16 on sit behind one test
// of P per mode: guarded one by one they cost P = 14 more than twice the time.
template <typename real>
constexpr int eval_reg_terms() { return sizeof(real) == 4 ? 40 : 16; }
constexpr int kEvalRegHead = 16;
template <typename real, int PR>
struct EvalRegK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, const EvalArgs<real>& a) {
    static_assert(PR >= 2, "two Chebyshev terms at least");
    constexpr int kHead = PR < kEvalRegHead ? PR : kEvalRegHead;
    const int P = a.P;
    using ctab = const __attribute__((address_space(4))) cpx<real>;
    ctab* ga = (ctab*)a.acoef;
    const int i = gpos.bid * kThreads + threadIdx.x;
    if (i >= a.n) return;
    double xx = a.x[3 * i], yy = a.x[3 * i + 1], zz = a.x[3 * i + 2];
    if (!(isfinite(xx) && isfinite(yy) && isfinite(zz))) xx = yy = zz = 0;
    const double xc = wrap_periodic(xx, a.L[0]) - 0.5 * a.L[0];
    const double yc = wrap_periodic(yy, a.L[1]) - 0.5 * a.L[1];
    double tt = 2.0 * (zz - 0.5 * a.L[2]) / a.L[2];
    tt = fmin(1.0, fmax(-1.0, tt));
    const real tr = (real)tt;
    real Tt[PR], Td[PR];
    {
        real T0 = 1, T1 = tr, U0 = 1, U1 = 2 * tr;
        Tt[0] = 1;
        Td[0] = 0;
        Tt[1] = tr;
        Td[1] = 1;
#pragma unroll
        for (int k = 2; k < kHead; ++k) {
            if (k < P) {
                const real T2 = (real)2 * tr * T1 - T0;
                Tt[k] = T2;
                Td[k] = (real)k * U1;
                const real U2 = (real)2 * tr * U1 - U0;
                T0 = T1; T1 = T2;
                U0 = U1; U1 = U2;
            }
        }
        if (PR > kHead && P > kHead) {
#pragma unroll
            for (int k = kHead; k < PR; ++k) {
                if (k < P) {
                    const real T2 = (real)2 * tr * T1 - T0;
                    Tt[k] = T2;
                    Td[k] = (real)k * U1;
                    const real U2 = (real)2 * tr * U1 - U0;
                    T0 = T1; T1 = T2;
                    U0 = U1; U1 = U2;
                }
            }
        }
    }
    const double kx0 = 2.0 * 3.14159265358979323846 / a.L[0], ky0 = 2.0 * 3.14159265358979323846 / a.L[1];
    real sx, cx, sy, cy;
    dsincos((real)(kx0 * xc), &sx, &cx);
    dsincos((real)(ky0 * yc), &sy, &cy);
    const cpx<real> e1 = {cx, sx}, e2 = {cy, sy};
    real phi = 0, gx = 0, gy = 0, gz = 0;
    const real rkx0 = (real)kx0, rky0 = (real)ky0;
    cpx<real> eneg = {1, 0};
    for (int k = 0; k < a.nkx; ++k) eneg = cmulc(eneg, e1);
    cpx<real> phy = {1, 0};
    int kk = 0;
    for (int ny = 0; ny <= a.nky; ++ny) {
        cpx<real> ph = (ny == 0) ? phy : cmul(phy, eneg);
        const int nxlo = (ny == 0) ? 0 : -a.nkx;
        for (int nx = nxlo; nx <= a.nkx; ++nx, ++kk) {
            real ur = 0, ui = 0, dr = 0, di = 0;
            ctab* row = ga + (size_t)kk * P;
#pragma unroll
            for (int k = 0; k < kHead; ++k) {
                if (k < P) {
                    const real c_x = row[k].x, c_y = row[k].y;
                    ur += Tt[k] * c_x;
                    ui += Tt[k] * c_y;
                    dr += Td[k] * c_x;
                    di += Td[k] * c_y;
                }
            }
            if (PR > kHead && P > kHead) {
#pragma unroll
                for (int k = kHead; k < PR; ++k) {
                    if (k < P) {
                        const real c_x = row[k].x, c_y = row[k].y;
                        ur += Tt[k] * c_x;
                        ui += Tt[k] * c_y;
                        dr += Td[k] * c_x;
                        di += Td[k] * c_y;
                    }
                }
            }
            const real re = ph.x * ur - ph.y * ui, im = ph.x * ui + ph.y * ur;
            phi += re;
            gx -= (real)nx * rkx0 * im;
            gy -= (real)ny * rky0 * im;
            gz += ph.x * dr - ph.y * di;
            ph = cmul(ph, e1);
        }
        phy = cmul(phy, e2);
    }
    a.part[i] = vec4<real>{phi, gx, gy, gz * (real)(2.0 / a.L[2])};
}
};

template <typename real>
hipError_t run_long_direct(Plan& p, const double* x, const double* q) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int n = (int)r.n, P = r.P, nh = r.nh;
    MomArgs<real> a;
    a.x = x;
    a.q = q;
    a.n = n;
    for (int d = 0; d < 3; ++d) a.L[d] = r.L[d];
    a.nkx = r.nk[0];
    a.nky = r.nk[1];
    a.nh = nh;
    a.P = P;
    const int nb = ws.long_blocks;
    a.per_block = (n + nb - 1) / nb;
    // LDS rows padded one (T_n) and four (exponentials) elements past the chunk: a wave reads
    // 4 degree rows and 4 modes at 4 consecutive particles, and a row stride that is a multiple
    // of the bank count puts all of them in the same 4 banks. Unpadded where only that fits.
    auto lds_of = [&](int ch, int pad) { return long_moments_lds(sizeof(real), P, r.nk[0], r.nk[1], ch, pad); };
    int CH = kMomThreads, pad = 1;
    for (;; pad = 0, CH = kMomThreads) {
        while (CH > kMomMinChunk && lds_of(CH, pad) > 49152) CH >>= 1;
        if (lds_of(CH, pad) <= kMomMaxLds || pad == 0) break;
    }
    if (lds_of(CH, pad) > kMomMaxLds) return hipErrorInvalidConfiguration;
    a.chunk = CH;
    a.ts = CH + pad;
    a.es = CH + 4 * pad;
    a.mu = ws.long_mu;
    const int PB = (P + 3) / 4;
    const int nitems = nh * PB;
    a.nitems = nitems;
    const size_t lds = lds_of(CH, pad);
    int t = timer_id(p, "long_moments");
    timer_begin(p, t);
    hipError_t e = launch<MomentsK<real>>(p, nb, lds, a);
    timer_end(p, t);
    if (e != hipSuccess) return e;
    t = timer_id(p, "long_contract");
    timer_begin(p, t);
    e = launch<ContractK<real>>(p, nh, 0, (const double*)ws.long_mu, nb, nh, P, (const double*)ws.long_kt,
                                1.0 / (r.L[0] * r.L[1]), (cpx<real>*)ws.long_a);
    timer_end(p, t);
    if (e != hipSuccess) return e;
    EvalArgs<real> ea;
    ea.x = x;
    ea.n = n;
    for (int d = 0; d < 3; ++d) ea.L[d] = r.L[d];
    ea.nkx = r.nk[0];
    ea.nky = r.nk[1];
    ea.nh = nh;
    ea.P = P;
    ea.acoef = (const cpx<real>*)ws.long_a;
    ea.part = (vec4<real>*)ws.parts + 2 * r.n;
    int B = 256;
    while (B > 64 && (size_t)nh * P * sizeof(cpx<real>) + 2 * (size_t)P * B * sizeof(real) > 65536) B >>= 1;
    size_t lds2 = (size_t)nh * P * sizeof(cpx<real>) + 2 * (size_t)P * B * sizeof(real);
    const bool staged = lds2 <= 65536;
    if (!staged) {
        B = 256;
        while (B > 64 && 2 * (size_t)P * B * sizeof(real) > 65536) B >>= 1;
        lds2 = 2 * (size_t)P * B * sizeof(real);
        if (lds2 > 65536) return hipErrorInvalidConfiguration;
    }
    t = timer_id(p, "long_eval");
    timer_begin(p, t);
    const int nbl = (n + B - 1) / B;
    if (P <= eval_reg_terms<real>())
        e = launch<EvalRegK<real, eval_reg_terms<real>()>>(p, (n + 255) / 256, 0, ea);
    else if (staged)
        e = B == 256 ? launch<EvalK<real, true, 256>>(p, nbl, lds2, ea)
                     : (B == 128 ? launch<EvalK<real, true, 128>>(p, nbl, lds2, ea) : launch<EvalK<real, true, 64>>(p, nbl, lds2, ea));
    else
        e = B == 256 ? launch<EvalK<real, false, 256>>(p, nbl, lds2, ea)
                     : (B == 128 ? launch<EvalK<real, false, 128>>(p, nbl, lds2, ea) : launch<EvalK<real, false, 64>>(p, nbl, lds2, ea));
    timer_end(p, t);
    return e;
}

}  // namespace

hipError_t launch_long_fft(Plan& p, const double* x, const double* q);  // k_long2.hip

hipError_t launch_long(Plan& p, const double* x, const double* q) {
    if (p.r.form == SOG_LONG_FFT) return launch_long_fft(p, x, q);
    if (p.r.prec == SOG_PREC_FP64) return run_long_direct<double>(p, x, q);
    return run_long_direct<float>(p, x, q);
}

}  // namespace sog
