// The library's own FFTs and the mid-range scaling (Alg. al::mid steps 2-4).
//
// Layout: the real grid is grid[(a * I_y + b) * I_z* + c]; its half spectrum is
// cgrid[(a * I_y + b) * K_z + k], K_z = I_z*/2 + 1.  The chain is
//   1. real-to-complex along z (a complex FFT of length I_z*/2 on packed pairs, then the
//      usual split into the half spectrum),
//   2. complex FFT along y,
//   3. complex FFT along x, multiplication by Ghat_mid(k) / What(k)^2 / (I_x I_y I_z*),
//      inverse FFT along x -- all in one kernel, the lines never leave LDS,
//   4. inverse FFT along y,
//   5. complex-to-real along z.
// Ghat_mid(k) = pi^{3/2} sum_{l<=m} w_l s_l^3 exp(-s_l^2 |k|^2/4) (eqs. phindf and
// widehat-tilde with the SOG screening), What the Gaussian window transform of eq. GS;
// both are separable per Gaussian, so the multiplier is formed on the fly from three
// small per-direction tables and costs no HBM traffic.
//
// Every line transform runs in LDS: a batch of W lines is loaded with coalesced
// accesses, transformed in place by Stockham radix-2/3/4/5/7 passes (natural order; each
// thread holds its butterflies in registers across a stage; small DFTs with constant
// coefficients; twiddles e^{-2 pi i t/n} from a float64-built table staged in LDS), and
// stored.  Each pass reads and writes the grid once.
#include "device_common.hpp"

namespace sog {

namespace {

// Per-stage constants of one line length, uniform over the launch.
struct FFTDev {
    int n;
    int nstages;
    int radix[kMaxStages];
    int Ns[kMaxStages];          // product of the radices of the earlier stages
    int nR[kMaxStages];          // n / R
    int tws[kMaxStages];         // n / (Ns R): step of the twiddle index
    unsigned mNs[kMaxStages];    // ceil(2^32 / Ns) (Ns >= 2): j / Ns = umulhi(j, mNs) for j < 2^16
};

FFTDev to_dev(const FFTFactors& f) {
    FFTDev d;
    d.n = f.n;
    d.nstages = f.nstages;
    int Ns = 1;
    for (int i = 0; i < kMaxStages; ++i) {
        const int R = (i < f.nstages) ? f.radix[i] : 1;
        d.radix[i] = R;
        d.Ns[i] = Ns;
        d.nR[i] = f.n / R;
        d.tws[i] = f.n / (Ns * R);
        d.mNs[i] = (Ns >= 2) ? (unsigned)((((uint64_t)1 << 32) + (uint64_t)Ns - 1) / (uint64_t)Ns) : 0u;
        if (i < f.nstages) Ns *= R;
    }
    return d;
}

// cos and sin of 2 pi q / R for the odd radices (exact to double precision)
__host__ __device__ constexpr double rot_c(int R, int q) {
    return R == 3 ? (q == 0 ? 1.0 : -0.5)
         : R == 5 ? (q == 0 ? 1.0 : (q == 1 || q == 4) ? 0.309016994374947424102293 : -0.809016994374947424102293)
         : (q == 0 ? 1.0 : (q == 1 || q == 6) ? 0.623489801858733530525004
                         : (q == 2 || q == 5) ? -0.222520933956314404288902 : -0.900968867902419126236102);
}
__host__ __device__ constexpr double rot_s(int R, int q) {
    return R == 3 ? (q == 0 ? 0.0 : q == 1 ? 0.866025403784438646763723 : -0.866025403784438646763723)
         : R == 5 ? (q == 0 ? 0.0 : q == 1 ? 0.951056516295153572116439 : q == 2 ? 0.587785252292473129168706
                    : q == 3 ? -0.587785252292473129168706 : -0.951056516295153572116439)
         : (q == 0 ? 0.0 : q == 1 ? 0.781831482468029808708444 : q == 2 ? 0.974927912181823607018131
            : q == 3 ? 0.433883739117558120475768 : q == 4 ? -0.433883739117558120475768
            : q == 5 ? -0.974927912181823607018131 : -0.781831482468029808708444);
}

// o_p = sum_r v_r e^{SIGN 2 pi i p r / R}
template <typename T, int R, int SIGN>
__device__ __forceinline__ void small_dft(const cpx<T> (&v)[R], cpx<T> (&o)[R]) {
    if constexpr (R == 2) {
        o[0] = cadd(v[0], v[1]);
        o[1] = csub(v[0], v[1]);
    } else if constexpr (R == 4) {
        const cpx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]), c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
        // d times e^{SIGN i pi/2}
        const cpx<T> di = (SIGN < 0) ? cpx<T>{d.y, -d.x} : cpx<T>{-d.y, d.x};
        o[0] = cadd(a, c);
        o[2] = csub(a, c);
        o[1] = cadd(b, di);
        o[3] = csub(b, di);
    } else {
        // odd R: pair r with R - r
        constexpr int H = (R - 1) / 2;
        cpx<T> a[H], b[H];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            a[k] = cadd(v[k + 1], v[R - 1 - k]);
            b[k] = csub(v[k + 1], v[R - 1 - k]);
        }
        cpx<T> s0 = v[0];
#pragma unroll
        for (int k = 0; k < H; ++k) s0 = cadd(s0, a[k]);
        o[0] = s0;
#pragma unroll
        for (int p = 1; p <= H; ++p) {
            cpx<T> re = v[0], im = {0, 0};
#pragma unroll
            for (int k = 1; k <= H; ++k) {
                const T c = (T)rot_c(R, (p * k) % R), sn = (T)rot_s(R, (p * k) % R);
                re.x += c * a[k - 1].x;
                re.y += c * a[k - 1].y;
                im.x += sn * b[k - 1].x;
                im.y += sn * b[k - 1].y;
            }
            // o_p = re + SIGN i im, o_{R-p} = re - SIGN i im
            o[p] = cpx<T>{re.x - (T)SIGN * im.y, re.y + (T)SIGN * im.x};
            o[R - p] = cpx<T>{re.x + (T)SIGN * im.y, re.y - (T)SIGN * im.x};
        }
    }
}

// Largest line batch (elements per block: n x W) of the in-place LDS transform; also
// bounds the butterflies a thread holds in registers during a stage.
template <typename T>
constexpr int kFFTCap = (sizeof(T) == 4) ? 4096 : 2048;
constexpr int kFFTThreads = 256;

// One Stockham stage of radix R, in place on A (element i of line w at A[i W + w]):
// every thread first reads all the butterflies it owns into registers, the block
// synchronises, then the results are written back.  twl: the twiddles e^{-2 pi i t/n}.
template <typename T, int R, int SIGN>
__device__ __forceinline__ void fft_stage(cpx<T>* A, const cpx<T>* __restrict__ twl, int W, int lw, int nR, int Ns,
                                          unsigned mNs, int tws) {
    constexpr int MAXB = (kFFTCap<T> / R + kFFTThreads - 1) / kFFTThreads;
    const int nb = nR * W;
    cpx<T> o[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int idx = threadIdx.x + b * kFFTThreads;
        dst[b] = -1;
        if (idx < nb) {
            const int w = idx & (W - 1), j = idx >> lw;
            const int g = (Ns == 1) ? j : (int)__umulhi((unsigned)j, mNs);
            const int k = j - g * Ns;
            cpx<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = A[(j + r * nR) * W + w];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cpx<T> t = twl[k * r * tws];
                    if (SIGN > 0) t.y = -t.y;
                    v[r] = cmul(v[r], t);
                }
            }
            small_dft<T, R, SIGN>(v, o[b]);
            dst[b] = (g * Ns * R + k) * W + w;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b)
        if (dst[b] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) A[dst[b] + r * Ns * W] = o[b][r];
        }
    __syncthreads();
}

// In-LDS transform of W interleaved lines (W a power of two, n W <= kFFTCap).  The
// caller synchronises before (data in A) and may read A after the return.
template <typename T, int SIGN>
__device__ void lds_fft(cpx<T>* A, const cpx<T>* __restrict__ twl, int W, const FFTDev& f) {
    const int lw = __ffs(W) - 1;
    for (int s = 0; s < f.nstages; ++s) {
        switch (f.radix[s]) {
            case 4: fft_stage<T, 4, SIGN>(A, twl, W, lw, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 2: fft_stage<T, 2, SIGN>(A, twl, W, lw, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 3: fft_stage<T, 3, SIGN>(A, twl, W, lw, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 5: fft_stage<T, 5, SIGN>(A, twl, W, lw, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            default: fft_stage<T, 7, SIGN>(A, twl, W, lw, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
        }
    }
}

template <typename T>
__device__ __forceinline__ void load_twiddles(cpx<T>* twl, const cpx<T>* __restrict__ tw, int n) {
    for (int t = threadIdx.x; t < n; t += kFFTThreads) twl[t] = tw[t];
}

// lines per block: a power of two, n W <= kFFTCap, at most 16
template <typename T>
int lines_per_block(int n) {
    int W = 16;
    while (W > 1 && (size_t)n * W > (size_t)kFFTCap<T>) W >>= 1;
    return W;
}

// 1. real-to-complex along z for W lines per block.  m = I_z*/2.
template <typename T>
__global__ __launch_bounds__(kFFTThreads) void k_fft_z_r2c(const T* __restrict__ grid, cpx<T>* __restrict__ cg,
                                                           int nlines, int Izs, int Kz, int Kzs, int W, FFTDev f,
                                                           const cpx<T>* __restrict__ tw,
                                                           const cpx<T>* __restrict__ twpost) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = f.n;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* twl = A + m * W;
    const int line0 = blockIdx.x * W;
    load_twiddles(twl, tw, m);
    for (int w = 0; w < W; ++w) {
        const int line = line0 + w;
        const cpx<T>* row = reinterpret_cast<const cpx<T>*>(grid + (size_t)min(line, nlines - 1) * Izs);
        for (int t = threadIdx.x; t < m; t += kFFTThreads) A[t * W + w] = (line < nlines) ? row[t] : cpx<T>{0, 0};
    }
    __syncthreads();
    lds_fft<T, -1>(A, twl, W, f);
    for (int w = 0; w < W; ++w) {
        const int line = line0 + w;
        if (line >= nlines) break;
        for (int k = threadIdx.x; k <= m; k += kFFTThreads) {
            const cpx<T> zk = A[(k == m ? 0 : k) * W + w];
            const cpx<T> zmk = cconj(A[(k == 0 ? 0 : m - k) * W + w]);
            const cpx<T> e = {(zk.x + zmk.x) * (T)0.5, (zk.y + zmk.y) * (T)0.5};
            const cpx<T> dd = csub(zk, zmk);
            const cpx<T> o = {dd.y * (T)0.5, -dd.x * (T)0.5};  // (zk - zmk) / (2i)
            cg[(size_t)line * Kzs + k] = cadd(e, cmul(twpost[k], o));
        }
    }
}

// 5. complex-to-real along z (unnormalised inverse).
template <typename T>
__global__ __launch_bounds__(kFFTThreads) void k_fft_z_c2r(const cpx<T>* __restrict__ cg, T* __restrict__ grid,
                                                           int nlines, int Izs, int Kz, int Kzs, int W, FFTDev f,
                                                           const cpx<T>* __restrict__ tw,
                                                           const cpx<T>* __restrict__ twpost) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = f.n;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* twl = A + m * W;
    const int line0 = blockIdx.x * W;
    load_twiddles(twl, tw, m);
    for (int w = 0; w < W; ++w) {
        const int line = line0 + w;
        const cpx<T>* row = cg + (size_t)min(line, nlines - 1) * Kzs;
        for (int k = threadIdx.x; k < m; k += kFFTThreads) {
            const cpx<T> xk = row[k];
            const cpx<T> xmk = cconj(row[m - k]);
            const cpx<T> e = cadd(xk, xmk);
            const cpx<T> o = cmulc(csub(xk, xmk), twpost[k]);  // times e^{+2 pi i k / I_z*}
            A[k * W + w] = (line < nlines) ? cpx<T>{e.x - o.y, e.y + o.x} : cpx<T>{0, 0};  // e + i o
        }
    }
    __syncthreads();
    lds_fft<T, +1>(A, twl, W, f);
    for (int w = 0; w < W; ++w) {
        const int line = line0 + w;
        if (line >= nlines) break;
        cpx<T>* row = reinterpret_cast<cpx<T>*>(grid + (size_t)line * Izs);
        for (int t = threadIdx.x; t < m; t += kFFTThreads) row[t] = A[t * W + w];
    }
}

// 2./4. complex FFT along y for (x, a batch of W consecutive k_z)
template <typename T, int SIGN>
__global__ __launch_bounds__(kFFTThreads) void k_fft_y(cpx<T>* __restrict__ cg, int Ix, int Iy, int Kz, int Kzs, int W,
                                                       FFTDev f, const cpx<T>* __restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* twl = A + Iy * W;
    const int nkb = (Kz + W - 1) / W;
    const int ix = blockIdx.x / nkb, kz0 = (blockIdx.x % nkb) * W;
    if (ix >= Ix) return;
    const int lw = __ffs(W) - 1;
    load_twiddles(twl, tw, Iy);
    cpx<T>* base = cg + (size_t)ix * Iy * Kzs + kz0;
    for (int idx = threadIdx.x; idx < Iy * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), iy = idx >> lw;
        A[idx] = (kz0 + w < Kz) ? base[(size_t)iy * Kzs + w] : cpx<T>{0, 0};
    }
    __syncthreads();
    lds_fft<T, SIGN>(A, twl, W, f);
    for (int idx = threadIdx.x; idx < Iy * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), iy = idx >> lw;
        if (kz0 + w < Kz) base[(size_t)iy * Kzs + w] = A[idx];
    }
}

// 3. forward FFT along x, the SOG multiplier, inverse FFT along x.  The multiplier is
// sum_l c_l ax_l(k_x) ay_l(k_y) az_l(k_z): the block's (k_y, k_z) factors and ax are
// staged in LDS.
template <typename T>
__global__ __launch_bounds__(kFFTThreads) void k_fft_x_scale(cpx<T>* __restrict__ cg, int Ix, int Iy, int Kz, int Kzs,
                                                             int W,
                                                             FFTDev f, const cpx<T>* __restrict__ tw, int nl,
                                                             const T* __restrict__ ax, const T* __restrict__ ay,
                                                             const T* __restrict__ az, const T* __restrict__ cl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* twl = A + Ix * W;
    T* cyz = reinterpret_cast<T*>(twl + Ix);  // nl x W
    T* axl = cyz + nl * W;                    // nl x Ix
    const int nkb = (Kz + W - 1) / W;
    const int iy = blockIdx.x / nkb, kz0 = (blockIdx.x % nkb) * W;
    if (iy >= Iy) return;
    const int lw = __ffs(W) - 1;
    const size_t stride = (size_t)Iy * Kzs;
    cpx<T>* base = cg + (size_t)iy * Kzs + kz0;
    load_twiddles(twl, tw, Ix);
    for (int idx = threadIdx.x; idx < Ix * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), ix = idx >> lw;
        A[idx] = (kz0 + w < Kz) ? base[ix * stride + w] : cpx<T>{0, 0};
    }
    for (int idx = threadIdx.x; idx < nl * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), l = idx >> lw;
        const int kz = min(kz0 + w, Kz - 1);
        cyz[idx] = cl[l] * ay[l * Iy + iy] * az[l * Kz + kz];
    }
    for (int idx = threadIdx.x; idx < nl * Ix; idx += kFFTThreads) axl[idx] = ax[idx];
    __syncthreads();
    lds_fft<T, -1>(A, twl, W, f);
    for (int idx = threadIdx.x; idx < Ix * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), ix = idx >> lw;
        T mlt = 0;
        for (int l = 0; l < nl; ++l) mlt += axl[l * Ix + ix] * cyz[l * W + w];
        cpx<T> v = A[idx];
        v.x *= mlt;
        v.y *= mlt;
        A[idx] = v;
    }
    __syncthreads();
    lds_fft<T, +1>(A, twl, W, f);
    for (int idx = threadIdx.x; idx < Ix * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), ix = idx >> lw;
        if (kz0 + w < Kz) base[ix * stride + w] = A[idx];
    }
}

// Generic batched line transform: W consecutive lines per block; line l starts at
// (l / ncols) * outer_stride + (l % ncols) * col_stride, elements at elem_stride.
// Lines adjacent in memory (col_stride == 1) load and store coalesced.
template <typename T, int SIGN>
__global__ __launch_bounds__(kFFTThreads) void k_fft_lines(cpx<T>* __restrict__ d, int nlines, int ncols,
                                                           size_t outer_stride, size_t col_stride, size_t elem_stride,
                                                           int W, FFTDev f, const cpx<T>* __restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = f.n;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* twl = A + n * W;
    const int line0 = blockIdx.x * W;
    const int lw = __ffs(W) - 1;
    load_twiddles(twl, tw, n);
    for (int idx = threadIdx.x; idx < n * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), e = idx >> lw, line = line0 + w;
        cpx<T> v = {0, 0};
        if (line < nlines) v = d[(size_t)(line / ncols) * outer_stride + (size_t)(line % ncols) * col_stride + (size_t)e * elem_stride];
        A[idx] = v;
    }
    __syncthreads();
    lds_fft<T, SIGN>(A, twl, W, f);
    for (int idx = threadIdx.x; idx < n * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), e = idx >> lw, line = line0 + w;
        if (line < nlines)
            d[(size_t)(line / ncols) * outer_stride + (size_t)(line % ncols) * col_stride + (size_t)e * elem_stride] = A[idx];
    }
}

template <typename T>
hipError_t run_fft_mid(Plan& p) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int Ix = r.I[0], Iy = r.I[1], Izs = r.Izs, Kz = Izs / 2 + 1, m = Izs / 2, Kzs = cgrid_stride(Izs);
    const int nlines = Ix * Iy;
    const size_t ce = sizeof(cpx<T>);
    const size_t budget = 65536;
    const int nl = r.m + 1;
    hipError_t e;
    if ((size_t)m > (size_t)kFFTCap<T> || (size_t)Ix > (size_t)kFFTCap<T> || (size_t)Iy > (size_t)kFFTCap<T>)
        return hipErrorInvalidConfiguration;
    // 1. z forward
    const int Wz = lines_per_block<T>(m);
    const size_t ldsz = (size_t)m * (Wz + 1) * ce;
    if (ldsz > budget) return hipErrorInvalidConfiguration;
    {
        int t = timer_id(p, "fft_z_fwd");
        timer_begin(p, t);
        k_fft_z_r2c<T><<<(nlines + Wz - 1) / Wz, kFFTThreads, ldsz, p.stream>>>(
            (const T*)ws.grid, (cpx<T>*)ws.cgrid, nlines, Izs, Kz, Kzs, Wz, to_dev(p.fz), (const cpx<T>*)ws.tw_z,
            (const cpx<T>*)ws.tw_zpost);
        timer_end(p, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 2. y forward
    const int Wy = lines_per_block<T>(Iy);
    const size_t ldsy = (size_t)Iy * (Wy + 1) * ce;
    if (ldsy > budget) return hipErrorInvalidConfiguration;
    const int nby = Ix * ((Kz + Wy - 1) / Wy);
    {
        int t = timer_id(p, "fft_y_fwd");
        timer_begin(p, t);
        k_fft_y<T, -1><<<nby, kFFTThreads, ldsy, p.stream>>>((cpx<T>*)ws.cgrid, Ix, Iy, Kz, Kzs, Wy, to_dev(p.fy),
                                                             (const cpx<T>*)ws.tw_y);
        timer_end(p, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 3. x forward, scale, x inverse
    {
        int W = lines_per_block<T>(Ix);
        auto lds_of = [&](int w) { return (size_t)Ix * (w + 1) * ce + (size_t)nl * (w + Ix) * sizeof(T); };
        while (W > 1 && lds_of(W) > budget) W >>= 1;
        const size_t lds = lds_of(W);
        if (lds > budget) return hipErrorInvalidConfiguration;
        int nb = Iy * ((Kz + W - 1) / W);
        int t = timer_id(p, "fft_x_scale");
        timer_begin(p, t);
        k_fft_x_scale<T><<<nb, kFFTThreads, lds, p.stream>>>((cpx<T>*)ws.cgrid, Ix, Iy, Kz, Kzs, W, to_dev(p.fx),
                                                             (const cpx<T>*)ws.tw_x, nl, (const T*)ws.mult_ax,
                                                             (const T*)ws.mult_ay, (const T*)ws.mult_az,
                                                             (const T*)ws.mult_c);
        timer_end(p, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 4. y inverse
    {
        int t = timer_id(p, "fft_y_inv");
        timer_begin(p, t);
        k_fft_y<T, +1><<<nby, kFFTThreads, ldsy, p.stream>>>((cpx<T>*)ws.cgrid, Ix, Iy, Kz, Kzs, Wy, to_dev(p.fy),
                                                             (const cpx<T>*)ws.tw_y);
        timer_end(p, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 5. z inverse
    {
        int t = timer_id(p, "fft_z_inv");
        timer_begin(p, t);
        k_fft_z_c2r<T><<<(nlines + Wz - 1) / Wz, kFFTThreads, ldsz, p.stream>>>(
            (const cpx<T>*)ws.cgrid, (T*)ws.grid, nlines, Izs, Kz, Kzs, Wz, to_dev(p.fz), (const cpx<T>*)ws.tw_z,
            (const cpx<T>*)ws.tw_zpost);
        timer_end(p, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_fft_lines(Plan& p, void* data, const FFTFactors& f, const void* tw, int nlines, int ncols,
                            size_t outer_stride, size_t col_stride, size_t elem_stride, int sign, int W) {
    const bool f64 = p.r.prec == SOG_PREC_FP64;
    const size_t ce = f64 ? 16 : 8;
    const int cap = f64 ? kFFTCap<double> : kFFTCap<float>;
    int Wp = 1;
    while (Wp * 2 <= W) Wp *= 2;  // a power of two
    while (Wp > 1 && (size_t)f.n * Wp > (size_t)cap) Wp >>= 1;
    const size_t lds = (size_t)f.n * (Wp + 1) * ce;
    if (f.n > cap || lds > 65536 || nlines <= 0) return hipErrorInvalidConfiguration;
    const int nb = (nlines + Wp - 1) / Wp;
    if (f64) {
        if (sign < 0)
            k_fft_lines<double, -1><<<nb, kFFTThreads, lds, p.stream>>>((cpx<double>*)data, nlines, ncols, outer_stride,
                                                                       col_stride, elem_stride, Wp, to_dev(f), (const cpx<double>*)tw);
        else
            k_fft_lines<double, +1><<<nb, kFFTThreads, lds, p.stream>>>((cpx<double>*)data, nlines, ncols, outer_stride,
                                                                       col_stride, elem_stride, Wp, to_dev(f), (const cpx<double>*)tw);
    } else {
        if (sign < 0)
            k_fft_lines<float, -1><<<nb, kFFTThreads, lds, p.stream>>>((cpx<float>*)data, nlines, ncols, outer_stride,
                                                                      col_stride, elem_stride, Wp, to_dev(f), (const cpx<float>*)tw);
        else
            k_fft_lines<float, +1><<<nb, kFFTThreads, lds, p.stream>>>((cpx<float>*)data, nlines, ncols, outer_stride,
                                                                      col_stride, elem_stride, Wp, to_dev(f), (const cpx<float>*)tw);
    }
    return hipGetLastError();
}

hipError_t launch_fft_mid(Plan& p) {
    if (p.r.prec == SOG_PREC_FP64) return run_fft_mid<double>(p);
    return run_fft_mid<float>(p);
}

}  // namespace sog
