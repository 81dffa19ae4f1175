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
// accesses, transformed by Stockham radix-2/3/4/5/7 passes (natural order, ping-pong
// between two LDS buffers, twiddles e^{-2 pi i t/n} from a float64-built table), and
// stored.  Each pass reads and writes the grid once.
#include "device_common.hpp"

namespace sog {

namespace {

struct FFTDev {
    int n;
    int nstages;
    int radix[kMaxStages];
};

FFTDev to_dev(const FFTFactors& f) {
    FFTDev d;
    d.n = f.n;
    d.nstages = f.nstages;
    for (int i = 0; i < kMaxStages; ++i) d.radix[i] = f.radix[i];
    return d;
}

template <typename T>
__device__ __forceinline__ cpx<T> twiddle(const cpx<T>* tw, int idx, int sign) {
    cpx<T> t = tw[idx];
    if (sign > 0) t.y = -t.y;
    return t;
}

// one radix-R butterfly of a Stockham pass: reads src[(j + r n/R) W + w], writes
// dst[((j / Ns) Ns R + j % Ns + r Ns) W + w]
template <typename T, int R>
__device__ __forceinline__ void butterfly(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst, int j, int nR,
                                          int Ns, int tws, int W, int w, const cpx<T>* __restrict__ tw, int n, int sign) {
    const int k = j % Ns;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(j + r * nR) * W + w];
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twiddle(tw, k * r * tws, sign));
    cpx<T> o[R];
    if (R == 2) {
        o[0] = cadd(v[0], v[1]);
        o[1] = csub(v[0], v[1]);
    } else if (R == 4) {
        const cpx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]), c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
        // d times e^{sign i pi/2}: -i d for the forward transform, +i d for the inverse
        const cpx<T> di = (sign < 0) ? cpx<T>{d.y, -d.x} : cpx<T>{-d.y, d.x};
        o[0] = cadd(a, c);
        o[2] = csub(a, c);
        o[1] = cadd(b, di);
        o[3] = csub(b, di);
    } else {
        const int step = n / R;
#pragma unroll
        for (int pp = 0; pp < R; ++pp) {
            cpx<T> s = v[0];
#pragma unroll
            for (int r = 1; r < R; ++r) s = cadd(s, cmul(v[r], twiddle(tw, ((pp * r) % R) * step, sign)));
            o[pp] = s;
        }
    }
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(base + r * Ns) * W + w] = o[r];
}

// In-LDS transform of W interleaved lines (element i of line w at A[i W + w]).
// Returns the buffer (A or B) that holds the result.
template <typename T>
__device__ cpx<T>* lds_fft(cpx<T>* A, cpx<T>* B, int W, const FFTDev& f, const cpx<T>* __restrict__ tw, int sign) {
    const int n = f.n;
    int Ns = 1;
    for (int s = 0; s < f.nstages; ++s) {
        const int R = f.radix[s];
        const int nR = n / R;
        const int tws = n / (Ns * R);
        for (int idx = threadIdx.x; idx < nR * W; idx += blockDim.x) {
            const int w = idx % W, j = idx / W;
            switch (R) {
                case 4: butterfly<T, 4>(A, B, j, nR, Ns, tws, W, w, tw, n, sign); break;
                case 2: butterfly<T, 2>(A, B, j, nR, Ns, tws, W, w, tw, n, sign); break;
                case 3: butterfly<T, 3>(A, B, j, nR, Ns, tws, W, w, tw, n, sign); break;
                case 5: butterfly<T, 5>(A, B, j, nR, Ns, tws, W, w, tw, n, sign); break;
                default: butterfly<T, 7>(A, B, j, nR, Ns, tws, W, w, tw, n, sign); break;
            }
        }
        __syncthreads();
        cpx<T>* t = A;
        A = B;
        B = t;
        Ns *= R;
    }
    return A;
}

constexpr int kFFTThreads = 256;

// 1. real-to-complex along z for W lines per block.  m = I_z*/2.
template <typename T>
__global__ __launch_bounds__(kFFTThreads) void k_fft_z_r2c(const T* __restrict__ grid, cpx<T>* __restrict__ cg,
                                                           int nlines, int Izs, int Kz, int W, FFTDev f,
                                                           const cpx<T>* __restrict__ tw,
                                                           const cpx<T>* __restrict__ twpost) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = f.n;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (m + 1) * W;
    const int line0 = blockIdx.x * W;
    for (int idx = threadIdx.x; idx < m * W; idx += blockDim.x) {
        const int w = idx / m, t = idx % m, line = line0 + w;
        cpx<T> v = {0, 0};
        if (line < nlines) {
            const T* row = grid + (size_t)line * Izs;
            v.x = row[2 * t];
            v.y = row[2 * t + 1];
        }
        A[t * W + w] = v;
    }
    __syncthreads();
    cpx<T>* Z = lds_fft(A, B, W, f, tw, -1);
    for (int idx = threadIdx.x; idx < (m + 1) * W; idx += blockDim.x) {
        const int w = idx / (m + 1), k = idx % (m + 1), line = line0 + w;
        if (line >= nlines) continue;
        const cpx<T> zk = Z[(k % m) * W + w];
        const cpx<T> zmk = cconj(Z[((m - k) % m) * W + w]);
        const cpx<T> e = {(zk.x + zmk.x) * (T)0.5, (zk.y + zmk.y) * (T)0.5};
        const cpx<T> dd = csub(zk, zmk);
        const cpx<T> o = {dd.y * (T)0.5, -dd.x * (T)0.5};  // (zk - zmk) / (2i)
        cg[(size_t)line * Kz + k] = cadd(e, cmul(twpost[k], o));
    }
}

// 5. complex-to-real along z (unnormalised inverse).
template <typename T>
__global__ __launch_bounds__(kFFTThreads) void k_fft_z_c2r(const cpx<T>* __restrict__ cg, T* __restrict__ grid,
                                                           int nlines, int Izs, int Kz, int W, FFTDev f,
                                                           const cpx<T>* __restrict__ tw,
                                                           const cpx<T>* __restrict__ twpost) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = f.n;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (m + 1) * W;
    const int line0 = blockIdx.x * W;
    for (int idx = threadIdx.x; idx < (m + 1) * W; idx += blockDim.x) {
        const int w = idx / (m + 1), k = idx % (m + 1), line = line0 + w;
        B[k * W + w] = (line < nlines) ? cg[(size_t)line * Kz + k] : cpx<T>{0, 0};
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * W; idx += blockDim.x) {
        const int w = idx % W, k = idx / W;
        const cpx<T> xk = B[k * W + w];
        const cpx<T> xmk = cconj(B[(m - k) * W + w]);
        const cpx<T> e = cadd(xk, xmk);
        const cpx<T> o = cmulc(csub(xk, xmk), twpost[k]);  // times e^{+2 pi i k / I_z*}
        A[k * W + w] = cpx<T>{e.x - o.y, e.y + o.x};        // e + i o
    }
    __syncthreads();
    cpx<T>* z = lds_fft(A, B, W, f, tw, +1);
    for (int idx = threadIdx.x; idx < m * W; idx += blockDim.x) {
        const int w = idx / m, t = idx % m, line = line0 + w;
        if (line >= nlines) continue;
        const cpx<T> v = z[t * W + w];
        T* row = grid + (size_t)line * Izs;
        row[2 * t] = v.x;
        row[2 * t + 1] = v.y;
    }
}

// 2./4. complex FFT along y for (x, a batch of W consecutive k_z)
template <typename T>
__global__ __launch_bounds__(kFFTThreads) void k_fft_y(cpx<T>* __restrict__ cg, int Ix, int Iy, int Kz, int W,
                                                       FFTDev f, const cpx<T>* __restrict__ tw, int sign) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + Iy * W;
    const int nkb = (Kz + W - 1) / W;
    const int ix = blockIdx.x / nkb, kz0 = (blockIdx.x % nkb) * W;
    if (ix >= Ix) return;
    cpx<T>* base = cg + (size_t)ix * Iy * Kz + kz0;
    for (int idx = threadIdx.x; idx < Iy * W; idx += blockDim.x) {
        const int w = idx % W, iy = idx / W;
        A[iy * W + w] = (kz0 + w < Kz) ? base[(size_t)iy * Kz + w] : cpx<T>{0, 0};
    }
    __syncthreads();
    cpx<T>* res = lds_fft(A, B, W, f, tw, sign);
    for (int idx = threadIdx.x; idx < Iy * W; idx += blockDim.x) {
        const int w = idx % W, iy = idx / W;
        if (kz0 + w < Kz) base[(size_t)iy * Kz + w] = res[iy * W + w];
    }
}

// 3. forward FFT along x, the SOG multiplier, inverse FFT along x
template <typename T>
__global__ __launch_bounds__(kFFTThreads) void k_fft_x_scale(cpx<T>* __restrict__ cg, int Ix, int Iy, int Kz, int W,
                                                             FFTDev f, const cpx<T>* __restrict__ tw, int nl,
                                                             const T* __restrict__ ax, const T* __restrict__ ay,
                                                             const T* __restrict__ az, const T* __restrict__ cl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + Ix * W;
    T* cyz = reinterpret_cast<T*>(B + Ix * W);  // nl x W
    const int nkb = (Kz + W - 1) / W;
    const int iy = blockIdx.x / nkb, kz0 = (blockIdx.x % nkb) * W;
    if (iy >= Iy) return;
    const size_t stride = (size_t)Iy * Kz;
    cpx<T>* base = cg + (size_t)iy * Kz + kz0;
    for (int idx = threadIdx.x; idx < Ix * W; idx += blockDim.x) {
        const int w = idx % W, ix = idx / W;
        A[ix * W + w] = (kz0 + w < Kz) ? base[ix * stride + w] : cpx<T>{0, 0};
    }
    for (int idx = threadIdx.x; idx < nl * W; idx += blockDim.x) {
        const int w = idx % W, l = idx / W;
        const int kz = min(kz0 + w, Kz - 1);
        cyz[l * W + w] = cl[l] * ay[l * Iy + iy] * az[l * Kz + kz];
    }
    __syncthreads();
    cpx<T>* res = lds_fft(A, B, W, f, tw, -1);
    for (int idx = threadIdx.x; idx < Ix * W; idx += blockDim.x) {
        const int w = idx % W, ix = idx / W;
        T mlt = 0;
        for (int l = 0; l < nl; ++l) mlt += ax[l * Ix + ix] * cyz[l * W + w];
        cpx<T> v = res[ix * W + w];
        v.x *= mlt;
        v.y *= mlt;
        res[ix * W + w] = v;
    }
    __syncthreads();
    cpx<T>* other = (res == A) ? B : A;
    cpx<T>* out = lds_fft(res, other, W, f, tw, +1);
    for (int idx = threadIdx.x; idx < Ix * W; idx += blockDim.x) {
        const int w = idx % W, ix = idx / W;
        if (kz0 + w < Kz) base[ix * stride + w] = out[ix * W + w];
    }
}

// Generic batched line transform: W consecutive lines per block; line l starts at
// (l / ncols) * outer_stride + (l % ncols) * col_stride, elements at elem_stride.
// Lines adjacent in memory (col_stride == 1) load and store coalesced.
template <typename T>
__global__ __launch_bounds__(kFFTThreads) void k_fft_lines(cpx<T>* __restrict__ d, int nlines, int ncols,
                                                           size_t outer_stride, size_t col_stride, size_t elem_stride,
                                                           int W, FFTDev f, const cpx<T>* __restrict__ tw, int sign) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = f.n;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + n * W;
    const int line0 = blockIdx.x * W;
    for (int idx = threadIdx.x; idx < n * W; idx += blockDim.x) {
        const int w = idx % W, e = idx / W, line = line0 + w;
        cpx<T> v = {0, 0};
        if (line < nlines) v = d[(size_t)(line / ncols) * outer_stride + (size_t)(line % ncols) * col_stride + (size_t)e * elem_stride];
        A[e * W + w] = v;
    }
    __syncthreads();
    cpx<T>* res = lds_fft(A, B, W, f, tw, sign);
    for (int idx = threadIdx.x; idx < n * W; idx += blockDim.x) {
        const int w = idx % W, e = idx / W, line = line0 + w;
        if (line < nlines)
            d[(size_t)(line / ncols) * outer_stride + (size_t)(line % ncols) * col_stride + (size_t)e * elem_stride] = res[e * W + w];
    }
}

int batch_for(int n, size_t elem, size_t extra_per_line, size_t budget) {
    int W = 16;
    while (W > 1 && (2 * (size_t)n * elem + extra_per_line) * W > budget) W >>= 1;
    return W;
}

template <typename T>
hipError_t run_fft_mid(Plan& p) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int Ix = r.I[0], Iy = r.I[1], Izs = r.Izs, Kz = Izs / 2 + 1, m = Izs / 2;
    const int nlines = Ix * Iy;
    const size_t ce = sizeof(cpx<T>);
    const size_t budget = 65536;
    const int nl = r.m + 1;
    hipError_t e;
    // 1. z forward
    {
        int W = 16;
        while (W > 1 && 2 * (size_t)(m + 1) * ce * W > budget) W >>= 1;
        size_t lds = 2 * (size_t)(m + 1) * ce * W;
        if (lds > budget) return hipErrorInvalidConfiguration;
        int t = timer_id(p, "fft_z_fwd");
        timer_begin(p, t);
        k_fft_z_r2c<T><<<(nlines + W - 1) / W, kFFTThreads, lds, p.stream>>>(
            (const T*)ws.grid, (cpx<T>*)ws.cgrid, nlines, Izs, Kz, W, to_dev(p.fz), (const cpx<T>*)ws.tw_z,
            (const cpx<T>*)ws.tw_zpost);
        timer_end(p, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 2. y forward
    int Wy = batch_for(Iy, ce, 0, budget);
    size_t ldsy = 2 * (size_t)Iy * ce * Wy;
    if (ldsy > budget) return hipErrorInvalidConfiguration;
    int nby = Ix * ((Kz + Wy - 1) / Wy);
    {
        int t = timer_id(p, "fft_y_fwd");
        timer_begin(p, t);
        k_fft_y<T><<<nby, kFFTThreads, ldsy, p.stream>>>((cpx<T>*)ws.cgrid, Ix, Iy, Kz, Wy, to_dev(p.fy),
                                                         (const cpx<T>*)ws.tw_y, -1);
        timer_end(p, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 3. x forward, scale, x inverse
    {
        int W = batch_for(Ix, ce, (size_t)nl * sizeof(T), budget);
        size_t lds = (2 * (size_t)Ix * ce + (size_t)nl * sizeof(T)) * W;
        if (lds > budget) return hipErrorInvalidConfiguration;
        int nb = Iy * ((Kz + W - 1) / W);
        int t = timer_id(p, "fft_x_scale");
        timer_begin(p, t);
        k_fft_x_scale<T><<<nb, kFFTThreads, lds, p.stream>>>((cpx<T>*)ws.cgrid, Ix, Iy, Kz, W, to_dev(p.fx),
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
        k_fft_y<T><<<nby, kFFTThreads, ldsy, p.stream>>>((cpx<T>*)ws.cgrid, Ix, Iy, Kz, Wy, to_dev(p.fy),
                                                         (const cpx<T>*)ws.tw_y, +1);
        timer_end(p, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 5. z inverse
    {
        int W = 16;
        while (W > 1 && 2 * (size_t)(m + 1) * ce * W > budget) W >>= 1;
        size_t lds = 2 * (size_t)(m + 1) * ce * W;
        if (lds > budget) return hipErrorInvalidConfiguration;
        int t = timer_id(p, "fft_z_inv");
        timer_begin(p, t);
        k_fft_z_c2r<T><<<(nlines + W - 1) / W, kFFTThreads, lds, p.stream>>>(
            (const cpx<T>*)ws.cgrid, (T*)ws.grid, nlines, Izs, Kz, W, to_dev(p.fz), (const cpx<T>*)ws.tw_z,
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
    while (W > 1 && 2 * (size_t)f.n * ce * W > 65536) W >>= 1;
    const size_t lds = 2 * (size_t)f.n * ce * W;
    if (lds > 65536 || nlines <= 0) return hipErrorInvalidConfiguration;
    const int nb = (nlines + W - 1) / W;
    if (f64)
        k_fft_lines<double><<<nb, kFFTThreads, lds, p.stream>>>((cpx<double>*)data, nlines, ncols, outer_stride, col_stride,
                                                               elem_stride, W, to_dev(f), (const cpx<double>*)tw, sign);
    else
        k_fft_lines<float><<<nb, kFFTThreads, lds, p.stream>>>((cpx<float>*)data, nlines, ncols, outer_stride, col_stride,
                                                              elem_stride, W, to_dev(f), (const cpx<float>*)tw, sign);
    return hipGetLastError();
}

hipError_t launch_fft_mid(Plan& p) {
    if (p.r.prec == SOG_PREC_FP64) return run_fft_mid<double>(p);
    return run_fft_mid<float>(p);
}

}  // namespace sog
