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
#include "launch.hpp"

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

// cos and sin of 2 pi q / R for the radices of the small DFTs (the doubles nearest the
// exact values; q taken mod R)
__host__ __device__ constexpr double rot_c(int R, int q) {
    q = ((q % R) + R) % R;
    if (R == 3) return q == 0 ? 1.0 : q == 1 ? -0.5 : -0.5;
    if (R == 5) return q == 0 ? 1.0 : q == 1 ? 0.30901699437494745 : q == 2 ? -0.8090169943749475 : q == 3 ? -0.8090169943749475 : 0.30901699437494745;
    if (R == 6) return q == 0 ? 1.0 : q == 1 ? 0.5 : q == 2 ? -0.5 : q == 3 ? -1.0 : q == 4 ? -0.5 : 0.5;
    if (R == 7) return q == 0 ? 1.0 : q == 1 ? 0.6234898018587335 : q == 2 ? -0.2225209339563144 : q == 3 ? -0.9009688679024191 : q == 4 ? -0.9009688679024191 : q == 5 ? -0.2225209339563144 : 0.6234898018587335;
    if (R == 8) return q == 0 ? 1.0 : q == 1 ? 0.7071067811865476 : q == 2 ? 0.0 : q == 3 ? -0.7071067811865476 : q == 4 ? -1.0 : q == 5 ? -0.7071067811865476 : q == 6 ? 0.0 : 0.7071067811865476;
    if (R == 9) return q == 0 ? 1.0 : q == 1 ? 0.766044443118978 : q == 2 ? 0.17364817766693036 : q == 3 ? -0.5 : q == 4 ? -0.9396926207859084 : q == 5 ? -0.9396926207859084 : q == 6 ? -0.5 : q == 7 ? 0.17364817766693036 : 0.766044443118978;
    if (R == 10) return q == 0 ? 1.0 : q == 1 ? 0.8090169943749475 : q == 2 ? 0.30901699437494745 : q == 3 ? -0.30901699437494745 : q == 4 ? -0.8090169943749475 : q == 5 ? -1.0 : q == 6 ? -0.8090169943749475 : q == 7 ? -0.30901699437494745 : q == 8 ? 0.30901699437494745 : 0.8090169943749475;
    if (R == 12) return q == 0 ? 1.0 : q == 1 ? 0.8660254037844386 : q == 2 ? 0.5 : q == 3 ? 0.0 : q == 4 ? -0.5 : q == 5 ? -0.8660254037844386 : q == 6 ? -1.0 : q == 7 ? -0.8660254037844386 : q == 8 ? -0.5 : q == 9 ? 0.0 : q == 10 ? 0.5 : 0.8660254037844386;
    if (R == 15) return q == 0 ? 1.0 : q == 1 ? 0.9135454576426009 : q == 2 ? 0.6691306063588582 : q == 3 ? 0.30901699437494745 : q == 4 ? -0.10452846326765347 : q == 5 ? -0.5 : q == 6 ? -0.8090169943749475 : q == 7 ? -0.9781476007338057 : q == 8 ? -0.9781476007338057 : q == 9 ? -0.8090169943749475 : q == 10 ? -0.5 : q == 11 ? -0.10452846326765347 : q == 12 ? 0.30901699437494745 : q == 13 ? 0.6691306063588582 : 0.9135454576426009;
    if (R == 16) return q == 0 ? 1.0 : q == 1 ? 0.9238795325112867 : q == 2 ? 0.7071067811865476 : q == 3 ? 0.3826834323650898 : q == 4 ? 0.0 : q == 5 ? -0.3826834323650898 : q == 6 ? -0.7071067811865476 : q == 7 ? -0.9238795325112867 : q == 8 ? -1.0 : q == 9 ? -0.9238795325112867 : q == 10 ? -0.7071067811865476 : q == 11 ? -0.3826834323650898 : q == 12 ? 0.0 : q == 13 ? 0.3826834323650898 : q == 14 ? 0.7071067811865476 : 0.9238795325112867;
    return 0.0;
}
__host__ __device__ constexpr double rot_s(int R, int q) {
    q = ((q % R) + R) % R;
    if (R == 3) return q == 0 ? 0.0 : q == 1 ? 0.8660254037844386 : -0.8660254037844386;
    if (R == 5) return q == 0 ? 0.0 : q == 1 ? 0.9510565162951535 : q == 2 ? 0.5877852522924731 : q == 3 ? -0.5877852522924731 : -0.9510565162951535;
    if (R == 6) return q == 0 ? 0.0 : q == 1 ? 0.8660254037844386 : q == 2 ? 0.8660254037844386 : q == 3 ? 0.0 : q == 4 ? -0.8660254037844386 : -0.8660254037844386;
    if (R == 7) return q == 0 ? 0.0 : q == 1 ? 0.7818314824680298 : q == 2 ? 0.9749279121818236 : q == 3 ? 0.4338837391175581 : q == 4 ? -0.4338837391175581 : q == 5 ? -0.9749279121818236 : -0.7818314824680298;
    if (R == 8) return q == 0 ? 0.0 : q == 1 ? 0.7071067811865476 : q == 2 ? 1.0 : q == 3 ? 0.7071067811865476 : q == 4 ? 0.0 : q == 5 ? -0.7071067811865476 : q == 6 ? -1.0 : -0.7071067811865476;
    if (R == 9) return q == 0 ? 0.0 : q == 1 ? 0.6427876096865394 : q == 2 ? 0.984807753012208 : q == 3 ? 0.8660254037844386 : q == 4 ? 0.3420201433256687 : q == 5 ? -0.3420201433256687 : q == 6 ? -0.8660254037844386 : q == 7 ? -0.984807753012208 : -0.6427876096865394;
    if (R == 10) return q == 0 ? 0.0 : q == 1 ? 0.5877852522924731 : q == 2 ? 0.9510565162951535 : q == 3 ? 0.9510565162951535 : q == 4 ? 0.5877852522924731 : q == 5 ? 0.0 : q == 6 ? -0.5877852522924731 : q == 7 ? -0.9510565162951535 : q == 8 ? -0.9510565162951535 : -0.5877852522924731;
    if (R == 12) return q == 0 ? 0.0 : q == 1 ? 0.5 : q == 2 ? 0.8660254037844386 : q == 3 ? 1.0 : q == 4 ? 0.8660254037844386 : q == 5 ? 0.5 : q == 6 ? 0.0 : q == 7 ? -0.5 : q == 8 ? -0.8660254037844386 : q == 9 ? -1.0 : q == 10 ? -0.8660254037844386 : -0.5;
    if (R == 15) return q == 0 ? 0.0 : q == 1 ? 0.4067366430758002 : q == 2 ? 0.7431448254773942 : q == 3 ? 0.9510565162951535 : q == 4 ? 0.9945218953682733 : q == 5 ? 0.8660254037844386 : q == 6 ? 0.5877852522924731 : q == 7 ? 0.20791169081775934 : q == 8 ? -0.20791169081775934 : q == 9 ? -0.5877852522924731 : q == 10 ? -0.8660254037844386 : q == 11 ? -0.9945218953682733 : q == 12 ? -0.9510565162951535 : q == 13 ? -0.7431448254773942 : -0.4067366430758002;
    if (R == 16) return q == 0 ? 0.0 : q == 1 ? 0.3826834323650898 : q == 2 ? 0.7071067811865476 : q == 3 ? 0.9238795325112867 : q == 4 ? 1.0 : q == 5 ? 0.9238795325112867 : q == 6 ? 0.7071067811865476 : q == 7 ? 0.3826834323650898 : q == 8 ? 0.0 : q == 9 ? -0.3826834323650898 : q == 10 ? -0.7071067811865476 : q == 11 ? -0.9238795325112867 : q == 12 ? -1.0 : q == 13 ? -0.9238795325112867 : q == 14 ? -0.7071067811865476 : -0.3826834323650898;
    return 0.0;
}

template <typename T, int R, int SIGN>
__device__ __forceinline__ void small_dft(const cpx<T> (&v)[R], cpx<T> (&o)[R]);

// x e^{SIGN 2 pi i q / R} for a constant q; the factors 1, -1 and +-i cost nothing
template <typename T, int R, int SIGN>
__device__ __forceinline__ cpx<T> twiddle_const(cpx<T> x, int q) {
    q %= R;
    if (q == 0) return x;
    if (2 * q == R) return cpx<T>{-x.x, -x.y};
    if (4 * q == R) return (SIGN > 0) ? cpx<T>{-x.y, x.x} : cpx<T>{x.y, -x.x};
    if (4 * q == 3 * R) return (SIGN > 0) ? cpx<T>{x.y, -x.x} : cpx<T>{-x.y, x.x};
    const T c = (T)rot_c(R, q), sn = (T)SIGN * (T)rot_s(R, q);
    return cpx<T>{x.x * c - x.y * sn, x.x * sn + x.y * c};
}

// DFT of length R = R1 R2 in registers (Cooley-Tukey): inner DFTs of length R1 over the
// inputs n = R2 n1 + n2, the twiddles e^{SIGN 2 pi i n2 k1 / R}, outer DFTs of length R2;
// output k = k1 + R1 k2
template <typename T, int R1, int R2, int SIGN>
__device__ __forceinline__ void composite_dft(const cpx<T> (&v)[R1 * R2], cpx<T> (&o)[R1 * R2]) {
    constexpr int R = R1 * R2;
    cpx<T> a[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        cpx<T> in[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) in[n1] = v[R2 * n1 + n2];
        small_dft<T, R1, SIGN>(in, a[n2]);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) a[n2][k1] = twiddle_const<T, R, SIGN>(a[n2][k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        cpx<T> in[R2], out[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) in[n2] = a[n2][k1];
        small_dft<T, R2, SIGN>(in, out);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) o[k1 + R1 * k2] = out[k2];
    }
}

// o_p = sum_r v_r e^{SIGN 2 pi i p r / R}
template <typename T, int R, int SIGN>
__device__ __forceinline__ void small_dft(const cpx<T> (&v)[R], cpx<T> (&o)[R]) {
    if constexpr (R == 6) {
        composite_dft<T, 2, 3, SIGN>(v, o);
    } else if constexpr (R == 8) {
        composite_dft<T, 2, 4, SIGN>(v, o);
    } else if constexpr (R == 9) {
        composite_dft<T, 3, 3, SIGN>(v, o);
    } else if constexpr (R == 10) {
        composite_dft<T, 2, 5, SIGN>(v, o);
    } else if constexpr (R == 16) {
        composite_dft<T, 4, 4, SIGN>(v, o);
    } else if constexpr (R == 2) {
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
// bounds the butterflies a thread holds in registers during a stage and the elements it
// holds while a batch moves between HBM and LDS.
template <typename T>
constexpr int kFFTCap = (sizeof(T) == 4) ? 4608 : 2304;  // 18 / 9 elements per thread
constexpr int kFFTThreads = 256;
static_assert(kFFTCap<float> == fft_max_line(SOG_PREC_FP32_BULK) && kFFTCap<double> == fft_max_line(SOG_PREC_FP64),
              "the planner's line limit is the batch capacity");
template <typename T>
constexpr int kStageK = kFFTCap<T> / kFFTThreads;

// e / d for 0 <= e < 2^16, 2 <= d < 2^16: multiply-high by ceil(2^32 / d) (exact while
// e d < 2^32)
struct UDiv {
    int d;
    unsigned mul;
};
UDiv make_udiv(int d) { return UDiv{d, (unsigned)((((uint64_t)1 << 32) + (uint64_t)d - 1) / (uint64_t)d)}; }
__device__ __forceinline__ int udiv(int e, UDiv u) { return (int)__umulhi((unsigned)e, u.mul); }

// dst[i] = src[i] for i < count, with up to K loads of a thread in flight together (every
// slot loads a valid element, so the staging array stays in registers)
template <int K, typename V>
__device__ __forceinline__ void copy_in(V* dst, const V* __restrict__ src, int count) {
    for (int b = 0; b < count; b += K * kFFTThreads) {
        V v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = src[min(b + (int)threadIdx.x + k * kFFTThreads, count - 1)];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = b + threadIdx.x + k * kFFTThreads;
            if (i < count) dst[i] = v[k];
        }
    }
}

// Moves the E <= kFFTCap elements of a batch from HBM into LDS.  Each thread issues all
// its loads before its first LDS write, so a block waits for one round trip, not one per
// element row; side() runs between the loads and the writes (small table copies whose
// loads then overlap the batch's).  Element e is src(e) and lands at A[dst(e)].
template <typename T, class Src, class Dst, class Side>
__device__ __forceinline__ void stage_in(cpx<T>* A, int E, Src src, Dst dst, Side side) {
    constexpr int K = kStageK<T>;
    cpx<T> v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = threadIdx.x + k * kFFTThreads;
        if (e < E) v[k] = src(e);
    }
    side();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = threadIdx.x + k * kFFTThreads;
        if (e < E) A[dst(e)] = v[k];
    }
}

// One Stockham stage of radix R, in place on A (element i of line w at A[i P + w], the
// row pitch P >= W):
// every thread first reads all the butterflies it owns into registers, the block
// synchronises, then the results are written back.  twl: the twiddles e^{-2 pi i t/n}.
template <typename T, int R, int SIGN>
__device__ __forceinline__ void fft_stage(cpx<T>* A, const cpx<T>* __restrict__ twl, int W, int lw, int P, int nR,
                                          int Ns, unsigned mNs, int tws) {
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
            for (int r = 0; r < R; ++r) v[r] = A[(j + r * nR) * P + w];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cpx<T> t = twl[k * r * tws];
                    if (SIGN > 0) t.y = -t.y;
                    v[r] = cmul(v[r], t);
                }
            }
            small_dft<T, R, SIGN>(v, o[b]);
            dst[b] = (g * Ns * R + k) * P + w;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b)
        if (dst[b] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) A[dst[b] + r * Ns * P] = o[b][r];
        }
    __syncthreads();
}

// In-LDS transform of W interleaved lines (W a power of two, n W <= kFFTCap; element i
// of line w at A[i P + w]).  The caller synchronises before (data in A) and may read A
// after the return.  Inlined (called, it costs its caller the calling convention's
// registers).
template <typename T, int SIGN>
__device__ __forceinline__ void lds_fft(cpx<T>* A, const cpx<T>* __restrict__ twl, int W, int P, const FFTDev& f) {
    const int lw = __ffs(W) - 1;
    for (int s = 0; s < f.nstages; ++s) {
        switch (f.radix[s]) {
            case 4: fft_stage<T, 4, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 2: fft_stage<T, 2, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 3: fft_stage<T, 3, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 5: fft_stage<T, 5, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 6: fft_stage<T, 6, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 8: fft_stage<T, 8, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 9: fft_stage<T, 9, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 10: fft_stage<T, 10, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            case 16: fft_stage<T, 16, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
            default: fft_stage<T, 7, SIGN>(A, twl, W, lw, P, f.nR[s], f.Ns[s], f.mNs[s], f.tws[s]); break;
        }
    }
}

// lines per block: a power of two, n W <= kFFTCap, at most 16
template <typename T>
int lines_per_block(int n) {
    return fft_lines_per_batch(sizeof(T) == 8 ? SOG_PREC_FP64 : SOG_PREC_FP32_BULK, n);
}

// 1. real-to-complex along z for W lines per block.  m = I_z*/2 packed pairs per line;
// only the pairs [t0, t0 + span) can be nonzero (the planes windows reach), the others
// are zero rows of the batch.  LDS rows have pitch W + 1, so the line-to-row transpose of
// the load and the k-ordered reads of the split hit distinct banks.
template <typename T>
struct FFTZr2cK {
    static constexpr int kThreads = kFFTThreads;
    __device__ static void run(GridPos gpos, const T* __restrict__ grid, cpx<T>* __restrict__ cg, int nlines, int Izs, int Kzs, int W, int t0, UDiv span, UDiv m1, const FFTDev& f, const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ twpost) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = f.n, P = W + 1, lw = __ffs(W) - 1;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);  // (m + 1) rows of pitch P
    cpx<T>* twl = A + (m + 1) * P;                     // m
    cpx<T>* tpl = twl + m;                             // m + 1
    const int line0 = gpos.bid * W;
    const size_t hz = (size_t)(Izs / 2);
    const cpx<T>* rows = reinterpret_cast<const cpx<T>*>(grid);
    for (int idx = threadIdx.x; idx < (m - span.d) * W; idx += kFFTThreads) {
        const int rr = idx >> lw, w = idx & (W - 1);
        A[(rr < t0 ? rr : rr + span.d) * P + w] = cpx<T>{0, 0};
    }
    stage_in<T>(A, span.d * W,
                [&](int e) {
                    const int w = udiv(e, span);
                    return rows[(size_t)min(line0 + w, nlines - 1) * hz + t0 + (e - w * span.d)];
                },
                [&](int e) {
                    const int w = udiv(e, span);
                    return (t0 + e - w * span.d) * P + w;
                },
                [&] {
                    copy_in<4>(twl, tw, m);
                    copy_in<4>(tpl, twpost, m + 1);
                });
    __syncthreads();
    lds_fft<T, -1>(A, twl, W, P, f);
    // half spectrum k = 0..m of each line, k fastest
    for (int e = threadIdx.x; e < m1.d * W; e += kFFTThreads) {
        const int w = udiv(e, m1), k = e - w * m1.d;
        const int line = line0 + w;
        if (line >= nlines) break;  // e grows: every later element is past nlines too
        const cpx<T> zk = A[(k == m ? 0 : k) * P + w];
        const cpx<T> zmk = cconj(A[(k == 0 ? 0 : m - k) * P + w]);
        const cpx<T> ev = {(zk.x + zmk.x) * (T)0.5, (zk.y + zmk.y) * (T)0.5};
        const cpx<T> dd = csub(zk, zmk);
        const cpx<T> od = {dd.y * (T)0.5, -dd.x * (T)0.5};  // (zk - zmk) / (2i)
        cg[(size_t)line * Kzs + k] = cadd(ev, cmul(tpl[k], od));
    }
}
};

// Z_k of the packed inverse from X_k and conj X_{m-k}: (X_k + conj X_{m-k}) + i (X_k -
// conj X_{m-k}) e^{+2 pi i k / I_z*}
template <typename T>
__device__ __forceinline__ cpx<T> c2r_pre(cpx<T> xk, cpx<T> xmkc, cpx<T> tp) {
    const cpx<T> ev = cadd(xk, xmkc);
    const cpx<T> od = cmulc(csub(xk, xmkc), tp);
    return cpx<T>{ev.x - od.y, ev.y + od.x};
}

// 5. complex-to-real along z (unnormalised inverse); only the pairs [t0, t0 + span) are
// stored (the planes the gathering reads).
template <typename T>
struct FFTZc2rK {
    static constexpr int kThreads = kFFTThreads;
    __device__ static void run(GridPos gpos, const cpx<T>* __restrict__ cg, T* __restrict__ grid, int nlines, int Izs, int Kzs, int W, int t0, UDiv span, UDiv m1, const FFTDev& f, const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ twpost) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = f.n, P = W + 1, lw = __ffs(W) - 1;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* twl = A + (m + 1) * P;
    cpx<T>* tpl = twl + m;
    const int line0 = gpos.bid * W;
    const size_t hz = (size_t)(Izs / 2);
    stage_in<T>(A, m1.d * W,
                [&](int e) {
                    const int w = udiv(e, m1);
                    return cg[(size_t)min(line0 + w, nlines - 1) * Kzs + (e - w * m1.d)];
                },
                [&](int e) {
                    const int w = udiv(e, m1);
                    return (e - w * m1.d) * P + w;
                },
                [&] {
                    copy_in<4>(twl, tw, m);
                    copy_in<4>(tpl, twpost, m + 1);
                });
    __syncthreads();
    // in place, pair (k, m - k) by one thread; row m holds X_m, the partner of k = 0
    for (int idx = threadIdx.x; idx < (m / 2 + 1) * W; idx += kFFTThreads) {
        const int k = idx >> lw, w = idx & (W - 1);
        const cpx<T> a = A[k * P + w], b = A[(m - k) * P + w];
        A[k * P + w] = c2r_pre(a, cconj(b), tpl[k]);
        if (k > 0 && 2 * k != m) A[(m - k) * P + w] = c2r_pre(b, cconj(a), tpl[m - k]);
    }
    __syncthreads();
    lds_fft<T, +1>(A, twl, W, P, f);
    cpx<T>* rows = reinterpret_cast<cpx<T>*>(grid);
    for (int e = threadIdx.x; e < span.d * W; e += kFFTThreads) {
        const int w = udiv(e, span), t = t0 + e - w * span.d;
        const int line = line0 + w;
        if (line >= nlines) break;
        rows[(size_t)line * hz + t] = A[t * P + w];
    }
}
};

// 2./4. complex FFT along y for (x, a batch of W consecutive k_z)
template <typename T, int SIGN>
struct FFTYK {
    static constexpr int kThreads = kFFTThreads;
    __device__ static void run(GridPos gpos, cpx<T>* __restrict__ cg, int Ix, int Iy, int Kz, int Kzs, int W, const FFTDev& f, const cpx<T>* __restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* twl = A + Iy * W;
    const int nkb = (Kz + W - 1) / W;
    const int ix = gpos.bid / nkb, kz0 = (gpos.bid % nkb) * W;
    if (ix >= Ix) return;
    const int lw = __ffs(W) - 1;
    cpx<T>* base = cg + (size_t)ix * Iy * Kzs + kz0;
    const int nw = min(W, Kz - kz0);
    stage_in<T>(A, Iy * W,
                [&](int e) {
                    const int w = e & (W - 1);
                    return (w < nw) ? base[(size_t)(e >> lw) * Kzs + w] : cpx<T>{0, 0};
                },
                [&](int e) { return e; }, [&] { copy_in<4>(twl, tw, Iy); });
    __syncthreads();
    lds_fft<T, SIGN>(A, twl, W, W, f);
    for (int idx = threadIdx.x; idx < Iy * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), iy = idx >> lw;
        if (w < nw) base[(size_t)iy * Kzs + w] = A[idx];
    }
}
};

// 3. forward FFT along x, the SOG multiplier, inverse FFT along x.  The multiplier is
// sum_l c_l ax_l(k_x) ay_l(k_y) az_l(k_z): the block's (k_y, k_z) factors are staged in
// LDS, and ax too when it fits (AXLDS); otherwise ax is read from global memory (L2).
template <typename T, bool AXLDS>
struct FFTXScaleK {
    static constexpr int kThreads = kFFTThreads;
    __device__ static void run(GridPos gpos, cpx<T>* __restrict__ cg, int Ix, int Iy, int Kz, int Kzs, int W, const FFTDev& f, const cpx<T>* __restrict__ tw, int nl, const T* __restrict__ ax, const T* __restrict__ ay, const T* __restrict__ az, const T* __restrict__ cl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* twl = A + Ix * W;
    T* cyz = reinterpret_cast<T*>(twl + Ix);  // nl x W
    T* axl = cyz + nl * W;                    // AXLDS: nl x Ix, then kStageK (256 / W) - Ix zeros
    const int nkb = (Kz + W - 1) / W;
    const int iy = gpos.bid / nkb, kz0 = (gpos.bid % nkb) * W;
    if (iy >= Iy) return;
    const int lw = __ffs(W) - 1;
    const size_t stride = (size_t)Iy * Kzs;
    cpx<T>* base = cg + (size_t)iy * Kzs + kz0;
    const int nw = min(W, Kz - kz0);
    stage_in<T>(A, Ix * W,
                [&](int e) {
                    const int w = e & (W - 1);
                    return (w < nw) ? base[(size_t)(e >> lw) * stride + w] : cpx<T>{0, 0};
                },
                [&](int e) { return e; },
                [&] {
                    copy_in<4>(twl, tw, Ix);
                    if constexpr (AXLDS) {
                        copy_in<16>(axl, ax, nl * Ix);
                        for (int i = threadIdx.x; i < kStageK<T> * (kFFTThreads >> lw) - Ix; i += kFFTThreads)
                            axl[nl * Ix + i] = 0;
                    }
                    for (int idx = threadIdx.x; idx < nl * W; idx += kFFTThreads) {
                        const int w = idx & (W - 1), l = idx >> lw;
                        const int kz = min(kz0 + w, Kz - 1);
                        cyz[idx] = cl[l] * ay[l * Iy + iy] * az[l * Kz + kz];
                    }
                });
    __syncthreads();
    lds_fft<T, -1>(A, twl, W, W, f);
    {
        // a thread's elements share one k_z (256 is a multiple of W): per Gaussian one read
        // of its (k_y, k_z) factor, then one read and FMA per element (the table of ax is
        // followed by K 256 / W - I_x zeros, so the unused tail elements read inside it)
        constexpr int K = kStageK<T>;
        const int w = threadIdx.x & (W - 1), ix0 = threadIdx.x >> lw, dix = kFFTThreads >> lw;
        T mlt[K];
#pragma unroll
        for (int k = 0; k < K; ++k) mlt[k] = 0;
        for (int l = 0; l < nl; ++l) {
            const T c = cyz[l * W + w];
            if constexpr (AXLDS) {
                const T* ar = axl + l * Ix + ix0;
#pragma unroll
                for (int k = 0; k < K; ++k) mlt[k] += ar[k * dix] * c;
            } else {
                const T* ar = ax + (size_t)l * Ix;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int ix = ix0 + k * dix;
                    mlt[k] += (ix < Ix ? ar[ix] : (T)0) * c;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = threadIdx.x + k * kFFTThreads;
            if (idx < Ix * W) {
                cpx<T> v = A[idx];
                v.x *= mlt[k];
                v.y *= mlt[k];
                A[idx] = v;
            }
        }
    }
    __syncthreads();
    lds_fft<T, +1>(A, twl, W, W, f);
    for (int idx = threadIdx.x; idx < Ix * W; idx += kFFTThreads) {
        const int w = idx & (W - 1), ix = idx >> lw;
        if (w < nw) base[(size_t)ix * stride + w] = A[idx];
    }
}
};

template <typename T>
hipError_t run_fft_mid(Plan& p) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int Ix = r.I[0], Iy = r.I[1], Izs = r.Izs, Kz = Izs / 2 + 1, m = Izs / 2, Kzs = cgrid_stride(Izs);
    const int nlines = Ix * Iy;
    const size_t ce = sizeof(cpx<T>);
    const size_t budget = kFFTLdsBudget;
    const int nl = r.m + 1;
    hipError_t e;
    if ((size_t)m > (size_t)kFFTCap<T> || (size_t)Ix > (size_t)kFFTCap<T> || (size_t)Iy > (size_t)kFFTCap<T>)
        return hipErrorInvalidConfiguration;
    // 1. z forward: W lines per block, LDS rows of pitch W + 1 (plus row m) and the two
    // twiddle tables
    const int t0 = r.zband[0] / 2, span = (r.zband[1] - r.zband[0]) / 2;
    if (span < 2 || t0 + span > m) return hipErrorInvalidConfiguration;
    auto ldsz_of = [&](int w) { return ((size_t)(m + 1) * (w + 1) + 2 * (size_t)m + 1) * ce; };
    int Wz = lines_per_block<T>(m + 1);  // the inverse's batch holds rows 0..m
    while (Wz > 1 && ldsz_of(Wz) > budget) Wz >>= 1;
    const size_t ldsz = ldsz_of(Wz);
    if (ldsz > budget) return hipErrorInvalidConfiguration;
    {
        int t = timer_id(p, "fft_z_fwd");
        timer_begin(p, t);
        e = launch<FFTZr2cK<T>>(p, (nlines + Wz - 1) / Wz, ldsz, (const T*)ws.grid, (cpx<T>*)ws.cgrid, nlines, Izs, Kzs,
                                Wz, t0, make_udiv(span), make_udiv(m + 1), to_dev(p.fz), (const cpx<T>*)ws.tw_z,
                                (const cpx<T>*)ws.tw_zpost);
        timer_end(p, t);
        if (e != hipSuccess) return e;
    }
    // 2. y forward
    int Wy = lines_per_block<T>(Iy);
    while (Wy > 1 && (size_t)Iy * (Wy + 1) * ce > budget) Wy >>= 1;
    const size_t ldsy = (size_t)Iy * (Wy + 1) * ce;
    if (ldsy > budget) return hipErrorInvalidConfiguration;
    const int nby = Ix * ((Kz + Wy - 1) / Wy);
    {
        int t = timer_id(p, "fft_y_fwd");
        timer_begin(p, t);
        e = launch<FFTYK<T, -1>>(p, nby, ldsy, (cpx<T>*)ws.cgrid, Ix, Iy, Kz, Kzs, Wy, to_dev(p.fy),
                                 (const cpx<T>*)ws.tw_y);
        timer_end(p, t);
        if (e != hipSuccess) return e;
    }
    // 3. x forward, scale, x inverse
    {
        int W = lines_per_block<T>(Ix);
        static_assert(kFFTThreads == 256 && kFFTCap<T> == fft_max_line(sizeof(T) == 8 ? SOG_PREC_FP64 : SOG_PREC_FP32_BULK),
                      "fft_x_lds_bytes models this launch");
        const int prec = sizeof(T) == 8 ? SOG_PREC_FP64 : SOG_PREC_FP32_BULK;
        auto lds_of = [&](int w) { return fft_x_lds_bytes(prec, Ix, nl, w); };
        while (W > 1 && lds_of(W) > budget) W >>= 1;
        // the x multipliers stay in global memory when even one line per block leaves no
        // room for them in LDS
        const bool axlds = lds_of(W) <= budget;
        if (!axlds) {
            W = lines_per_block<T>(Ix);
            while (W > 1 && fft_x_lds_min_bytes(prec, Ix, nl, W) > budget) W >>= 1;
        }
        const size_t lds = axlds ? lds_of(W) : fft_x_lds_min_bytes(prec, Ix, nl, W);
        if (lds > budget) return hipErrorInvalidConfiguration;
        int nb = Iy * ((Kz + W - 1) / W);
        int t = timer_id(p, "fft_x_scale");
        timer_begin(p, t);
        if (axlds)
            e = launch<FFTXScaleK<T, true>>(p, nb, lds, (cpx<T>*)ws.cgrid, Ix, Iy, Kz, Kzs, W, to_dev(p.fx),
                                            (const cpx<T>*)ws.tw_x, nl, (const T*)ws.mult_ax, (const T*)ws.mult_ay,
                                            (const T*)ws.mult_az, (const T*)ws.mult_c);
        else
            e = launch<FFTXScaleK<T, false>>(p, nb, lds, (cpx<T>*)ws.cgrid, Ix, Iy, Kz, Kzs, W, to_dev(p.fx),
                                             (const cpx<T>*)ws.tw_x, nl, (const T*)ws.mult_ax, (const T*)ws.mult_ay,
                                             (const T*)ws.mult_az, (const T*)ws.mult_c);
        timer_end(p, t);
        if (e != hipSuccess) return e;
    }
    // 4. y inverse
    {
        int t = timer_id(p, "fft_y_inv");
        timer_begin(p, t);
        e = launch<FFTYK<T, +1>>(p, nby, ldsy, (cpx<T>*)ws.cgrid, Ix, Iy, Kz, Kzs, Wy, to_dev(p.fy),
                                 (const cpx<T>*)ws.tw_y);
        timer_end(p, t);
        if (e != hipSuccess) return e;
    }
    // 5. z inverse
    {
        int t = timer_id(p, "fft_z_inv");
        timer_begin(p, t);
        e = launch<FFTZc2rK<T>>(p, (nlines + Wz - 1) / Wz, ldsz, (const cpx<T>*)ws.cgrid, (T*)ws.grid, nlines, Izs, Kzs,
                                Wz, t0, make_udiv(span), make_udiv(m + 1), to_dev(p.fz), (const cpx<T>*)ws.tw_z,
                                (const cpx<T>*)ws.tw_zpost);
        timer_end(p, t);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

namespace {

// The 2D transforms of the long range's FFT form on `planes` planes of I2x x I2y reals
// (y fastest): forward (sign < 0) real-to-complex along y (the z pass's kernel on lines of
// I2y reals, every pair nonzero), then complex along x (the y pass's kernel with the
// planes as its outer index); inverse (sign > 0) the reverse, unnormalised.  Half
// spectrum: planes of I2x rows of Ky = I2y/2 + 1 complex, row stride cgrid_stride(I2y).
template <typename T>
hipError_t run_fft_long2(Plan& p, int sign, int planes) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int Ix = r.I2[0], Iy = r.I2[1], m = Iy / 2, Ky = m + 1, Kys = cgrid_stride(Iy);
    const int nlines = planes * Ix;
    const size_t ce = sizeof(cpx<T>);
    const size_t budget = kFFTLdsBudget;
    if (planes < 1 || (Iy & 1) || m < 2 || (size_t)m > (size_t)kFFTCap<T> || (size_t)Ix > (size_t)kFFTCap<T> ||
        p.f2y.n != m || p.f2x.n != Ix)
        return hipErrorInvalidConfiguration;
    auto ldsz_of = [&](int w) { return ((size_t)(m + 1) * (w + 1) + 2 * (size_t)m + 1) * ce; };
    int Wz = lines_per_block<T>(m + 1);
    while (Wz > 1 && ldsz_of(Wz) > budget) Wz >>= 1;
    const size_t ldsz = ldsz_of(Wz);
    int Wx = lines_per_block<T>(Ix);
    while (Wx > 1 && (size_t)Ix * (Wx + 1) * ce > budget) Wx >>= 1;
    const size_t ldsx = (size_t)Ix * (Wx + 1) * ce;
    if (ldsz > budget || ldsx > budget) return hipErrorInvalidConfiguration;
    const int nbx = planes * ((Ky + Wx - 1) / Wx);
    T* grid = (T*)ws.l2_grid;
    cpx<T>* cg = (cpx<T>*)ws.l2_cgrid;
    const cpx<T>* twy = (const cpx<T>*)ws.l2_tw_y;
    const cpx<T>* twp = (const cpx<T>*)ws.l2_tw_ypost;
    const cpx<T>* twx = (const cpx<T>*)ws.l2_tw_x;
    hipError_t e = hipSuccess;
    if (sign < 0) {
        int t = timer_id(p, "long2_fft_y_fwd");
        timer_begin(p, t);
        e = launch<FFTZr2cK<T>>(p, (nlines + Wz - 1) / Wz, ldsz, (const T*)grid, cg, nlines, Iy, Kys, Wz, 0,
                                make_udiv(m), make_udiv(m + 1), to_dev(p.f2y), twy, twp);
        timer_end(p, t);
        if (e != hipSuccess) return e;
        t = timer_id(p, "long2_fft_x_fwd");
        timer_begin(p, t);
        e = launch<FFTYK<T, -1>>(p, nbx, ldsx, cg, planes, Ix, Ky, Kys, Wx, to_dev(p.f2x), twx);
        timer_end(p, t);
    } else {
        int t = timer_id(p, "long2_fft_x_inv");
        timer_begin(p, t);
        e = launch<FFTYK<T, +1>>(p, nbx, ldsx, cg, planes, Ix, Ky, Kys, Wx, to_dev(p.f2x), twx);
        timer_end(p, t);
        if (e != hipSuccess) return e;
        t = timer_id(p, "long2_fft_y_inv");
        timer_begin(p, t);
        e = launch<FFTZc2rK<T>>(p, (nlines + Wz - 1) / Wz, ldsz, (const cpx<T>*)cg, grid, nlines, Iy, Kys, Wz, 0,
                                make_udiv(m), make_udiv(m + 1), to_dev(p.f2y), twy, twp);
        timer_end(p, t);
    }
    return e;
}

}  // namespace

hipError_t launch_fft_long2(Plan& p, int sign, int planes) {
    if (p.r.prec == SOG_PREC_FP64) return run_fft_long2<double>(p, sign, planes);
    return run_fft_long2<float>(p, sign, planes);
}

hipError_t launch_fft_mid(Plan& p) {
    if (p.r.prec == SOG_PREC_FP64) return run_fft_mid<double>(p);
    return run_fft_mid<float>(p);
}

}  // namespace sog
