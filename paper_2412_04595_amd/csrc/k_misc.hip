// Utility kernels: fills, input validation, counting sort (histogram, exclusive scan,
// scatter), and the final combination of the parts (eqs. splitting and phisplit):
// Phi_i = Phi_N + Phi_mid + Phi_long - q_i sum_l w_l, F_i = -q_i grad Phi_i,
// U = 1/2 sum_i q_i Phi_i (float64 reduction in a fixed order).
#include "device_common.hpp"

namespace sog {

namespace {

__global__ void k_fill_int(int* p, int v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_zero_u32(uint32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void k_hist(const int* __restrict__ key, int n, int* __restrict__ count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) atomicAdd(&count[key[i]], 1);
}

__global__ void k_scatter(const int* __restrict__ key, int n, const int* __restrict__ start, int* __restrict__ cursor,
                          int* __restrict__ perm) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int k = key[i];
        int pos = start[k] + atomicAdd(&cursor[k], 1);
        perm[pos] = i;
    }
}

constexpr int kScanPer = 4;
constexpr int kScanThreads = 256;
constexpr int kScanChunk = kScanPer * kScanThreads;

// Exclusive scan of 256 per-thread totals in LDS; returns this thread's exclusive prefix,
// and the block total in *total.
__device__ int block_exclusive_scan(int v, int* lds, int* total) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        int add = (threadIdx.x >= o) ? lds[threadIdx.x - o] : 0;
        __syncthreads();
        lds[threadIdx.x] += add;
        __syncthreads();
    }
    int incl = lds[threadIdx.x];
    *total = lds[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_local(int* data, int len, int* block_sums) {
    __shared__ int lds[kScanThreads];
    const int base = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    int v[kScanPer];
    int sum = 0;
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = (base + j < len) ? data[base + j] : 0;
        sum += v[j];
    }
    int total;
    int pre = block_exclusive_scan(sum, lds, &total);
    for (int j = 0; j < kScanPer; ++j) {
        if (base + j < len) data[base + j] = pre;
        pre += v[j];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// single block: exclusive scan of nb block sums, chunk by chunk with a running carry
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int* block_sums, int nb) {
    __shared__ int lds[kScanThreads];
    int carry = 0;
    for (int c0 = 0; c0 < nb; c0 += kScanChunk) {
        const int base = c0 + threadIdx.x * kScanPer;
        int v[kScanPer];
        int sum = 0;
        for (int j = 0; j < kScanPer; ++j) {
            v[j] = (base + j < nb) ? block_sums[base + j] : 0;
            sum += v[j];
        }
        int total;
        int pre = block_exclusive_scan(sum, lds, &total);
        pre += carry;
        for (int j = 0; j < kScanPer; ++j) {
            if (base + j < nb) block_sums[base + j] = pre;
            pre += v[j];
        }
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int* data, int len, const int* block_sums) {
    const int add = block_sums[blockIdx.x];
    const int base = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    for (int j = 0; j < kScanPer; ++j)
        if (base + j < len) data[base + j] += add;
}

template <typename real>
__global__ void k_combine(const vec4<real>* __restrict__ part, const double* __restrict__ q,
                          int64_t n, double self_coeff, double* __restrict__ phi, double* __restrict__ force,
                          double* __restrict__ grad, double* __restrict__ red) {
    __shared__ double lds[16];
    double e = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double qi = q[i];
        const vec4<real> a = part[i], b = part[n + i], c = part[2 * n + i];
        double ph = (double)a.x + (double)b.x + (double)c.x - qi * self_coeff;
        const double g[3] = {(double)a.y + (double)b.y + (double)c.y, (double)a.z + (double)b.z + (double)c.z,
                             (double)a.w + (double)b.w + (double)c.w};
        if (phi) phi[i] = ph;
        if (force)
            for (int d = 0; d < 3; ++d) force[3 * i + d] = -qi * g[d];
        if (grad)
            for (int d = 0; d < 3; ++d) grad[3 * i + d] = g[d];
        e += qi * ph;
    }
    double t = block_sum_double(e, lds);
    if (threadIdx.x == 0) red[blockIdx.x] = t;
}

__global__ void k_energy_final(const double* __restrict__ red, int nb, double* __restrict__ energy) {
    __shared__ double lds[16];
    double s = 0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += red[i];
    // fixed-order tree: each thread's strided partial, then the block sum
    double t = block_sum_double(s, lds);
    if (threadIdx.x == 0) energy[0] = 0.5 * t;
}

template <typename real>
__global__ void k_parts_out(const vec4<real>* __restrict__ part, int64_t n, double* __restrict__ phi_parts,
                            double* __restrict__ grad_parts) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * blockDim.x) {
        const vec4<real> v = part[i];
        if (phi_parts) phi_parts[i] = (double)v.x;
        if (grad_parts) {
            grad_parts[3 * i] = (double)v.y;
            grad_parts[3 * i + 1] = (double)v.z;
            grad_parts[3 * i + 2] = (double)v.w;
        }
    }
}

// Input check of a batch of systems stored one after another (system s holds particles
// [off[s], off[s + 1]), off strictly increasing): per system the sum of the charges and of
// their magnitudes (qsum[2s], qsum[2s + 1], for the neutrality test of Prop.
// lem::summation) and flags (status[s]: 1 a non-finite position or charge, 2 a z outside
// [0, Lz_s]).  A wave whose particles all belong to one system adds its two sums once.
__global__ __launch_bounds__(256) void k_batch_check(const double* __restrict__ x, const double* __restrict__ q,
                                                     const int64_t* __restrict__ off, int nsys,
                                                     const double* __restrict__ lz, int64_t n,
                                                     double* __restrict__ qsum, int* __restrict__ status) {
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        int s = -1, fl = 0;
        double a = 0.0, b = 0.0;
        if (i < n) {
            int lo = 0, hi = nsys - 1;  // the last s with off[s] <= i
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (off[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            s = lo;
            const double x0 = x[3 * i], y0 = x[3 * i + 1], z0 = x[3 * i + 2], qq = q[i];
            if (!(isfinite(x0) && isfinite(y0) && isfinite(z0) && isfinite(qq))) {
                fl = 1;
            } else {
                if (z0 < 0.0 || z0 > lz[s]) fl = 2;
                a = qq;
                b = fabs(qq);
            }
        }
        if (fl) atomicOr(&status[s], fl);
        // lane 0 holds the wave's lowest index, so it is in range whenever any lane is
        const int s0 = __shfl(s, 0);
        if (__all(s == s0 || s < 0)) {
            for (int m = 32; m >= 1; m >>= 1) {
                a += __shfl_xor(a, m);
                b += __shfl_xor(b, m);
            }
            if ((threadIdx.x & 63) == 0 && s0 >= 0) {
                atomicAdd(&qsum[2 * s0], a);
                atomicAdd(&qsum[2 * s0 + 1], b);
            }
        } else if (s >= 0) {
            atomicAdd(&qsum[2 * s], a);
            atomicAdd(&qsum[2 * s + 1], b);
        }
    }
}

int grid_for(int64_t n, int threads, int maxb = 4096) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > maxb) b = maxb;
    return (int)b;
}

}  // namespace

hipError_t launch_fill_int(int* p, int value, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_int<<<grid_for(n, 256), 256, 0, s>>>(p, value, n);
    return hipGetLastError();
}

hipError_t launch_fill_bytes_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4) return hipErrorInvalidValue;
    int64_t n = (int64_t)(bytes / 4);
    k_fill_zero_u32<<<grid_for(n, 256), 256, 0, s>>>((uint32_t*)p, n);
    return hipGetLastError();
}

hipError_t launch_batch_check(const double* x, const double* q, const int64_t* off, int nsys, const double* lz,
                              int64_t n, double* qsum, int* status, hipStream_t s) {
    if (nsys < 1 || n < 1) return hipErrorInvalidValue;
    hipError_t e = launch_fill_bytes_zero(qsum, 2 * (size_t)nsys * sizeof(double), s);
    if (e == hipSuccess) e = launch_fill_int(status, 0, nsys, s);
    if (e != hipSuccess) return e;
    k_batch_check<<<grid_for(n, 256), 256, 0, s>>>(x, q, off, nsys, lz, n, qsum, status);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(Plan& p, int* data, int len, int* tmp) {
    int nb = (len + kScanChunk - 1) / kScanChunk;
    k_scan_local<<<nb, kScanThreads, 0, p.stream>>>(data, len, tmp);
    k_scan_sums<<<1, kScanThreads, 0, p.stream>>>(tmp, nb);
    k_scan_add<<<nb, kScanThreads, 0, p.stream>>>(data, len, tmp);
    return hipGetLastError();
}

// start has nbins + 1 entries; cursor has nbins; keys must lie in [0, nbins).
hipError_t launch_counting_sort(Plan& p, const int* key, int n, int nbins, int* start, int* cursor, int* perm) {
    hipError_t e = launch_fill_int(start, 0, (int64_t)nbins + 1, p.stream);
    if (e != hipSuccess) return e;
    e = launch_fill_int(cursor, 0, nbins, p.stream);
    if (e != hipSuccess) return e;
    k_hist<<<grid_for(n, 256), 256, 0, p.stream>>>(key, n, start);
    e = launch_exclusive_scan(p, start, nbins + 1, p.ws.scan_tmp);
    if (e != hipSuccess) return e;
    k_scatter<<<grid_for(n, 256), 256, 0, p.stream>>>(key, n, start, cursor, perm);
    return hipGetLastError();
}

hipError_t launch_combine(Plan& p, const double* q, double* phi, double* force, double* grad, double* energy) {
    int nb = p.ws.red_blocks;
    int t = timer_id(p, "combine");
    timer_begin(p, t);
    if (p.r.prec == SOG_PREC_FP64)
        k_combine<double><<<nb, 256, 0, p.stream>>>((const vec4<double>*)p.ws.parts, q,
                                                     p.r.n, p.r.self_coeff, phi, force, grad, p.ws.red);
    else
        k_combine<float><<<nb, 256, 0, p.stream>>>((const vec4<float>*)p.ws.parts, q,
                                                    p.r.n, p.r.self_coeff, phi, force, grad, p.ws.red);
    if (energy) k_energy_final<<<1, 256, 0, p.stream>>>(p.ws.red, nb, energy);
    timer_end(p, t);
    return hipGetLastError();
}

hipError_t launch_parts_out(Plan& p, double* phi_parts, double* grad_parts) {
    if (p.r.prec == SOG_PREC_FP64)
        k_parts_out<double><<<grid_for(3 * p.r.n, 256), 256, 0, p.stream>>>(
            (const vec4<double>*)p.ws.parts, p.r.n, phi_parts, grad_parts);
    else
        k_parts_out<float><<<grid_for(3 * p.r.n, 256), 256, 0, p.stream>>>(
            (const vec4<float>*)p.ws.parts, p.r.n, phi_parts, grad_parts);
    return hipGetLastError();
}

hipError_t launch_zero_parts(Plan& p, int part) {
    size_t rs = (p.r.prec == SOG_PREC_FP64) ? 8 : 4;
    char* pp = (char*)p.ws.parts + (size_t)part * p.r.n * 4 * rs;
    return launch_fill_bytes_zero(pp, p.r.n * 4 * rs, p.stream);
}

}  // namespace sog
