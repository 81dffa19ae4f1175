// Utility kernels: fills, input validation, counting sort (histogram, exclusive scan,
// scatter), and the final combination of the parts (eqs. splitting and phisplit):
// Phi_i = Phi_N + Phi_mid + Phi_long - q_i sum_l w_l, F_i = -q_i grad Phi_i,
// U = 1/2 sum_i q_i Phi_i (float64 reduction in a fixed order).
#include "launch.hpp"

namespace sog {

namespace {

struct FillIntK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos g, int* const& p, const int& v, const int64_t& n) {
        for (int64_t i = g.bid * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)g.nb * kThreads) p[i] = v;
    }
};

struct FillZeroK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos g, uint32_t* const& p, const int64_t& n) {
        for (int64_t i = g.bid * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)g.nb * kThreads) p[i] = 0u;
    }
};

struct HistK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos g, const int* const& key, const int& n, int* const& count) {
        for (int i = g.bid * kThreads + threadIdx.x; i < n; i += g.nb * kThreads) atomicAdd(&count[key[i]], 1);
    }
};

struct ScatterK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos g, const int* const& key, const int& n, const int* const& start,
                               int* const& cursor, int* const& perm) {
        for (int i = g.bid * kThreads + threadIdx.x; i < n; i += g.nb * kThreads) {
            int k = key[i];
            int pos = start[k] + atomicAdd(&cursor[k], 1);
            perm[pos] = i;
        }
    }
};

// Canonical order of a counting sort (the deterministic mode): the sort's atomic ranks put
// the members of a bin in an arbitrary order; CanonScatterK lists each bin's members (by
// particle index) at the ranks they got, and CanonRankK replaces every member's rank by
// its rank by particle index within the bin, so the packing that follows puts each bin in
// index order whatever order the atomics took.
struct CanonScatterK {
    static constexpr int kThreads = 256;
    // key[i] = (bin, rank) (int2) when cursor is null, else key[i] = bin (int) and the rank
    // is taken from cursor[bin] here
    __device__ static void run(GridPos g, const int* const& key, const int& n, const int* const& start,
                               int* const& cursor, int* const& idx) {
        for (int i = g.bid * kThreads + threadIdx.x; i < n; i += g.nb * kThreads) {
            int pos;
            if (cursor) {
                const int k = key[i];
                pos = start[k] + atomicAdd(&cursor[k], 1);
            } else {
                pos = start[key[2 * i]] + key[2 * i + 1];
            }
            idx[pos] = i;
        }
    }
};

// One wave per bin (four per block, bins strided over the grid): each lane takes members
// of the bin, 64 at a time, and counts the members with a smaller particle index (all
// lanes read the same member at once); rank[stride * i] = that count.  Work grows with
// the square of a bin's size: about 30 per near-field cell and a few hundred per gridding
// tile on uniform input.
struct CanonRankK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos g, const int* const& start, const int& nbins, const int* const& idx,
                               int* const& rank, const int& stride) {
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int b = g.bid * 4 + wv; b < nbins; b += g.nb * 4) {
            const int s = start[b], e = start[b + 1];
            for (int base = s; base < e; base += 64) {
                const int p = base + lane;
                const int mine = p < e ? idx[p] : 0x7fffffff;
                int cnt = 0;
                for (int q = s; q < e; ++q) cnt += idx[q] < mine ? 1 : 0;
                if (p < e) rank[(size_t)stride * mine] = cnt;
            }
        }
    }
};

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

struct ScanLocalK {
    static constexpr int kThreads = kScanThreads;
    __device__ static void run(GridPos g, int* const& data, const int& len, int* const& block_sums) {
        __shared__ int lds[kScanThreads];
        const int base = g.bid * kScanChunk + threadIdx.x * kScanPer;
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
        if (threadIdx.x == 0) block_sums[g.bid] = total;
    }
};

// single block: exclusive scan of nb block sums, chunk by chunk with a running carry
struct ScanSumsK {
    static constexpr int kThreads = kScanThreads;
    __device__ static void run(GridPos, int* const& block_sums, const int& nb) {
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
};

struct ScanAddK {
    static constexpr int kThreads = kScanThreads;
    __device__ static void run(GridPos g, int* const& data, const int& len, const int* const& block_sums) {
        const int add = block_sums[g.bid];
        const int base = g.bid * kScanChunk + threadIdx.x * kScanPer;
        for (int j = 0; j < kScanPer; ++j)
            if (base + j < len) data[base + j] += add;
    }
};

template <typename real>
struct CombineK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos g, const vec4<real>* const& part, const double* const& q, const int64_t& n,
                               const double& self_coeff, double* const& phi, double* const& force,
                               double* const& grad, double* const& red) {
        __shared__ double lds[16];
        double e = 0;
        for (int64_t i = g.bid * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)g.nb * kThreads) {
            double qi = q[i];
            const vec4<real> a = part[i], b = part[n + i], c = part[2 * n + i];
            double ph = (double)a.x + (double)b.x + (double)c.x - qi * self_coeff;
            const double gv[3] = {(double)a.y + (double)b.y + (double)c.y, (double)a.z + (double)b.z + (double)c.z,
                                  (double)a.w + (double)b.w + (double)c.w};
            if (phi) phi[i] = ph;
            if (force)
                for (int d = 0; d < 3; ++d) force[3 * i + d] = -qi * gv[d];
            if (grad)
                for (int d = 0; d < 3; ++d) grad[3 * i + d] = gv[d];
            e += qi * ph;
        }
        double t = block_sum_double(e, lds);
        if (threadIdx.x == 0) red[g.bid] = t;
    }
};

struct EnergyFinalK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos, const double* const& red, const int& nb, double* const& energy) {
        __shared__ double lds[16];
        double s = 0;
        for (int i = threadIdx.x; i < nb; i += kThreads) s += red[i];
        // fixed-order tree: each thread's strided partial, then the block sum
        double t = block_sum_double(s, lds);
        if (threadIdx.x == 0) energy[0] = 0.5 * t;
    }
};

template <typename real>
struct PartsOutK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos g, const vec4<real>* const& part, const int64_t& n, double* const& phi_parts,
                               double* const& grad_parts) {
        for (int64_t i = g.bid * (int64_t)kThreads + threadIdx.x; i < 3 * n; i += (int64_t)g.nb * kThreads) {
            const vec4<real> v = part[i];
            if (phi_parts) phi_parts[i] = (double)v.x;
            if (grad_parts) {
                grad_parts[3 * i] = (double)v.y;
                grad_parts[3 * i + 1] = (double)v.z;
                grad_parts[3 * i + 2] = (double)v.w;
            }
        }
    }
};

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

hipError_t launch_fill_int(Plan& p, int* ptr, int value, int64_t n) {
    if (n <= 0) return hipSuccess;
    return launch<FillIntK>(p, grid_for(n, 256), 0, ptr, value, n);
}

hipError_t launch_fill_bytes_zero(Plan& p, void* ptr, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 4);
    return launch<FillZeroK>(p, grid_for(n, 256), 0, (uint32_t*)ptr, n);
}

hipError_t launch_batch_check(const double* x, const double* q, const int64_t* off, int nsys, const double* lz,
                              int64_t n, double* qsum, int* status, hipStream_t s) {
    if (nsys < 1 || n < 1) return hipErrorInvalidValue;
    const int64_t nq = 4 * (int64_t)nsys;  // 2 nsys doubles
    k_single<FillZeroK><<<grid_for(nq, 256), 256, 0, s>>>((uint32_t*)qsum, nq);
    k_single<FillIntK><<<grid_for(nsys, 256), 256, 0, s>>>(status, 0, (int64_t)nsys);
    k_batch_check<<<grid_for(n, 256), 256, 0, s>>>(x, q, off, nsys, lz, n, qsum, status);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(Plan& p, int* data, int len, int* tmp) {
    int nb = (len + kScanChunk - 1) / kScanChunk;
    hipError_t e = launch<ScanLocalK>(p, nb, 0, data, len, tmp);
    if (e == hipSuccess) e = launch<ScanSumsK>(p, 1, 0, tmp, nb);
    if (e == hipSuccess) e = launch<ScanAddK>(p, nb, 0, data, len, (const int*)tmp);
    return e;
}

// start has nbins + 1 entries; cursor has nbins; keys must lie in [0, nbins).
hipError_t launch_counting_sort(Plan& p, const int* key, int n, int nbins, int* start, int* cursor, int* perm) {
    hipError_t e = launch_fill_int(p, start, 0, (int64_t)nbins + 1);
    if (e == hipSuccess) e = launch_fill_int(p, cursor, 0, nbins);
    if (e == hipSuccess) e = launch<HistK>(p, grid_for(n, 256), 0, key, n, start);
    if (e == hipSuccess) e = launch_exclusive_scan(p, start, nbins + 1, p.ws.scan_tmp);
    if (e == hipSuccess) e = launch<ScatterK>(p, grid_for(n, 256), 0, key, n, (const int*)start, cursor, perm);
    return e;
}

hipError_t launch_combine(Plan& p, const double* q, double* phi, double* force, double* grad, double* energy) {
    int nb = p.ws.red_blocks;
    int t = timer_id(p, "combine");
    timer_begin(p, t);
    hipError_t e;
    if (p.r.prec == SOG_PREC_FP64)
        e = launch<CombineK<double>>(p, nb, 0, (const vec4<double>*)p.ws.parts, q, p.r.n, p.r.self_coeff, phi, force,
                                     grad, p.ws.red);
    else
        e = launch<CombineK<float>>(p, nb, 0, (const vec4<float>*)p.ws.parts, q, p.r.n, p.r.self_coeff, phi, force,
                                    grad, p.ws.red);
    if (e == hipSuccess && energy) e = launch<EnergyFinalK>(p, 1, 0, (const double*)p.ws.red, nb, energy);
    timer_end(p, t);
    return e;
}

hipError_t launch_parts_out(Plan& p, double* phi_parts, double* grad_parts) {
    if (p.r.prec == SOG_PREC_FP64)
        return launch<PartsOutK<double>>(p, grid_for(3 * p.r.n, 256), 0, (const vec4<double>*)p.ws.parts, p.r.n,
                                         phi_parts, grad_parts);
    return launch<PartsOutK<float>>(p, grid_for(3 * p.r.n, 256), 0, (const vec4<float>*)p.ws.parts, p.r.n, phi_parts,
                                    grad_parts);
}

hipError_t launch_canonical_ranks(Plan& p, int* key, bool pairs, int n, const int* start, int nbins, int* cursor,
                                  int* idx, int* rank) {
    if (n <= 0 || nbins <= 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (!pairs) e = launch_fill_int(p, cursor, 0, nbins);
    if (e == hipSuccess)
        e = launch<CanonScatterK>(p, grid_for(n, 256), 0, (const int*)key, n, start, pairs ? (int*)nullptr : cursor,
                                  idx);
    if (e == hipSuccess)
        e = launch<CanonRankK>(p, std::min((nbins + 3) / 4, 16384), 0, start, nbins, (const int*)idx,
                               pairs ? key + 1 : rank, pairs ? 2 : 1);
    return e;
}

hipError_t launch_zero_parts(Plan& p, int part) {
    const size_t rs = p.r.prec == SOG_PREC_FP64 ? 8 : 4;
    char* pp = static_cast<char*>(p.ws.parts) + (size_t)part * p.r.n * 4 * rs;
    return launch_fill_bytes_zero(p, pp, p.r.n * 4 * rs);
}

}  // namespace sog
