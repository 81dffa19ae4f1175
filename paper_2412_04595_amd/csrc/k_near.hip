// Near field (eq. phiNDR): Phi^N_i = sum'_{j, n: |r_ij + n o L| < r_c} q_j N(|r_ij + n o L|),
// N(r) = 1/r - F(r) (eq. SOGDEcomp), over xy images only (z is free), with a cell list
// of cells at least r_c wide (the paper's cell list, Sec. 2.2).
//
// F(r) and F'(r)/r are evaluated as Chebyshev series in x = 2 r^2/r_c^2 - 1 (fitted in
// float64 at plan time), so the cost per pair does not depend on the number of
// Gaussians M (Remark rmk::sum asks for that; a polynomial in r^2 is this library's way
// of getting it).
//
// Pipeline: a counting sort of the particles by cell (cells z-fastest, so a column is one
// contiguous range), then a sort by z inside each cell, so every column is z-ordered.
// Work units are formed per column on the device: chunks of at most 32 consecutive
// targets within at most kNearUnitCells cells (NearChunksK); the pair kernel (NearMfmaK)
// tests candidates against them on the matrix cores in float32 and evaluates the hits in
// the plan's precision.  A unit's candidates are, per neighbouring column (9 of them),
// the cells from below the unit to above it, cut where they cross a z frame (below) and
// narrowed by bisection to the unit's z extent +- r_c.
//
// Coordinates enter the pair kernel as offsets from the corner of the particle's x, y
// cell and of its z frame (kNearFrameCells cells), formed in float64, so the float32 form
// does not lose the ~1e-5 absolute precision that raw float32 coordinates of a 100-wide
// box would.  A candidate is seen from a target shifted by the geometric offset of their
// columns and frames; that shift is an exact zero for the target's own column and frame,
// so the pair of a particle with itself has r^2 == 0 exactly.
#include "launch.hpp"

namespace sog {

namespace {

struct NearGeom {
    double L[3];
    double ch[3];
    int nc[3];
};

constexpr int kNearFrameCells = 8;  // z cells per coordinate frame; a work unit spans at most
                                    // kNearUnitCells = 7 cells, so its candidate z range
                                    // (<= 9 cells) crosses at most one frame boundary
static_assert(kNearUnitCells + 2 <= kNearFrameCells + 1, "candidate range crosses two frame boundaries");

__device__ __forceinline__ void cell_of(const NearGeom& g, double xw, double yw, double z, int c[3]) {
    double v[3] = {xw, yw, z};
    for (int d = 0; d < 3; ++d) {
        int k = (int)floor(v[d] / g.ch[d]);
        c[d] = min(max(k, 0), g.nc[d] - 1);
    }
}

// Cell of every particle and the cell histogram of the counting sort; in the same pass
// the input checks of the problem statement (Sec. 2.1): finite inputs, z in [0, L_z]
// (status bits 1 and 2), and the charge sums sum q, sum |q| for the neutrality test of
// Prop. lem::summation (block b adds into slot b mod kQsumSlots; the host adds the
// slots).  Block sums need blockDim.x a multiple of 64.
struct NearKeyK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, const double* __restrict__ x, const double* __restrict__ q, int n, NearGeom g, int2* __restrict__ key, int* __restrict__ count, double* __restrict__ qsum, int* __restrict__ status) {
    __shared__ double red[16];
    double s = 0, sa = 0;
    int flags = 0;
    for (int i = gpos.bid * kThreads + threadIdx.x; i < n; i += gpos.nb * kThreads) {
        const double x0 = x[3 * i], y0 = x[3 * i + 1], z0 = x[3 * i + 2], qq = q[i];
        if (!(isfinite(x0) && isfinite(y0) && isfinite(z0) && isfinite(qq))) {
            flags |= 1;
        } else {
            if (z0 < 0.0 || z0 > g.L[2]) flags |= 2;
            s += qq;
            sa += fabs(qq);
        }
        double xw = wrap_periodic(x0, g.L[0]), yw = wrap_periodic(y0, g.L[1]);
        double z = z0;
        if (!isfinite(xw)) xw = 0;
        if (!isfinite(yw)) yw = 0;
        if (!isfinite(z)) z = 0;
        int c[3];
        cell_of(g, xw, yw, z, c);
        const int k = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
        key[i] = make_int2(k, atomicAdd(&count[k], 1));  // cell and rank within it
    }
    if (flags) atomicOr(status, flags);
    double* slot = qsum + 2 * (gpos.bid % kQsumSlots);  // spread over slots: few adds per address
    double t = block_sum_double(s, red);
    if (threadIdx.x == 0) atomicAdd(&slot[0], t);
    t = block_sum_double(sa, red);
    if (threadIdx.x == 0) atomicAdd(&slot[1], t);
}
};

// Scatter of the counting sort, writing each particle's packed record at its place in
// cell order, cell start plus the rank the histogram pass gave it (particles read in their
// own order, records written once, no atomics).
template <typename real>
struct NearPackK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, const double* __restrict__ x, const double* __restrict__ q, int n, NearGeom g, const int2* __restrict__ key, const int* __restrict__ start, vec4<real>* __restrict__ pos, int* __restrict__ orig) {
    for (int i = gpos.bid * kThreads + threadIdx.x; i < n; i += gpos.nb * kThreads) {
        const int2 kr = key[i];
        const int p = start[kr.x] + kr.y;
        double xw = wrap_periodic(x[3 * i], g.L[0]), yw = wrap_periodic(x[3 * i + 1], g.L[1]);
        double z = x[3 * i + 2];
        double qq = q[i];
        if (!isfinite(xw)) xw = 0;
        if (!isfinite(yw)) yw = 0;
        if (!isfinite(z)) z = 0;
        if (!isfinite(qq)) qq = 0;
        int c[3];
        cell_of(g, xw, yw, z, c);
        vec4<real> v;
        v.x = (real)(xw - c[0] * g.ch[0]);
        v.y = (real)(yw - c[1] * g.ch[1]);
        v.z = (real)(z - (c[2] / kNearFrameCells) * kNearFrameCells * g.ch[2]);
        v.w = (real)qq;
        pos[p] = v;
        orig[p] = i;
    }
}
};

constexpr int kUnitsLds = 4096;  // cells of a column staged in LDS at a time
constexpr int kGrabStride = 32;  // ints between the per-XCD work counters (own 128-byte lines)
// Work units of the float32 pair kernel: chunks of at most kNearChunk consecutive targets
// of a column, cut where a chunk would span more than kNearUnitCells cells; unit =
// (cell of the first target, first target, end target, end cell), in the column's slots
// (see near_unit_slots), unused slots marked by -1.  One wave per column: the column's
// cell starts are staged in LDS when they fit, and lane 0 walks them.
struct NearChunksK {
    static constexpr int kThreads = 64;
    __device__ static void run(GridPos gpos, const int* __restrict__ cell_start, int ncz, int extra, int4* __restrict__ units, int* __restrict__ grab) {
    __shared__ int cs_lds[kUnitsLds + 1];
    const int col = gpos.bid;
    if (col == 0 && threadIdx.x < 8) grab[threadIdx.x * kGrabStride] = 0;  // the pair kernel's work counters
    const int* gcs = cell_start + (size_t)col * ncz;
    const int* cs = gcs;
    if (ncz <= kUnitsLds) {
        for (int i = threadIdx.x; i <= ncz; i += 64) cs_lds[i] = gcs[i];
        __syncthreads();
        cs = cs_lds;
    }
    const int64_t s0 = (int64_t)(gcs[0] / kNearChunk) + (int64_t)col * extra;
    const int64_t s1 = (int64_t)(gcs[ncz] / kNearChunk) + (int64_t)(col + 1) * extra;
    int u = 0;
    if (threadIdx.x == 0) {
        int4* us = units + s0;
        u = near_chunk_walk(cs, ncz, [&](int za, int p, int e, int z1) { *us++ = make_int4(col * ncz + za, p, e, z1); });
    }
    u = __shfl(u, 0, 64);
    for (int64_t i = s0 + u + (int)threadIdx.x; i < s1; i += 64) units[i] = make_int4(0, -1, -1, 0);
}
};

// Particles of each cell sorted by z.  The columns become z-ordered,
// so a chunk of consecutive targets spans the least z and the candidates of a neighbour
// column within r_c of the chunk in z form one contiguous range, which the pair kernel
// finds by bisection.  One wave per cell: a bitonic network over the cell's (z, index)
// pairs, across the lanes for up to 64 particles, in LDS for more, then the records
// written back in order.  A cell of more than
// kZsortMax particles stays unsorted and sets status bit 4, which switches the
// bisection off for the call.
constexpr int kZsortMax = 256;
template <typename real>
struct NearZsortK {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos gpos, const int* __restrict__ cell_start, int ncells, vec4<real>* __restrict__ pos, int* __restrict__ orig, int* __restrict__ status) {
    __shared__ real key_all[4][kZsortMax];
    __shared__ int idx_all[4][kZsortMax];
    __shared__ vec4<real> rec_all[4][kZsortMax];
    __shared__ int org_all[4][kZsortMax];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = gpos.bid * 4 + wv;
    if (c >= ncells) return;
    const int b = cell_start[c], n = cell_start[c + 1] - b;
    if (n <= 1) return;
    if (n > kZsortMax) {
        if (lane == 0) atomicOr(status, 4);
        return;
    }
    if (n <= 64) {
        // in registers: lane i holds element i (padding +inf), the network by lane shuffles
        const vec4<real> rv = lane < n ? pos[b + lane] : vec4<real>{0, 0, 0, 0};
        const int ov = lane < n ? orig[b + lane] : 0;
        real kk = lane < n ? rv.z : (real)INFINITY;
        int ii = lane;
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const real ko = __shfl_xor(kk, j, 64);
                const int io = __shfl_xor(ii, j, 64);
                const bool other_less = ko < kk || (ko == kk && io < ii);
                const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
                if (keep_min == other_less) {
                    kk = ko;
                    ii = io;
                }
            }
        vec4<real> w;
        w.x = __shfl(rv.x, ii, 64);
        w.y = __shfl(rv.y, ii, 64);
        w.z = __shfl(rv.z, ii, 64);
        w.w = __shfl(rv.w, ii, 64);
        const int ow = __shfl(ov, ii, 64);
        if (lane < n) {
            pos[b + lane] = w;
            orig[b + lane] = ow;
        }
        return;
    }
    real* key = key_all[wv];
    int* idx = idx_all[wv];
    vec4<real>* rec = rec_all[wv];
    int* org = org_all[wv];
    int S = 2;
    while (S < n) S <<= 1;
    for (int i = lane; i < S; i += 64) {
        if (i < n) {
            rec[i] = pos[b + i];
            org[i] = orig[b + i];
            key[i] = rec[i].z;
        } else {
            key[i] = (real)INFINITY;
        }
        idx[i] = i;
    }
    auto sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    sync();
    // ascending by (z, original index): a strict order, so the result is unique
    for (int k = 2; k <= S; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int pi = lane; pi < S / 2; pi += 64) {
                const int i = 2 * j * (pi / j) + pi % j, q = i + j;
                const real ki = key[i], kq = key[q];
                const int ii = idx[i], iq = idx[q];
                const bool gt = ki > kq || (ki == kq && ii > iq);
                if (gt == ((i & k) == 0)) {
                    key[i] = kq;
                    key[q] = ki;
                    idx[i] = iq;
                    idx[q] = ii;
                }
            }
            sync();
        }
    for (int i = lane; i < n; i += 64) {
        const int src = idx[i];
        pos[b + i] = rec[src];
        orig[b + i] = org[src];
    }
}
};

// the 8 work counters live after the units, on 128-byte boundaries
inline int* near_grab(const Workspace& ws, int64_t slots) {
    return reinterpret_cast<int*>(static_cast<char*>(ws.near_units) + ((size_t)slots * 16 + 127) / 128 * 128);
}

template <typename real>
struct NearArgs {
    const vec4<real>* __restrict__ pos;
    const int* __restrict__ orig;
    const int* __restrict__ cell_start;
    vec4<real>* __restrict__ part;  // near part of each particle: phi, grad
    const int4* __restrict__ units;  // (column, first cell, end cell); first cell -1: none
    int* grab;                       // per-XCD counters of units taken (zeroed by NearChunksK)
    const int* status;               // bit 4: some cell is not z-sorted (no bisection of the ranges)
    float zcut;                      // r_c with a rounding margin: the z reach of the ranges
    int max_units;
    int nc[3];
    real ch[3];
    real rc2, inv_rc2;
    int deg;
    real cF[kMaxNearDeg + 1];
    real cG[kMaxNearDeg + 1];
    real mF[kMaxNearDeg + 1];  // the same in monomial form (float32 kernel, Horner)
    real mG[kMaxNearDeg + 1];
    // float32 kernel: pairs closer than sqrt(rclose2) take their separation from the
    // float64 input coordinates x (minimum image over L in x, y) instead of from the
    // float32 offsets, whose rounding (~5e-7 of a cell) would cost 5e-7 / r of 1/r
    const double* __restrict__ x;
    double L[2];
    real rclose2;
    // the candidate test's float32 positions (the records themselves in float32 plans) and
    // the margin added to r_c^2 in that test (float64 plans: the float32 test must not
    // lose a pair inside r_c; the evaluation cuts at r_c exactly)
    const vec4<float>* __restrict__ pos32;
    float test_margin;
};

constexpr int kNearWaves = 4;   // independent waves per block
// resident near-field blocks per compute unit: the kernel is persistent, and at this
// occupancy the FFT passes and the gathering launched on the other stream find room
// (LDS and waves) on every compute unit beside it
constexpr int kNearBlocksPerCU = 4;
constexpr int kNearCap = 32;    // float32 hit-list entries per lane (a ring; power of two)
constexpr int kNearCodeShift = 26;  // candidate code: source index | (neighbour range << 26)
// the neighbour columns (dx + 1) + 3 (dy + 1) in the order of the walk, 4 bits each: the
// unit's own column first, then opposite corners and opposite edges in turn, so that the
// hits of consecutive blocks fall on targets on opposite sides of the column (the
// float32 lists then fill more evenly); ranges 0 and 1 are the own column's
constexpr unsigned long long kNearColumnOrder = 0x537162804ull;

// 1/sqrt: the hardware reciprocal square root in float32 (r^2 is far from denormal here)
__device__ __forceinline__ float near_rsqrt(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double near_rsqrt(double v) { return rsqrt(v); }

template <typename real, int DEG>
__device__ __forceinline__ void near_pair(const NearArgs<real>& a, real rx, real ry, real rz, real qj, real& phi,
                                          real& gx, real& gy, real& gz, real r2) {
    // F(r) and F'(r)/r as Chebyshev series in xs = 2 r^2/r_c^2 - 1, one forward
    // recurrence for both (coefficients above the fitted degree are zero)
    const real xs = (real)2 * r2 * a.inv_rc2 - (real)1;
    const real x2 = xs + xs;
    real T0 = 1, T1 = xs;
    real F = a.cF[0] + a.cF[1] * xs, G = a.cG[0] + a.cG[1] * xs;
#pragma unroll
    for (int k = 2; k <= DEG; ++k) {
        const real T2 = x2 * T1 - T0;
        F += a.cF[k] * T2;
        G += a.cG[k] * T2;
        T0 = T1;
        T1 = T2;
    }
    const real ri = near_rsqrt(r2);
    phi += qj * (ri - F);                       // N(r) = 1/r - F(r)
    const real c = qj * (-ri * ri * ri - G);   // N'(r)/r
    gx += c * rx;
    gy += c * ry;
    gz += c * rz;
}

// The pair kernel with the candidate test on the matrix cores (float32 test; evaluation in
// float32 or, for float64 plans, float64: see NearMfmaK).  A pass takes 32
// targets; lanes l and l + 32 share target l % 32 and split its candidates between them.
// The unit's 18 candidate ranges are walked as one sequence in blocks of 32,
// and one block against the pass's targets is a 32 x 32 matrix
//     D[i][j] = |c_i|^2 - 2 c_i . t_j  =  r_ij^2 - |t_j|^2,
// the product of the rows (c_x, c_y, c_z, |c|^2) and the columns (-2 t_x, -2 t_y,
// -2 t_z, 1), two v_mfma_f32_32x32x2f32 steps.  Candidate i of the block sits in lane
// i and i + 32 (k = 0 and 1 of the contraction), target j in lanes j and j + 32;
// register r of lane l holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].  A pair is a hit
// when D < r_c^2 - |t_j|^2.  Coordinates are offsets from the centre of the unit's
// column cell in x, y and from the middle of its run in z, so |c|^2 stays below about
// 25 cells^2 and the rounding of D is far below the cut-off's width.
// The hits are evaluated from hit lists (float32: a ring per lane for the lane's target;
// float64: a stack per wave, compacted across the lanes, so that every lane evaluates a
// pair in every round whatever the spread of the hits over the targets).  r is computed
// directly as t - c: the target and a candidate of its own column and frame get their
// coordinates by adding the same shift to the same stored values, so the particle paired
// with itself has r^2 == 0 exactly and is dropped there.
typedef float near_v16f __attribute__((ext_vector_type(16)));

// lane k's value of a float (the builtin moves 32-bit integers: pass the bits, not the value)
__device__ __forceinline__ float readlane_f(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
constexpr int kNearMfmaRows = 16;  // matrix rows per lane: candidate-target pairs a lane tests per block

// F(r) and F'(r)/r from their monomial form in x = 2 r^2/r_c^2 - 1 by Horner (2 FMAs per
// degree against the Chebyshev recurrence's 3; in float32 no less accurate on [-1, 1],
// which the planner's host checks compare), then as near_pair; the particle paired with
// itself (r^2 == 0) adds nothing
template <int DEG>
__device__ __forceinline__ void near_pair_nz(const NearArgs<float>& a, float rx, float ry, float rz, float qj,
                                             float& phi, float& gx, float& gy, float& gz) {
    const float r2 = rx * rx + ry * ry + rz * rz;
    const bool nz = r2 > 0.f;
    const float q = nz ? qj : 0.f, r2s = nz ? r2 : 1.f;
    const float xs = fmaf(r2s, 2.f * a.inv_rc2, -1.f);  // 2 r^2/r_c^2 - 1 (the factor 2 is exact)
    float F = a.mF[DEG], G = a.mG[DEG];
#pragma unroll
    for (int k = DEG - 1; k >= 0; --k) {
        F = fmaf(F, xs, a.mF[k]);
        G = fmaf(G, xs, a.mG[k]);
    }
    const float ri = near_rsqrt(r2s);
    phi += q * (ri - F);
    const float c = q * (-ri * ri * ri - G);
    gx += c * rx;
    gy += c * ry;
    gz += c * rz;
}

// The separation x_i - x_j of a close pair (packed positions pi, pj) from the float64
// input coordinates: minimum image in x and y (the near field reaches at most L/2), none
// in z.  Left unchanged for non-finite input (whose records hold zeros).
__device__ __forceinline__ void near_close_separation(const NearArgs<float>& a, int pi, int pj, float& rx, float& ry,
                                                   float& rz) {
    const int i = a.orig[pi], j = a.orig[pj];
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = a.x[3 * (size_t)i + k] - a.x[3 * (size_t)j + k];
    d[0] -= a.L[0] * rint(d[0] / a.L[0]);
    d[1] -= a.L[1] * rint(d[1] / a.L[1]);
    if (isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2])) {
        rx = (float)d[0];
        ry = (float)d[1];
        rz = (float)d[2];
    }
}

// E: the evaluation precision.  The candidate test always runs in float32 on the matrix
// cores (positions a.pos32); with E = double the hits are tested with a margin of
// a.test_margin and then evaluated, and cut at r_c exactly, in float64 (positions a.pos).
template <int DEG, typename E = float>
struct NearMfmaK {
    static constexpr int kThreads = 64 * kNearWaves;
    static constexpr bool kF64 = sizeof(E) == 8;
    __device__ static void run(GridPos gpos, const NearArgs<E>& a) {
    // The hits go to one of two sinks.  float32: a ring per lane (the lane's target, its
    // sums in registers), drained kEval entries per lane at a time while every lane has that
    // many.  float64: a stack per wave (codes, targets), evaluated kRound entries at a time,
    // each pair adding its terms to its target's sums in LDS (ds_add_f64; on gfx950 the
    // float32 LDS add, ds_add_f32, runs at about a twentieth of ds_add_f64's rate, so the
    // float32 kernel keeps its sums in registers).
    constexpr int kEval = kF64 ? 2 : 4;           // entries evaluated per lane per round
    constexpr int kRound = 64 * kEval;            // stack: entries evaluated per round
    constexpr int kStack = kRound - 1 + 1024;     // stack: entries left below a round + one block's hits
    __shared__ uint32_t hits_all[kNearWaves][kF64 ? 1 : kNearCap * 64];
    __shared__ uint32_t stack_all[kNearWaves][kF64 ? kStack : 1];
    __shared__ uint8_t stackt_all[kNearWaves][kF64 ? kStack : 1];
    // stack: targets' positions in the unit frame and sums (phi, grad), one array per
    // component, so the lanes of an access spread over the banks by target
    __shared__ E tpos_all[kNearWaves][3][kF64 ? 32 : 1];
    __shared__ E tsum_all[kNearWaves][4][kF64 ? 32 : 1];
    __shared__ vec4<float> shift_all[kNearWaves][18];
    __shared__ vec4<E> shiftE_all[kNearWaves][kF64 ? 18 : 1];  // float64 shifts (E = double)
    __shared__ alignas(16) uint32_t codes_all[kNearWaves][32];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, half = lane >> 5, jl = lane & 31;
    uint32_t* hits = hits_all[wv];
    char* hits_bytes = reinterpret_cast<char*>(&hits_all[0][0]);
    static_assert(kNearCap * 256 == 8192, "list slot bits 8..12 between the lane and wave bits");
    const uint32_t lb = (uint32_t)wv * (kNearCap * 256) | (uint32_t)lane * 4;
    uint32_t* stack = stack_all[wv];
    uint8_t* stackt = stackt_all[wv];
    auto tpos = tpos_all[wv];
    auto tsum = tsum_all[wv];
    vec4<float>* shift = shift_all[wv];
    vec4<E>* shiftE = kF64 ? shiftE_all[wv] : reinterpret_cast<vec4<E>*>(shift_all[wv]);
    uint32_t* codes = codes_all[wv];
    const int per = (a.max_units + 7) >> 3;
    const int ibeg = (gpos.bid & 7) * per, iend = min(a.max_units, ibeg + per);
    int* grab = a.grab + (gpos.bid & 7) * kGrabStride;
    const float fh = (float)kNearFrameCells * (float)a.ch[2];  // frame height
    const E fhE = (E)kNearFrameCells * a.ch[2];
    const vec4<float>* __restrict__ pos32 = a.pos32;  // the test's positions
    const bool trim = (__builtin_amdgcn_readfirstlane(*a.status) & 4) == 0;
    for (;;) {
    int g = 0;
    if (lane == 0) g = atomicAdd(grab, 1);
    const int item = ibeg + __builtin_amdgcn_readfirstlane(g);
    if (item >= iend) break;
    const int4 unit = a.units[item];
    if (unit.y < 0) continue;
    const int col = unit.x / a.nc[2], z0 = unit.x - col * a.nc[2], z1 = unit.w;
    const int cy = col % a.nc[1], cx = col / a.nc[1];
    const int tb = unit.y, te = unit.z;
    const int za = max(z0 - 1, 0), zb = min(z1 + 1, a.nc[2]);
    const int bnd = (za / kNearFrameCells + 1) * kNearFrameCells;
    const float zmid = 0.5f * (float)(z0 + z1) * (float)a.ch[2];
    const E zmidE = (E)0.5 * (E)(z0 + z1) * a.ch[2];
    // the chunk's z extent (its targets are z-sorted): frame-relative z plus the frame base
    const float tzlo = pos32[tb].z + (float)(z0 / kNearFrameCells) * fh;
    const float tzhi = pos32[te - 1].z + (float)((z1 - 1) / kNearFrameCells) * fh;
    // lane k < 18: range k = neighbour column k / 2 of the walk (kNearColumnOrder), piece
    // k % 2 of the cells from below the run to above it, cut at the frame boundary; its
    // shift into the unit frame
    int rs = 0, len = 0;
    vec4<float> sk = {0.f, 0.f, 0.f, 0.f};
    if (lane < 18) {
        const int c9 = (int)((kNearColumnOrder >> (4 * (lane >> 1))) & 15), piece = lane & 1;
        const int dx = c9 % 3 - 1, dy = c9 / 3 - 1;
        const int ncol = imod(cx + dx, a.nc[0]) * a.nc[1] + imod(cy + dy, a.nc[1]);
        const int pa = piece ? bnd : za, pb = piece ? zb : min(zb, bnd);
        if (pa < pb) {
            rs = a.cell_start[ncol * a.nc[2] + pa];
            len = a.cell_start[ncol * a.nc[2] + pb] - rs;
        }
        sk = vec4<float>{((float)dx - 0.5f) * (float)a.ch[0], ((float)dy - 0.5f) * (float)a.ch[1],
                         (float)(pa / kNearFrameCells) * fh - zmid, 0.f};
        shift[lane] = sk;
        if constexpr (kF64)
            shiftE[lane] = vec4<E>{((E)dx - (E)0.5) * a.ch[0], ((E)dy - (E)0.5) * a.ch[1],
                                   (E)(pa / kNearFrameCells) * fhE - zmidE, (E)0};
        if (trim && len > 0) {
            // the columns are z-sorted: keep the candidates within zcut of the chunk's z
            // extent [z of the first target, z of the last], by bisection in the piece's
            // frame coordinates
            const float fo = (float)(pa / kNearFrameCells) * fh;
            const float lo = tzlo - a.zcut - fo, hi = tzhi + a.zcut - fo;
            int l = rs, h = rs + len;
            while (l < h) {
                const int mid = (l + h) >> 1;
                if (pos32[mid].z < lo) l = mid + 1; else h = mid;
            }
            const int nrs = l;
            h = rs + len;
            while (l < h) {
                const int mid = (l + h) >> 1;
                if (pos32[mid].z <= hi) l = mid + 1; else h = mid;
            }
            len = l - nrs;
            rs = nrs;
        }
    }
    // the ranges as one sequence: range k holds positions [pre_k, pre_k + len_k), and
    // position v of it is particle base_k + v
    int inc = len;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    const int pre = inc - len, base = rs - pre;
    const int total = __builtin_amdgcn_readlane(inc, 17);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int t0 = tb; t0 < te; t0 += 32) {
        const int p = t0 + jl;
        const bool act = p < te;
        const vec4<float> me = act ? pos32[p] : vec4<float>{0.f, 0.f, 0.f, 0.f};
        int tcz = z0;
        for (int c = z0 + 1; c < z1; ++c)
            if (p >= a.cell_start[col * a.nc[2] + c]) tcz = c;
        // the target in the unit frame: the shift of its own column (dx = dy = 0, ranges
        // 0 and 1) in its own frame
        const int sti = (tcz / kNearFrameCells) != (za / kNearFrameCells) ? 1 : 0;
        const vec4<float> st = shift[sti];
        const float tx = me.x + st.x, ty = me.y + st.y, tz = me.z + st.z;
        const float thr = act ? (float)a.rc2 + a.test_margin - (tx * tx + ty * ty + tz * tz) : -INFINITY;
        // the target in the evaluation precision
        E txE = tx, tyE = ty, tzE = tz;
        if constexpr (kF64) {
            const vec4<E> meE = act ? a.pos[p] : vec4<E>{0, 0, 0, 0};
            const vec4<E> stE = shiftE[sti];
            txE = meE.x + stE.x;
            tyE = meE.y + stE.y;
            tzE = meE.z + stE.z;
        }
        const float b1 = half ? -2.f * ty : -2.f * tx;
        const float b2 = half ? 1.f : -2.f * tz;
        // float32 sink: this lane's ring [hd, tp) and sums
        E phi = 0, gx = 0, gy = 0, gz = 0;
        int tp = 0, hd = 0;
        constexpr int kMask = kNearCap - 1;
        // up to kEval entries off this lane's ring
        auto chunk = [&]() {
            if constexpr (!kF64) {
                const int cnt = (tp - hd) & kMask;
                vec4<E> o[kEval], sh[kEval];
                int src[kEval];
#pragma unroll
                for (int u = 0; u < kEval; ++u) {
                    const uint32_t e = (cnt > 0) ? hits[((hd + min(u, cnt - 1)) & kMask) * 64 + lane] : (uint32_t)tb;
                    src[u] = (int)(e & ((1u << kNearCodeShift) - 1));
                    o[u] = a.pos[src[u]];
                    sh[u] = shiftE[e >> kNearCodeShift];
                }
#pragma unroll
                for (int u = 0; u < kEval; ++u)
                    if (u < cnt) {
                        E rx = txE - (o[u].x + sh[u].x), ry = tyE - (o[u].y + sh[u].y), rz = tzE - (o[u].z + sh[u].z);
                        if (rx * rx + ry * ry + rz * rz < a.rclose2) near_close_separation(a, p, src[u], rx, ry, rz);
                        near_pair_nz<DEG>(a, rx, ry, rz, o[u].w, phi, gx, gy, gz);
                    }
                hd = (hd + min(cnt, kEval)) & kMask;
            }
        };
        // rounds of chunks until some active lane holds fewer than kEval entries, as long as
        // no ring lacks room for half a block's rows (a block's hits go on in two halves,
        // with a check for room between them)
        constexpr int kRoom = kNearCap - 1 - kNearMfmaRows / 2;
        auto drain_ready = [&]() {
            while (true) {
                const int cnt = (tp - hd) & kMask;
                if (__ballot(act && cnt < kEval) != 0 && __ballot(cnt > kRoom) == 0) break;
                chunk();
            }
        };
        // float64 sink: the targets' positions and zeroed sums
        if constexpr (kF64) {
            if (half == 0) {
                tpos[0][jl] = txE;
                tpos[1][jl] = tyE;
                tpos[2][jl] = tzE;
#pragma unroll
                for (int c = 0; c < 4; ++c) tsum[c][jl] = (E)0;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // the stack's entries [s0, s0 + cnt) (cnt <= kRound, wave-uniform): entry s0 + 64 u
        // + lane for lane and round u
        auto evaluate = [&](int s0, int cnt) {
            if constexpr (kF64) {
                vec4<E> o[kEval], sh[kEval];
                int ti[kEval];
#pragma unroll
                for (int u = 0; u < kEval; ++u) {
                    const bool ok = 64 * u + lane < cnt;
                    const uint32_t e = ok ? stack[s0 + 64 * u + lane] : (uint32_t)tb;
                    ti[u] = ok ? (int)stackt[s0 + 64 * u + lane] : 0;
                    o[u] = a.pos[e & ((1u << kNearCodeShift) - 1)];
                    sh[u] = shiftE[e >> kNearCodeShift];
                }
                // the target of entry u + 1 is read while entry u is evaluated
                E ttx = tpos[0][ti[0]], tty = tpos[1][ti[0]], ttz = tpos[2][ti[0]];
#pragma unroll
                for (int u = 0; u < kEval; ++u) {
                    const int t = ti[u];
                    const E cx = ttx, cy = tty, cz = ttz;
                    if (u + 1 < kEval) {
                        ttx = tpos[0][ti[u + 1]];
                        tty = tpos[1][ti[u + 1]];
                        ttz = tpos[2][ti[u + 1]];
                    }
                    if (64 * u + lane < cnt) {
                        const E rx = cx - (o[u].x + sh[u].x), ry = cy - (o[u].y + sh[u].y), rz = cz - (o[u].z + sh[u].z);
                        // the float32 test admits pairs up to the margin beyond r_c: the cut
                        // at r_c is made here; the particle itself has r^2 = 0
                        const E r2 = rx * rx + ry * ry + rz * rz;
                        if (r2 < a.rc2 && r2 > (E)0) {
                            E ph = 0, fx = 0, fy = 0, fz = 0;
                            near_pair<E, DEG>(a, rx, ry, rz, o[u].w, ph, fx, fy, fz, r2);
                            atomicAdd(&tsum[0][t], ph);
                            atomicAdd(&tsum[1][t], fx);
                            atomicAdd(&tsum[2][t], fy);
                            atomicAdd(&tsum[3][t], fz);
                        }
                    }
                }
            }
        };
        int top = 0;  // float64 sink: stack height (wave-uniform)
        // this lane's candidate of a block at v0: the range it falls in, its particle and
        // shift.  Every lane starts from the range holding v0 (k0, uniform, found from
        // the previous block's) and moves on to each later range that starts at or
        // before its own position v0 + lane % 32.  The next block's record is loaded
        // while the current one is tested.
        int k0 = 0, kl = 0, bl = 0;
        float sx = 0.f, sy = 0.f, sz = 0.f;
        auto advance = [&](int v0) {
            while (k0 + 1 < 18 && __builtin_amdgcn_readlane(pre, k0 + 1) <= v0) ++k0;
            kl = k0;
            bl = __builtin_amdgcn_readlane(base, k0);
            sx = readlane_f(sk.x, k0);
            sy = readlane_f(sk.y, k0);
            sz = readlane_f(sk.z, k0);
            const int v = v0 + jl;
            for (int kk = k0 + 1; kk < 18 && __builtin_amdgcn_readlane(pre, kk) <= v0 + 31; ++kk) {
                const int bk = __builtin_amdgcn_readlane(base, kk);
                const float xk = readlane_f(sk.x, kk), yk = readlane_f(sk.y, kk),
                            zk = readlane_f(sk.z, kk);
                if (v >= __builtin_amdgcn_readlane(pre, kk)) {
                    kl = kk;
                    bl = bk;
                    sx = xk;
                    sy = yk;
                    sz = zk;
                }
            }
        };
        advance(0);
        bool vn = jl < total;
        uint32_t cn = (uint32_t)(vn ? bl + jl : tb) | ((uint32_t)kl << kNearCodeShift);
        vec4<float> on = pos32[cn & ((1u << kNearCodeShift) - 1)];
        float sxn = sx, syn = sy, szn = sz;
        for (int v0 = 0; v0 < total; v0 += 32) {
            const bool valid = vn;
            const uint32_t code = cn;
            float ux = on.x + sxn, uy = on.y + syn, uz = on.z + szn;
            float u2 = ux * ux + uy * uy + uz * uz;
            if (!valid) {
                ux = uy = uz = 0.f;
                u2 = 1e30f;
            }
            const float a1 = half ? uy : ux;
            const float a2 = half ? u2 : uz;
            if (half == 0) codes[jl] = code;
            near_v16f acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, b2, acc, 0, 0, 0);
            // while the matrix core works: the next block's record, and full rounds off the
            // top of the stack (the block's hits go on after them)
            if (v0 + 32 < total) {
                advance(v0 + 32);
                vn = v0 + 32 + jl < total;
                cn = (uint32_t)(vn ? bl + v0 + 32 + jl : tb) | ((uint32_t)kl << kNearCodeShift);
                on = pos32[cn & ((1u << kNearCodeShift) - 1)];
                sxn = sx;
                syn = sy;
                szn = sz;
            }
            if constexpr (kF64) {
                while (top >= kRound) {
                    top -= kRound;
                    evaluate(top, kRound);
                }
            } else {
                drain_ready();
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            uint4 cd[4];
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) cd[q4] = *reinterpret_cast<const uint4*>(&codes[8 * q4 + 4 * half]);
            if constexpr (kF64) {
                // the hits of row r of every lane go on in lane order: a lane's slot is the
                // height plus the hits of the lanes below it
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const uint32_t cr = r % 4 == 0 ? cd[r / 4].x : r % 4 == 1 ? cd[r / 4].y : r % 4 == 2 ? cd[r / 4].z : cd[r / 4].w;
                    const bool hit = acc[r] < thr;
                    const uint64_t m = __ballot(hit);
                    if (hit) {
                        const int slot = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)top));
                        stack[slot] = cr;
                        stackt[slot] = (uint8_t)jl;
                    }
                    top += __popcll(m);
                }
            } else {
                // every row is written at this lane's tail slot, which moves on for a hit: the
                // tail as a byte offset into the lists of all waves (wave, slot and lane bits
                // are disjoint, so stepping the slot is an add and an and-or).  Rows 0-7 (the
                // block's candidates 0-15), then rounds while some ring lacks room for 8
                // more, then rows 8-15.
#pragma unroll
                for (int h8 = 0; h8 < 2; ++h8) {
                    if (h8 == 1) {
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        while (__ballot(((tp - hd) & kMask) > kRoom)) chunk();
                    }
                    uint32_t at = lb | ((uint32_t)tp << 8);
#pragma unroll
                    for (int r = 8 * h8; r < 8 * h8 + 8; ++r) {
                        const uint32_t cr = r % 4 == 0 ? cd[r / 4].x : r % 4 == 1 ? cd[r / 4].y : r % 4 == 2 ? cd[r / 4].z : cd[r / 4].w;
                        *reinterpret_cast<uint32_t*>(hits_bytes + at) = cr;
                        const uint32_t nx = ((at + 256u) & ((uint32_t)kMask << 8)) | lb;
                        at = acc[r] < thr ? nx : at;
                    }
                    tp = (int)(at >> 8) & kMask;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if constexpr (kF64) {
            while (top > 0) {
                const int c = min(top, kRound);
                top -= c;
                evaluate(top, c);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (act && half == 0) a.part[a.orig[p]] = vec4<E>{tsum[0][jl], tsum[1][jl], tsum[2][jl], tsum[3][jl]};
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            while (__ballot(tp != hd)) chunk();
            phi += __shfl_xor(phi, 32, 64);
            gx += __shfl_xor(gx, 32, 64);
            gy += __shfl_xor(gy, 32, 64);
            gz += __shfl_xor(gz, 32, 64);
            if (act && half == 0) a.part[a.orig[p]] = vec4<E>{phi, gx, gy, gz};
        }
    }
    }
}
};

// The float32 copy of the float64 records (after the per-cell z sort) for the float32
// candidate test of float64 plans.
struct NearPos32K {
    static constexpr int kThreads = 256;
    __device__ static void run(GridPos g, const vec4<double>* __restrict__ pos, int n, vec4<float>* __restrict__ pos32) {
        for (int i = g.bid * kThreads + threadIdx.x; i < n; i += g.nb * kThreads) {
            const vec4<double> v = pos[i];
            pos32[i] = vec4<float>{(float)v.x, (float)v.y, (float)v.z, (float)v.w};
        }
    }
};

// polynomial degrees compiled; the fitted degree is rounded up to one of these
template <typename real, int DEG>
hipError_t launch_near_deg(Plan& p, const NearArgs<real>& a, int blocks) {
    return launch<NearMfmaK<DEG, real>>(p, blocks, 0, a);
}

template <typename real>
hipError_t launch_near_kernel(Plan& p, const NearArgs<real>& a, int blocks) {
    if (a.deg <= 8) return launch_near_deg<real, 8>(p, a, blocks);
    if (a.deg <= 10) return launch_near_deg<real, 10>(p, a, blocks);
    if (a.deg <= 12) return launch_near_deg<real, 12>(p, a, blocks);
    if (a.deg <= 14) return launch_near_deg<real, 14>(p, a, blocks);
    if (a.deg <= 16) return launch_near_deg<real, 16>(p, a, blocks);
    if (a.deg <= 20) return launch_near_deg<real, 20>(p, a, blocks);
    if (a.deg <= 24) return launch_near_deg<real, 24>(p, a, blocks);
    if (a.deg <= 32) return launch_near_deg<real, 32>(p, a, blocks);
    if (a.deg <= 48) return launch_near_deg<real, 48>(p, a, blocks);
    return launch_near_deg<real, kMaxNearDeg>(p, a, blocks);
}

template <typename real>
hipError_t run_near(Plan& p, const double* x, const double* q, int stages) {
    const Resolved& r = p.r;
    // the float32 kernel evaluates the monomial form, which the planner gives up to degree 24
    if (sizeof(real) == 4 && r.near_deg > 24) return hipErrorInvalidConfiguration;
    Workspace& ws = p.ws;
    const int n = (int)r.n;
    NearGeom g;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = r.L[d];
        g.ch[d] = r.ch[d];
        g.nc[d] = r.nc[d];
    }
    const int ncells = r.nc[0] * r.nc[1] * r.nc[2];
    if (stages & 1) {
        const int t = timer_id(p, "near_sort");
        timer_begin(p, t);
        const int blocks = std::min((n + 255) / 256, 8192);
        hipError_t e = launch_fill_int(p, ws.cell_start, 0, (int64_t)ncells + 1);
        if (e == hipSuccess) e = launch_fill_bytes_zero(p, ws.qsum, 2 * kQsumSlots * sizeof(double));
        if (e == hipSuccess) e = launch_fill_int(p, ws.status, 0, 1);
        if (e == hipSuccess)
            e = launch<NearKeyK>(p, blocks, 0, x, q, n, g, (int2*)ws.key, ws.cell_start, ws.qsum, ws.status);
        if (e == hipSuccess) e = launch_exclusive_scan(p, ws.cell_start, ncells + 1, ws.scan_tmp);
        if (e == hipSuccess && r.deterministic)
            e = launch_canonical_ranks(p, ws.key, true, n, ws.cell_start, ncells, nullptr, ws.det_idx, nullptr);
        if (e == hipSuccess)
            e = launch<NearPackK<real>>(p, blocks, 0, x, q, n, g, (const int2*)ws.key, (const int*)ws.cell_start,
                                        (vec4<real>*)ws.near_pos, ws.near_orig);
        const int ncols = r.nc[0] * r.nc[1];
        if (e == hipSuccess)
            e = launch<NearZsortK<real>>(p, (ncells + 3) / 4, 0, (const int*)ws.cell_start, ncells,
                                         (vec4<real>*)ws.near_pos, ws.near_orig, ws.status);
        if (e == hipSuccess && sizeof(real) == 8)
            e = launch<NearPos32K>(p, std::min((n + 255) / 256, 4096), 0, (const vec4<double>*)ws.near_pos, n,
                                   (vec4<float>*)ws.near_pos32);
        if (e == hipSuccess)
            e = launch<NearChunksK>(p, ncols, 0, (const int*)ws.cell_start, r.nc[2], near_chunk_extra(r.nc[2]),
                                    (int4*)ws.near_units, near_grab(ws, near_unit_slots(r)));
        timer_end(p, t);
        if (e != hipSuccess || !(stages & 2)) return e;
    }
    NearArgs<real> a;
    a.pos = (const vec4<real>*)ws.near_pos;
    a.orig = ws.near_orig;
    a.units = (const int4*)ws.near_units;
    a.grab = near_grab(ws, near_unit_slots(r));
    a.status = ws.status;
    a.zcut = (float)(r.rc * (1.0 + 1e-5) + 1e-4 * r.ch[2]);
    a.max_units = (int)near_unit_slots(r);
    a.cell_start = ws.cell_start;
    a.part = (vec4<real>*)ws.parts;
    for (int d = 0; d < 3; ++d) {
        a.nc[d] = r.nc[d];
        a.ch[d] = (real)r.ch[d];
    }
    a.rc2 = (real)(r.rc * r.rc);
    a.inv_rc2 = (real)(1.0 / (r.rc * r.rc));
    a.x = x;
    a.L[0] = r.L[0];
    a.L[1] = r.L[1];
    a.rclose2 = (real)(r.rc * r.rc / (32.0 * 32.0));
    a.pos32 = sizeof(real) == 4 ? (const vec4<float>*)ws.near_pos : (const vec4<float>*)ws.near_pos32;
    // the float32 test's rounding stays below 1e-5 r_c^2 (coordinates within a few cells of
    // the unit's centre); float64 plans admit 4e-5 r_c^2 more and cut exactly
    a.test_margin = sizeof(real) == 4 ? 0.f : (float)(4e-5 * r.rc * r.rc);
    a.deg = r.near_deg;
    for (int k = 0; k <= kMaxNearDeg; ++k) {
        a.cF[k] = (real)r.near_cF[k];
        a.cG[k] = (real)r.near_cG[k];
        a.mF[k] = (real)r.near_mF[k];
        a.mG[k] = (real)r.near_mG[k];
    }
    const int t = timer_id(p, "near");
    timer_begin(p, t);
    // persistent blocks in groups of 8 (one per XCD's share of the units)
    const int want = std::min(p.num_cus * kNearBlocksPerCU, (a.max_units + kNearWaves - 1) / kNearWaves);
    const hipError_t e = launch_near_kernel<real>(p, a, std::max(8, (want + 7) / 8 * 8));
    timer_end(p, t);
    return e;
}

}  // namespace

hipError_t launch_near(Plan& p, const double* x, const double* q, int stages) {
    if (p.r.prec == SOG_PREC_FP64) return run_near<double>(p, x, q, stages);
    return run_near<float>(p, x, q, stages);
}

}  // namespace sog
