// Internal declarations of the SOG library: the resolved plan, the device
// workspace and the kernel launchers.  Host code only (no device code here).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sog.h"

namespace sog {

constexpr int kMaxStages = 24;    // radix stages of one 1D FFT
constexpr int kMaxNearDeg = 63;   // Chebyshev degree of the near-field polynomials
constexpr int kMaxMid = 96;       // max number of mid-range Gaussians (m + 1)
constexpr int kMidSub = 8;        // rank counters per mid-range tile in the counting sort (fewer atomics per address)
static_assert((kMidSub & (kMidSub - 1)) == 0, "kMidSub is a power of two");
constexpr int kQsumSlots = 64;    // slots of the charge sums (spreads the float64 atomics of the key pass)
// Colour of tile t in one direction for the deterministic gridding, which adds the tiles'
// blocks (tile plus (P_w - 1)/2 nodes each side) into the grid one colour at a time with
// plain read-add-writes.  Two tiles of one colour must be at least m tiles apart, m - 1
// full tiles covering the P_w - 1 nodes of the two half-widths; so t mod m, except in a
// periodic direction (x, y), where the first q m tiles take t mod m and every tile after
// them (the short last tile among them) a colour of its own, m, m + 1, ...; the planner
// picks m and q (Resolved::dcol_m, dcol_q).
constexpr int tile_colour(int t, bool periodic, int m, int q) {
    return (!periodic || t < q * m) ? t % m : m + (t - q * m);
}

constexpr int kMaxWinPoly = 16;   // highest degree of a polynomial window
// coefficients per node in the device table of a polynomial window of degree nu: nu + 1
// rounded up to a multiple of 4 (leading zeros)
constexpr int window_poly_row(int nu) { return (nu + 1 + 3) / 4 * 4; }
constexpr int kMaxPw = 15;        // widest mid-range window the gridding and gathering kernels take
constexpr int kSpreadStage = 32;  // particles whose window weights the gridding kernel stages at a time
// LDS of one gridding or gathering workgroup at most: for narrow float32 windows (P_w <=
// 9) three workgroups share the 160 KiB of a compute unit (more waves to hide the
// per-particle LDS round trips: 0.55 -> 0.48 ms gridding and 0.20 -> 0.15 ms gathering at
// P_w = 7, N = 1e6), otherwise two (larger tiles waste less on the halo: at P_w = 11 the
// smaller budget was 8% slower in all, and float64 tiles, with twice the bytes per node,
// were 1.6x slower at P_w = 9)
constexpr size_t kTileLdsBytes = 81920;  // the largest budget
inline size_t tile_lds_budget(int Pw, size_t real_bytes) { return (real_bytes == 4 && Pw <= 9) ? 53248 : kTileLdsBytes; }

// LDS layout of the mid-range gridding kernel: the tile plus its (P_w - 1) halo (and
// 4 ceil(P_w / 4) - P_w padding planes), 64 sink slots for masked lanes, and per staged
// particle its y and z window weights and a zero (2 P_w + 1 reals); then, on a 32-byte
// boundary, the staged particles' x weights rotated for the four plane groups (16 reals
// each, read four at a time), their offsets from their grid points and charges (real4
// each), the four groups' plane offsets (int4) and the x nodes (int).
inline size_t spread_lds_offset_records(size_t real_bytes, int Pw, int Bx, int By, int Bz) {
    const size_t plane = (size_t)(By + Pw - 1) * (Bz + Pw - 1);
    const size_t tot = (size_t)(Bx + Pw - 1 + 4 * ((Pw + 3) / 4) - Pw) * plane;
    return ((tot + 64 + (size_t)kSpreadStage * (2 * Pw + 1)) * real_bytes + 31) / 32 * 32 +
           (size_t)kSpreadStage * 16 * real_bytes;
}
inline size_t spread_lds_bytes(size_t real_bytes, int Pw, int Bx, int By, int Bz) {
    return spread_lds_offset_records(real_bytes, Pw, Bx, By, Bz) + (size_t)kSpreadStage * (4 * real_bytes + 20);
}

// LDS of the direct long range's moments kernel (kMomThreads threads) for a batch of ch
// particles: the P Chebyshev rows (ch + pad reals each, rounded up to 4 entries), the
// 2 n_kx + 1 and n_ky + 1 rows of plane waves (ch + 4 pad complex each) and the threads'
// 4 complex partial sums.  pad = 1 staggers the rows across the LDS banks.
constexpr int kMomThreads = 256;
constexpr int kMomMinChunk = 16;
constexpr size_t kMomMaxLds = 65536;
inline size_t long_moments_lds(size_t real_bytes, int P, int nkx, int nky, int ch, int pad) {
    const size_t rows = (size_t)(2 * nkx + 1) + (size_t)(nky + 1);
    return ((size_t)P * (ch + pad) + 3) / 4 * 4 * real_bytes + rows * (ch + 4 * pad) * 2 * real_bytes +
           (size_t)kMomThreads * 4 * 2 * real_bytes;
}

// Row stride (complex entries) of the mid-range half spectrum: I_z*/2 + 1 rounded up to a
// multiple of 16, so that the 16-entry row segments the y and x passes move are whole
// 128-byte lines.
inline int cgrid_stride(int Izs) { return ((Izs / 2 + 1) + 15) / 16 * 16; }

// A 1D FFT of length n as a product of small radices (Stockham, natural order).
struct FFTFactors {
    int n = 0;
    int nstages = 0;
    int radix[kMaxStages] = {0};
};

// Everything the planner decides (float64, host).  Symbols follow the paper.
// Longest line the LDS line transforms take (a batch holds at most this many elements):
// 4608 complex in the float32 form, 2304 in float64.
constexpr int fft_max_line(int prec) { return prec == SOG_PREC_FP64 ? 2304 : 4608; }
// lines of length n that the line kernels transform per batch: a power of two, at most
// 16, with n W <= fft_max_line
inline int fft_lines_per_batch(int prec, int n) {
    int W = 16;
    while (W > 1 && (int64_t)n * W > fft_max_line(prec)) W >>= 1;
    return W;
}
// dynamic LDS of one FFT line block at most (above 64 KiB, as the gridding's 80 KiB tiles)
constexpr size_t kFFTLdsBudget = 98304;

// LDS of the mid-range x pass (forward FFT along x, multiplier, inverse) with W lines per
// block: the lines (complex), the x multipliers of the nl mid-range Gaussians and the
// staging of each thread's line loads (k_fft.hip).
inline size_t fft_x_lds_bytes(int prec, int Ix, int nl, int W) {
    const size_t rs = prec == SOG_PREC_FP64 ? 8 : 4;
    const size_t stage = (size_t)(fft_max_line(prec) / 256) * (256 / W);
    return (size_t)Ix * (W + 1) * 2 * rs + ((size_t)nl * (W + Ix) + stage - Ix) * rs;
}

// The same without the x multipliers (read from global memory instead)
inline size_t fft_x_lds_min_bytes(int prec, int Ix, int nl, int W) {
    const size_t rs = prec == SOG_PREC_FP64 ? 8 : 4;
    return (size_t)Ix * (W + 1) * 2 * rs + (size_t)nl * W * rs;
}

// Transform of the ES window in grid units, What_g(kappa) = int psi(d) cos(kappa d) dd
// over |d| < P_w/2 (planner.cpp); the physical transform is h What_g(k h).
double es_hat_grid(double kappa, int Pw, double beta);
double kb_value_grid(double d, int Pw, double beta);
double kb_hat_grid(double kappa, int Pw, double beta);
void window_poly_fit(int Pw, double beta, int nu, std::vector<double>& coef);
double window_poly_error(int Pw, double beta, int nu, const std::vector<double>& coef, double* derr);
int window_poly_degree(int Pw, double beta, double eps);

struct Resolved {
    double L[3] = {0, 0, 0};
    int64_t n = 0;
    double tol = 0;
    int prec = SOG_PREC_FP64;
    bool deterministic = false;  // canonical bin orders and coloured gridding (no float atomics)
    int dcol_m[3] = {1, 1, 1};   // deterministic gridding: tile_colour's m, q and the colours
    int dcol_q[3] = {0, 0, 0};   // per direction
    int dcol_n[3] = {1, 1, 1};
    double eta = 0;              // range-splitting factor as given (0: m chosen by cost)

    // decomposition (Sec. 2.2)
    double b = 0, r0 = 0, omega = 0, rc = 0, sigma = 0;
    int M = 0, m = -1;
    std::vector<double> w, s;
    double self_coeff = 0;  // sum_l w_l

    // near field: cells of side >= r_c; polynomials in x = 2 r^2/r_c^2 - 1
    int nc[3] = {1, 1, 1};
    double ch[3] = {0, 0, 0};
    int near_deg = 0;
    double near_cF[kMaxNearDeg + 1] = {0};  // F(r)
    double near_cG[kMaxNearDeg + 1] = {0};  // F'(r)/r
    // the same polynomials in monomial form, F = sum_k near_mF[k] x^k (float32 plans, whose
    // degree stays small enough for the conversion; evaluated by Horner)
    double near_mF[kMaxNearDeg + 1] = {0};
    double near_mG[kMaxNearDeg + 1] = {0};

    // mid range (Alg. al::mid)
    bool has_mid = false;
    int I[3] = {0, 0, 0};  // I_x, I_y, I_z (intervals over the box)
    int Izs = 0;           // padded z points I_z*
    int Pw = 0;            // window points (same in every direction)
    double S = 0;          // Gaussian window shape
    int window = SOG_WINDOW_GAUSSIAN;  // SOG_WINDOW_GAUSSIAN, SOG_WINDOW_ES or SOG_WINDOW_KB
    double beta = 0;       // ES / KB window shape
    int nu = 0;            // KB: degree of the window's polynomials
    double h[3] = {0, 0, 0};
    double H[3] = {0, 0, 0};
    double Lzs = 0;
    // stored z planes [zband[0], zband[1]) (even bounds) that can carry window mass for
    // z in [0, L_z]: the z transforms read and write only these, the rest stays zero
    int zband[2] = {0, 0};
    int B[3] = {0, 0, 0};      // spread/gather tile
    // gridding: (y, z) window node of each lane in each of up to 4 passes of 64 lanes
    // (-1: none), chosen so that the 64 nodes of a pass fall in distinct LDS banks
    signed char node_oy[4 * 64] = {0};
    signed char node_oz[4 * 64] = {0};
    bool spread_dummy = false;  // every lane without a node has a dummy node (oz >= P_w)
    int ntile[3] = {0, 0, 0};

    // long range (Sec. 3.3 / App. B)
    bool has_long = false;
    int form = SOG_LONG_DIRECT;
    int P = 0;
    int nk[2] = {0, 0};        // direct form
    int nh = 0;                // half-plane modes of the direct form
    int I2[2] = {0, 0};        // FFT form grid
    int Pw2 = 0;
    double S2 = 0;
    double h2[2] = {0, 0};
    double H2[2] = {0, 0};
    int ntile2[2] = {0, 0};    // tiles of kLong2Tile x kLong2Tile nodes
    int Q = 0;                 // FFT form: Taylor terms of the z kernel (App. C); 0: exact kernel
    int Ps = 0;                // FFT form: source planes (P exact, 2Q - 1 Taylor); P target planes
};

// The long range's FFT form: gridding and gathering tiles of kLong2Tile^2 nodes; at most
// kLong2MaxPlanes source or target planes (Chebyshev terms in z).
constexpr int kLong2Tile = 16;
constexpr int kLong2MaxPlanes = 32;

// Near-field work units: chunks of at most kNearChunk consecutive targets of a column
// within at most kNearUnitCells cells, formed greedily; a column of
// ncz cells needs at most floor(count / kNearChunk) full chunks, one last chunk and
// ceil(ncz / kNearUnitCells) - 1 chunks cut short (their first cells lie below
// ncz - kNearUnitCells, kNearUnitCells apart), so column c's slots start at
// floor(first particle of c / kNearChunk) + c * (ceil(ncz / kNearUnitCells) + 1), one
// slot of slack per column.
constexpr int kNearUnitCells = 7;
constexpr int kNearChunk = 32;
inline int near_chunk_extra(int ncz) { return (ncz + kNearUnitCells - 1) / kNearUnitCells + 1; }

#if defined(__HIP__)
#define SOG_HOST_DEVICE __host__ __device__
#else
#define SOG_HOST_DEVICE
#endif
// The greedy chunking of one column, given its ncz + 1 cell starts cs (particle indices):
// emit(first cell, first target, end target, end cell) for each chunk in z order;
// returns the number of chunks.
template <class Emit>
SOG_HOST_DEVICE inline int near_chunk_walk(const int* cs, int ncz, Emit&& emit) {
    const int pend = cs[ncz];
    int p = cs[0], z = 0, u = 0;
    while (p < pend) {
        while (cs[z + 1] <= p) ++z;  // the cell holding p
        const int za = z;
        int e = p + kNearChunk < pend ? p + kNearChunk : pend;
        const int lim = za + kNearUnitCells < ncz ? za + kNearUnitCells : ncz;
        if (cs[lim] < e) e = cs[lim];
        int zb = za;
        while (cs[zb + 1] < e) ++zb;  // the cell holding e - 1
        emit(za, p, e, zb + 1);
        ++u;
        p = e;
    }
    return u;
}
inline int64_t near_unit_slots(const Resolved& r) {
    const int64_t ncols = (int64_t)r.nc[0] * r.nc[1];
    return r.n / kNearChunk + ncols * near_chunk_extra(r.nc[2]);
}

struct RecLaunch;  // launch.hpp

struct KernelTimer {
    const char* name;
    double total_ms = 0;
    int64_t launches = 0;
};

// Device workspace; every pointer is owned by the plan.
struct Workspace {
    // staging of host inputs/outputs
    double* x = nullptr;
    double* q = nullptr;
    double* phi = nullptr;
    double* force = nullptr;
    double* energy = nullptr;
    // validation: [0] sum q, [1] sum |q| (double), status bits in an int
    double* qsum = nullptr;     // kQsumSlots x (sum q, sum |q|): block b adds into slot b mod kQsumSlots
    int* status = nullptr;
    // per-part results in the particles' own order, one record per particle and part
    void* parts = nullptr;      // 3 x n x real4 (phi, dphi/dx, dphi/dy, dphi/dz): near, mid, long
    // counting sorts
    int* key = nullptr;       // 2n: near-field (cell, rank) pairs; the long-range FFT form reuses n of it
    int* perm = nullptr;      // n
    int* scan_tmp = nullptr;  // block sums
    int* key2 = nullptr;      // 2n: the mid range's (tile, rank) pairs (it runs on the main stream while
    int* scan_tmp2 = nullptr; //    the near field and long range sort on the side stream)
    // near field
    int* cell_start = nullptr;  // ncells + 1
    int* near_orig = nullptr;   // n
    void* near_pos = nullptr;   // n x real4 (x, y, z relative to the cell corner; q)
    void* near_pos32 = nullptr; // float64 plans: n x float4, the same records in float32
    void* near_units = nullptr; // near_unit_slots() int4 work units, then 8 work counters
    // mid range
    int* tile_start = nullptr;  // ntiles * kMidSub + 1: tile t owns [tile_start[t kMidSub], tile_start[(t+1) kMidSub])
    signed char* spread_nodes = nullptr;  // 2 x 256: node_oy, node_oz of the plan
    int* mid_g = nullptr;       // n x int4 (grid point of each sorted particle, original index)
    void* mid_u = nullptr;      // n x real4 (offset from the grid point in units of h, q)
    void* grid = nullptr;       // I_x I_y I_z* reals
    void* cgrid = nullptr;      // I_x I_y rows of I_z*/2 + 1 complex, row stride cgrid_stride(I_z*)
    void* tw_x = nullptr;       // twiddles e^{-2 pi i t/n} for each FFT length
    void* tw_y = nullptr;
    void* tw_z = nullptr;       // length I_z*/2
    void* tw_zpost = nullptr;   // e^{-2 pi i k / I_z*}, k = 0..I_z*/2
    void* mult_ax = nullptr;    // (m+1) x I_x: exp(-s^2 kx^2/4) / What_x^2
    void* mult_ay = nullptr;    // (m+1) x I_y
    void* mult_az = nullptr;    // (m+1) x (I_z*/2+1)
    void* mult_c = nullptr;     // (m+1): pi^{3/2} w_l s_l^3 / (I_x I_y I_z*)
    void* wpoly = nullptr;      // KB window: P_w x (nu+1) monomial coefficients per node (real)
    // long range
    int* long_modes = nullptr;  // nh x int2 (direct form)
    double* long_kt = nullptr;  // per mode P x P kernel in the Chebyshev basis (float64)
    double* long_mu = nullptr;  // nh x P x blocks complex partial moments (float64)
    void* long_a = nullptr;     // nh x P complex coefficients a(k,n) (real type)
    int long_blocks = 0;
    // FFT form of the long range
    int* l2_tile_start = nullptr;  // ntiles + 1
    int* l2_tile_cursor = nullptr; // ntiles
    // deterministic mode: bin member lists (near field / long range, mid range) and the
    // long range's canonical ranks (n ints each)
    int* det_idx = nullptr;
    int* det_idx2 = nullptr;
    int* det_rank = nullptr;
    int* l2_g = nullptr;        // n x int4 (gx, gy, -, orig), in tile order
    void* l2_u = nullptr;       // n x real4 (ux, uy, t = 2z/Lz, q)
    void* l2_grid = nullptr;    // max(P_s, P) planes of I2x x I2y reals
    void* l2_cgrid = nullptr;   // max(P_s, P) planes of I2x rows of cgrid_stride(I2y) complex
    void* l2_tw_x = nullptr;    // e^{-2 pi i t / I2x}
    void* l2_tw_y = nullptr;    // e^{-2 pi i t / (I2y/2)}
    void* l2_tw_ypost = nullptr;  // e^{-2 pi i k / I2y}, k <= I2y/2
    void* l2_kt_r = nullptr;    // exact kernel: (I2x/2+1) x (I2y/2+1) x P x P, divided by What2^2 and I2x I2y
    void* l2_el = nullptr;      // Taylor: s_l^2/4 per long-range Gaussian
    void* l2_coef = nullptr;    // Taylor: (M - m) x Q, pi ((-1)^p/p!) w_l L_z^{2p} s_l^{2-2p} / (I2x I2y)
    void* l2_bp = nullptr;      // Taylor: Q x P x P_s
    void* l2_winv_x = nullptr;  // Taylor: 1/What2_x(k_x)^2, I2x
    void* l2_winv_y = nullptr;  // Taylor: 1/What2_y(k_y)^2, I2y/2 + 1
    // energy reduction
    double* red = nullptr;
    int red_blocks = 0;
    size_t bytes = 0;  // device bytes the plan holds: tables and its per-call region
};

struct TunedCandidate {
    double rc;
    int m;
    double ms;
};

struct Plan {
    Resolved r;
    Workspace ws;
    std::vector<TunedCandidate> tuning;  // autotuned plans: the discretisations timed
    int device = 0;
    int num_cus = 256;              // compute units of the device
    hipStream_t stream = nullptr;   // the stream kernels are launched on (the caller's, or side)
    hipStream_t side = nullptr;     // plan-owned stream: near field and long range
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_grid = nullptr;
    bool on_device = false;
    bool check = true;
    bool timing = false;
    // the call's kernels replayed as a HIP graph, captured at the first call on a
    // plan-owned stream (inputs and outputs staged in the plan's buffers)
    bool graphable = false;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    FFTFactors fx, fy, fz;          // mid-range FFT lengths I_x, I_y, I_z*/2
    FFTFactors f2x, f2y;            // long-range FFT form: I2x and I2y/2 (real-to-complex along y)
    // per-call buffers: one region of region_bytes (offsets in region_slots) that the plan
    // allocates, unless static_region (then every call binds a region of its own)
    void* region = nullptr;
    size_t region_bytes = 0;
    bool static_region = false;
    std::vector<std::pair<void**, size_t>> region_slots;
    // when set, kernel launches are recorded here instead of launched (batches, launch.hpp)
    std::vector<RecLaunch>* rec = nullptr;
    std::vector<KernelTimer> timers;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
};

// planner.cpp
// A feasible discretisation the planner considered: its modelled cost, r_c and split m.
struct PlanCandidate {
    double cost;
    double rc;
    int m;
};
// cands (optional): every feasible (r_c, m) the planner's search met, with its cost
sog_status resolve(const double box[3], int64_t n, double tol, const sog_options& opt, Resolved& r,
                   std::string& err, std::vector<PlanCandidate>* cands = nullptr);
bool factor_fft(int n, FFTFactors& f);
int next_smooth(int n, bool even);
void near_chebyshev(Resolved& r);
void long_kernel_cheb_basis(const Resolved& r, const double* k2, int nk, double* out);
void cheb_V_inverse(int P, double* C);

// error reporting
void set_error(const std::string& msg);

// kernel launchers (k_*.hip); every launcher checks its own shapes on the host
struct Timed;  // RAII helper in api.cpp
hipError_t launch_fill_int(Plan& p, int* ptr, int value, int64_t n);
hipError_t launch_fill_bytes_zero(Plan& p, void* ptr, size_t bytes);
// per-system charge sums and flags of a batch of systems stored one after another
// (off: nsys + 1 device offsets; lz: nsys heights; qsum: 2 nsys; status: nsys)
hipError_t launch_batch_check(const double* x, const double* q, const int64_t* off, int nsys, const double* lz,
                              int64_t n, double* qsum, int* status, hipStream_t s);
hipError_t launch_counting_sort(Plan& p, const int* key, int n, int nbins, int* start, int* cursor, int* perm);
// zero the counts (nbins + 1) and cursors (nbins) of a counting sort whose histogram the
// caller's key kernel builds; launch_exclusive_scan then turns counts into starts
hipError_t launch_exclusive_scan(Plan& p, int* data, int nbins, int* tmp);  // in place; tmp: block sums
// deterministic mode: after a counting sort's scan (start: nbins + 1 bin starts), rank the
// members of every bin by particle index.  pairs: key holds (bin, rank) int2 records and
// the ranks are replaced in place; else key holds bins (int), the ranks go to rank[i], and
// cursor (nbins ints) is scratch.  idx: n ints of scratch.
hipError_t launch_canonical_ranks(Plan& p, int* key, bool pairs, int n, const int* start, int nbins, int* cursor,
                                  int* idx, int* rank);
// stages (bit mask): near 1 = cell sort, 2 = pair kernel; mid 1 = tile sort and gridding,
// 2 = FFT chain and gathering
hipError_t launch_near(Plan& p, const double* x, const double* q, int stages = 3);
hipError_t launch_mid(Plan& p, const double* x, const double* q, int stages = 3);
hipError_t launch_long(Plan& p, const double* x, const double* q);
hipError_t launch_combine(Plan& p, const double* q, double* phi, double* force, double* grad, double* energy);
hipError_t launch_parts_out(Plan& p, double* phi_parts, double* grad_parts);
hipError_t launch_zero_parts(Plan& p, int part);

// timing hooks (api.cpp)
void timer_begin(Plan& p, int id);
void timer_end(Plan& p, int id);
int timer_id(Plan& p, const char* name);

}  // namespace sog
