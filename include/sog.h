/*
 * sog.h -- C ABI of the MI355X (gfx950) fast spectral sum-of-Gaussians solver for
 * quasi-2D electrostatics: x and y periodic, z free.
 *
 * The problem (paper Sec. 2.1, eqs. Poisson, chargeneutral, Phi): N point charges
 * q_i at r_i in the box [0,Lx) x [0,Ly) x [0,Lz], periodic in x and y, free in z,
 * with sum_i q_i = 0.  In Gaussian units
 *
 *     Phi_i = sum_j sum'_{n in Z^2 x {0}} q_j / |r_i - r_j + n o L|     (prime: no j = i, n = 0)
 *     U     = 1/2 sum_i q_i Phi_i
 *     F_i   = -q_i grad Phi(r_i) = -dU/dr_i
 *
 * The solver splits 1/r with the u-series sum-of-Gaussians decomposition
 * (eq. SOGdecomp): a near-field part summed directly over cell lists (eq. phiNDR),
 * a mid-range part by a 3D Fourier spectral solver without upsampling (Alg. al::mid),
 * and a long-range part by a Fourier-Chebyshev solver with Chebyshev interpolation
 * and anterpolation in z (Alg. al::long_nonfft, or Alg. al::long with 2D FFTs), and
 * subtracts the self term (eq. phiNDR).  Every step runs in the library's own HIP
 * kernels (including its FFTs); the host only plans.
 *
 * Conventions shared by every entry point
 *   - Coordinates: x (n x 3, row-major, float64).  x and y may be any finite value
 *     (wrapped modulo Lx, Ly); z must lie in [0, Lz].
 *   - Charges: q (n, float64), charge neutral to |sum q| <= 1e-10 sum |q|
 *     (Prop. lem::summation: the lattice sum converges only for a neutral cell).
 *   - Ownership: the caller owns x, q and all outputs; the plan owns all device
 *     workspace, allocated at plan time.  Pointers are host pointers unless the plan
 *     was created with options.pointers_on_device = 1, in which case every array
 *     argument (inputs and outputs) is a device pointer on options.device.
 *   - Streams: all work of a call is ordered on options.stream (NULL = the default
 *     stream).  A call returns after its results are complete when pointers are on
 *     the host, or when check_inputs is on; otherwise it may return before the
 *     device finishes (outputs are then ready in stream order).
 *   - Errors: every entry point returns a status and never aborts the process.
 *     Outputs are unspecified when the status is not SOG_OK.  sog_last_error()
 *     returns a message for the last failure on the calling thread.
 *   - Thread safety: a plan must not be used by two calls at once; distinct plans
 *     are independent.
 */
#ifndef SOG_H
#define SOG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sog_plan_s* sog_plan_t;

typedef enum {
    SOG_OK = 0,
    SOG_ERR_INVALID_ARG = 1,     /* null pointer, n <= 0, bad box, non-finite input, bad override */
    SOG_ERR_NOT_NEUTRAL = 2,     /* |sum q| > 1e-10 sum |q| (Prop. lem::summation)                */
    SOG_ERR_OUT_OF_BOX = 3,      /* some z outside [0, Lz]                                          */
    SOG_ERR_TOL_UNREACHABLE = 4, /* tol outside [1e-12, 1e-2] (FP64) or [1e-5, 1e-2] (FP32 bulk),  */
                                 /* or no discretisation within the kernels' limits reaches tol     */
                                 /* (Gaussian windows of at most 15 points, FFT lines of at most    */
                                 /* 4608 / 2304 points): about 1e-8 for boxes that need the mid     */
                                 /* range                                                            */
    SOG_ERR_OUT_OF_MEMORY = 5,   /* device allocation failed, or above SOG_MAX_DEVICE_BYTES       */
    SOG_ERR_DEVICE = 6           /* any other HIP runtime error                                    */
} sog_status;

typedef enum {
    SOG_PREC_FP64 = 0,      /* every step in float64                                             */
    SOG_PREC_FP32_BULK = 1  /* spread, FFTs, gathers, near and long-range arithmetic in float32;  */
                            /* float64 for the decomposition, tables, reductions over particles  */
                            /* and the final energy; particle coordinates enter float32 only as  */
                            /* offsets from a cell or grid point, formed in float64              */
} sog_precision;

typedef enum { SOG_LONG_AUTO = 0, SOG_LONG_DIRECT = 1, SOG_LONG_FFT = 2 } sog_long_form;

/* Mid-range window.  GAUSSIAN: the truncated Gaussian of eq. GS, shape mid_S.  ES: the
 * "exponential of semicircle" W(x) = exp(beta (sqrt(1 - (x/a)^2) - 1)), |x| < a = P_w h/2,
 * a compactly supported window of the Kaiser-Bessel family the paper's experiments use
 * (Sec. 5; the paper prints no formula for it), shape mid_beta; its transform is computed
 * by quadrature.  KB: the Kaiser-Bessel window W(x) = I_0(beta sqrt(1 - (x/a)^2)) / I_0(beta),
 * |x| <= a, shape mid_beta, with its closed-form transform; the kernels evaluate it as in
 * Remark rmk::PWindow, by polynomials of degree mid_nu (Chebyshev interpolation of each
 * node's weight over the particle's offset from its nearest node).  AUTO: the cheapest
 * that meets the tolerance (the Gaussian when mid_S is given; KB over ES on a tie: the ES
 * window's derivative is unbounded at its support's edge, which costs float32 gradients). */
typedef enum { SOG_WINDOW_AUTO = 0, SOG_WINDOW_GAUSSIAN = 1, SOG_WINDOW_ES = 2, SOG_WINDOW_KB = 3 } sog_window;

/*
 * Discretisation parameters.  In options, a zero field means "choose it from tol";
 * sog_plan_info() returns the fully resolved set.  Symbols follow the paper.
 */
typedef struct {
    /* SOG decomposition (Sec. 2.2-2.3, Table 1): b, r0, omega as a set, or all 0. */
    double b, r0, omega;
    double rc;          /* near-field cutoff r_c (sigma = r_c / r0), <= min(Lx,Ly)/2      */
    int32_t M;          /* index of the last Gaussian, w_0..w_M                            */
    int32_t m;          /* index of the last mid-range Gaussian (Sec. 3.1); -1: no mid    */
    int32_t set_m;      /* options only: 1 = use m as given (else chosen by cost)         */
    /* mid range (Alg. al::mid, Sec. 3.4): I_x, I_y, I_z grid intervals over the box,  */
    /* I_z* points in the padded free direction (even), window points P_w (odd) and   */
    /* the Gaussian window shape S (eq. GS).                                           */
    int32_t mid_I[3];
    int32_t mid_Izs;
    int32_t mid_Pw[3];
    double mid_S;
    /* long range (Sec. 3.3, App. B): form, Chebyshev points P, Fourier modes          */
    /* |n_x| <= nk_x, |n_y| <= nk_y for the direct form, or an I^long grid, window     */
    /* points and shape for the FFT form.                                              */
    int32_t long_form;
    int32_t long_P;
    int32_t long_nk[2];
    int32_t long_I[2];
    int32_t long_Pw[2];
    double long_S;
    /* mid-range window (sog_window) and the ES / KB shape beta (0: chosen)            */
    int32_t mid_window;
    double mid_beta;
    /* FFT form of the long range: the z kernel in App. C's Taylor form with long_Q    */
    /* terms (Lemma lemma::Taylor; 2 long_Q - 1 source planes), or -1: the exact       */
    /* kernel interpolated at the Chebyshev nodes (long_P source planes); 0: chosen.   */
    int32_t long_Q;
    /* KB window: degree nu of its polynomials, in [2, 16] (0: chosen, Sec. 4: the     */
    /* smallest whose weights are within tol/20 of the window)                         */
    int32_t mid_nu;
    /* range-splitting factor eta (Sec. 3.1, the range-splitting definition): the     */
    /* Gaussians with s_l <= eta L_z are mid range, the rest long range, so            */
    /* m = max{l : s_l <= eta L_z} (-1 if none); 0: m chosen by cost; ignored when     */
    /* set_m is 1.  Resolved: the given eta, or s_m / L_z of the split (0 if m = -1).  */
    double eta;
} sog_params;

typedef struct {
    int32_t precision;          /* sog_precision                                              */
    int32_t device;             /* HIP device ordinal                                         */
    void* stream;               /* hipStream_t, or NULL for the default stream                */
    int32_t pointers_on_device; /* 1: x, q and outputs are device pointers                    */
    int32_t check_inputs;       /* 1: check neutrality and z range on the device; costs one   */
                                /*    device-to-host synchronisation per call                  */
    int32_t timing;             /* 1: time every kernel with HIP events (sog_kernel_times)    */
    sog_params params;          /* overrides; all zero = choose everything from tol          */
    int32_t static_workspace;   /* 1: the plan allocates only its tables; its calls run in    */
                                /*    the library's static scratch, through                   */
                                /*    sog_energy_potential_force_static only                  */
    int32_t deterministic;      /* 1: bitwise reproducible results for the same inputs: every */
                                /*    counting sort orders each bin by particle index, and    */
                                /*    the mid-range gridding adds the tiles' blocks into the  */
                                /*    grid in a fixed order of tile colours (no atomics)      */
                                /*    instead of with atomics; 0: the faster atomic form,     */
                                /*    whose sums may differ in the last bits between calls   */
    int32_t eager;              /* 1: every call launches its kernels one by one; 0: the     */
                                /*    first call captures them into a HIP graph that later    */
                                /*    calls replay (sog_energy_potential_force; inputs and    */
                                /*    outputs pass through plan buffers).  timing and         */
                                /*    static_workspace plans are always eager.                */
    int32_t autotune;           /* 1: measure instead of model: the planner's cheapest few    */
                                /*    discretisations by its cost model (the cheapest of each */
                                /*    of three r_c) are each built and timed on the device on */
                                /*    uniformly random neutral charges of the plan's size and */
                                /*    box, and the fastest is kept (sog_plan_tuning reports    */
                                /*    them); plan creation then costs a few solves.  Not with */
                                /*    static_workspace.                                       */
} sog_options;

/* Fill *opt with the defaults: FP64, device 0, default stream, host pointers, checks on,
 * timing off, no overrides. */
void sog_options_default(sog_options* opt);

/* Plan for n particles (2 <= n <= 2^26) in box (Lx, Ly, Lz) at relative tolerance tol with the default
 * options.  tol is the target relative error of potentials, energy and forces. */
sog_status sog_plan(const double box[3], int64_t n, double tol, sog_plan_t* out);

/* As sog_plan with explicit options (opt may be NULL for the defaults). */
sog_status sog_plan_ex(const double box[3], int64_t n, double tol, const sog_options* opt,
                       sog_plan_t* out);

/* Energy, potentials and forces (eqs. splitting and phisplit):
 *   energy: 1 value or NULL; phi: n values or NULL; force: n x 3 row-major or NULL.
 * x: n x 3 row-major positions; q: n charges (see the conventions above). */
sog_status sog_energy_potential_force(sog_plan_t plan, const double* x, const double* q,
                                      double* energy, double* phi, double* force);

/* As sog_energy_potential_force, with the gradient of the potential at each particle,
 * grad_i = grad Phi(r_i) (n x 3 row-major, or NULL), in place of the force F_i = -q_i grad_i
 * (Sec. 2.1; the same gathers).  Phi is linear in q through a symmetric operator, so this
 * call with the cotangent of the potentials as charges gives the gradients of any loss of
 * the potentials (the differentiable binding uses it that way); such charges need not be
 * neutral when the plan's check_inputs is 0 (the sum of the charges then multiplies only
 * the k = 0 constant, which every call leaves out). */
sog_status sog_energy_potential_gradient(sog_plan_t plan, const double* x, const double* q,
                                         double* energy, double* phi, double* grad);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): sog_energy_potential_force with every per-call
 * buffer (sort keys, grids, partial results, counters, host staging) in a static device
 * array of the library instead of the plan's own memory.  The call allocates nothing:
 * no hipMalloc, hipFree or allocating library routine; the plan (made beforehand, outside
 * such code) keeps only its tables.  Any plan works; one made with
 * options.static_workspace = 1 holds no per-call buffers at all and runs only here.
 *   - Limit: the plan's per-call buffers must fit the scratch, 128 MiB (about 10^5
 *     particles at tol 1e-4); larger plans return SOG_ERR_OUT_OF_MEMORY with the sizes.
 *   - The scratch is one array per device, held from the library's load until the process
 *     ends, shared by every call on that device and keeping the last call's contents
 *     (each call clears what it needs).  Calls that overlap on one device race: order them
 *     on one stream, or synchronise between them.
 *   - A plan with timing on is refused (timing creates events during calls).
 * Arguments, pointer rules, outputs and errors as for sog_energy_potential_force. */
sog_status sog_energy_potential_force_static(sog_plan_t plan, const double* x, const double* q,
                                             double* energy, double* phi, double* force);

/* The parts of the potential and its gradient (eq. splitting), for checking each solver
 * on its own: phi_parts is 3 x n (near, mid, long; the self term is not included),
 * grad_parts is 3 x n x 3 (gradient of each part at r_i).  Same pointer rules. */
sog_status sog_potential_parts(sog_plan_t plan, const double* x, const double* q,
                               double* phi_parts, double* grad_parts);

/* Run only the planner (no device work, no allocation): the parameters sog_plan_ex would
 * use for this box, n, tol and options.  Works on a machine without a GPU. */
sog_status sog_plan_resolve(const double box[3], int64_t n, double tol, const sog_options* opt,
                            sog_params* out);

/* The discretisations an autotuned plan timed (options.autotune): up to max of them, in
 * the order built, with r_c, the range split m and the milliseconds per call on the
 * synthetic sample (calls back to back; the candidates timed in turn over several
 * rounds, each keeping its fastest); *count = 0 for a plan that was not autotuned.  The
 * plan's own
 * parameters (sog_plan_info) are those of the fastest. */
sog_status sog_plan_tuning(sog_plan_t plan, int32_t max, int32_t* count, double* rc, int32_t* m, double* ms);

/* The resolved parameters of a plan. */
sog_status sog_plan_info(sog_plan_t plan, sog_params* out);

/* Sizes of the plan: grid points of the mid-range grid, long-range modes or grid
 * points, device bytes held, near-field cells. */
typedef struct {
    int64_t mid_grid_points;   /* I_x I_y I_z*                                */
    int64_t long_points;       /* direct: modes (full plane); fft: I^long_x I^long_y */
    int64_t device_bytes;      /* workspace held by the plan                  */
    int32_t near_cells[3];
    int32_t tile[3];           /* mid-range spread/gather tile, grid points  */
    int32_t near_degree;       /* Chebyshev degree of the near-field kernel  */
    int32_t mid_zband[2];      /* stored z planes [lo, hi) that can carry window mass for z in
                                  [0, Lz]; the z transforms read and write only these      */
} sog_plan_sizes;
sog_status sog_plan_sizes_get(sog_plan_t plan, sog_plan_sizes* out);

/* Per-kernel device times of the calls made since the plan was created (or since the
 * last reset), when the plan was made with options.timing = 1.  Fills up to max
 * entries (name, total milliseconds, launches) and returns the number of kernels in
 * *count.  Names are static strings owned by the library. */
typedef struct {
    const char* name;
    double total_ms;
    int64_t launches;
} sog_kernel_time;
sog_status sog_kernel_times(sog_plan_t plan, sog_kernel_time* out, int32_t max, int32_t* count);
sog_status sog_kernel_times_reset(sog_plan_t plan);

/* Release the plan and its device workspace.  NULL is ignored. */
void sog_destroy(sog_plan_t plan);

/* Batched independent systems: nsys systems, each its own box, particle count and charge
 * neutrality (every system is a separate instance of the problem of Sec. 2.1), solved by
 * one call at the same tolerance and options.  The mid/long split of the Gaussians
 * depends on each system's height (Sec. 3; a thin enough system is all long range, per
 * the remark after the far-field split), so each system gets its own parameters (cutoff,
 * grids, windows, long-range form) from the planner.  Systems whose parameters use the
 * same kernels form a group; each kernel of a group runs once for all its systems (its
 * blocks dealt to the systems by a table, each system's arguments read from a table in
 * device memory), and the launches of all groups are captured at batch-plan time into one
 * HIP graph of a few dozen kernel nodes that each call launches once.
 *
 * Layout: the systems' particles are stored one after another, system s holding
 * particles [off_s, off_s + n[s]) with off_s = n[0] + ... + n[s-1]; x is (sum n) x 3
 * row-major, q has sum n entries, phi sum n, force (sum n) x 3, energy nsys (one per
 * system).  Pointer rules, precision, device and stream come from opt as for sog_plan_ex
 * (opt->params applies to every system; opt->timing must be 0).  The batch owns device
 * staging buffers for inputs and outputs: a call copies x and q into them, checks them
 * (opt->check_inputs: one validation kernel for all systems and one read-back; errors
 * name the first failing system), launches the graph and copies the outputs out.
 * Outputs are unspecified on error.  Errors as for sog_plan_ex, plus SOG_ERR_INVALID_ARG
 * for nsys < 1, NULL arrays, timing on, a total above 2^31 particles, or a system whose
 * plan takes the long range's FFT form (batches run the direct form only).  A batch must
 * not be used by two calls at once. */
typedef struct sog_batch_s* sog_batch_t;
sog_status sog_batch_plan(int32_t nsys, const double* boxes /* nsys x 3 */, const int64_t* n /* nsys */,
                          double tol, const sog_options* opt, sog_batch_t* out);
sog_status sog_batch_energy_potential_force(sog_batch_t batch, const double* x, const double* q,
                                            double* energy, double* phi, double* force);
/* The structure of a batch's graph: the number of groups of systems that share kernels,
 * and the number of kernel launches (graph nodes) of one call. */
sog_status sog_batch_graph_info(sog_batch_t batch, int32_t* groups, int32_t* launches);
/* The resolved parameters of system s of a batch. */
sog_status sog_batch_plan_info(sog_batch_t batch, int32_t s, sog_params* out);
/* Release the batch, its plans, graph and buffers.  NULL is ignored. */
void sog_batch_destroy(sog_batch_t batch);

const char* sog_status_string(sog_status s);
const char* sog_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SOG_H */
