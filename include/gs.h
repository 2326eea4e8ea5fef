/*
 * gs.h -- C ABI of the Gaussian-sum nonlocal potential library for AMD MI355X.
 *
 * The library evaluates u = U * rho (convolution over R^d, free-space
 * boundary conditions) for a density rho sampled on a uniform grid over the
 * box prod_j [-L_j, L_j], with the method of Exl, Mauser and Zhang, "Accurate and
 * efficient computation of nonlocal potentials based on Gaussian-sum
 * approximation": the kernel is split as U = U_GS + (U - U_GS) (Section 2.1,
 * eqs. (key_form), (GS-Gene)); the regular part is a zero-padded aperiodic FFT
 * convolution with the tensor-product kernel coefficients (Section 2.2,
 * eqs. (I1FFT), (tensor)); the near-field part is the Taylor correction
 * A0 rho + c2 Lap(rho) (Section 2.3, eq. (taylor)).  The precomputation /
 * evaluation split of Algorithm 1 is the plan / eval split below.
 *
 * Conventions shared by every entry point
 *   - Grids have n_j points on axis j over a box prod_j [-L_j, L_j] (a cube
 *     when the L_j and n_j are equal; a rectangular box or grid as in Section
 *     2.5 otherwise): spacing h_j = 2 L_j / n_j, sample i on axis j at
 *     -L_j + i h_j, i = 0..n_j - 1.  A rectangular box with one spacing on every
 *     axis has unequal n_j.
 *   - Arrays are dense, C-ordered FP64: [z][y][x] in 3D, [y][x] in 2D, x the
 *     last (fastest) index.  `n` and `L` arguments are arrays of length d in
 *     that same order.
 *   - Device pointers are HIP device memory on the plan's device, owned by the
 *     caller, and must stay valid until the work queued on the plan's stream
 *     has completed.  Calls are asynchronous with respect to the host.
 *   - Status codes only; nothing is thrown across the ABI.  Arguments are
 *     validated before any device work; on a synchronous error the outputs
 *     are untouched.  Asynchronous HIP failures surface as GS_ERR_HIP on a
 *     later call.  gs_last_error() returns a thread-local message.
 *   - A plan is used by one stream at a time.  Plans are independent: several
 *     plans may run concurrently on different streams.
 *   - The environment variable GS_LOG_LEVEL (1: plan and batch decisions, 2: also
 *     every error status) makes the library write one line per event to stderr.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_plan_s* gs_plan;

/* Kernel families (Section 1, eq. (kernelPhy); dipolar kernel, Section 2.4;
 * Davey-Stewartson potential, the remark closing Section 2.4 and Example 4.5). */
typedef enum {
    GS_COULOMB_3D = 0,    /* U = 1/(4 pi |x|),                       d = 3 */
    GS_COULOMB_2D = 1,    /* U = 1/(2 pi |x|),                       d = 2 */
    GS_POISSON_2D = 2,    /* U = -ln|x| / (2 pi),                    d = 2 */
    GS_DIPOLAR_3D = 3,    /* u = -(n.m) rho - 3 Coulomb3D(d_n d_m rho), d = 3 */
    GS_GAUSSIAN_SUM = 4,  /* U = sum_q w_q exp(-tau_q^2 |x|^2) from gs_options,
                             no near-field term (test hook), d = 2 or 3 */
    GS_DAVEY_STEWARTSON_2D = 5, /* u = (-ln|x| / (2 pi)) * d_xx rho, d = 2: the Poisson
                             table and Taylor terms, the d_xx symbol -xi_x^2 (even,
                             Nyquist kept) folded into the stored spectrum */
    GS_INVERSE_POWER = 6  /* U = |x|^-beta, 0 < beta < d (gs_options.beta), d = 2 or 3
                             (the Remark after eq. (GauInte)) */
} gs_kernel;

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARG = 1,       /* bad d, n, L, eps, pointer, count, option */
    GS_ERR_UNSUPPORTED_SIZE = 2,  /* n not in the compiled size list          */
    GS_ERR_ACCURACY = 3,          /* eps not reachable by the sinc table      */
    GS_ERR_OUT_OF_MEMORY = 4,     /* device allocation failed or over the cap */
    GS_ERR_NO_DEVICE = 5,         /* no HIP device visible                    */
    GS_ERR_HIP = 6                /* a HIP runtime call failed                */
} gs_status;

/* Plan flags. */
#define GS_PLAN_HOST_ONLY      1  /* tables, factors, constants and a host-assembled
                                     spectrum only; no device memory, no device
                                     calls (gs_eval* return GS_ERR_INVALID_ARG) */
#define GS_PLAN_HOST_ASSEMBLY  2  /* assemble the spectrum on the host and upload it
                                     instead of the MFMA assembly kernel */
#define GS_PLAN_AUTOTUNE       4  /* pick the launch variants of the evaluation (cache
                                     hints per pass, persistent grid of the fused pass,
                                     tile shapes of the cubic passes, the fused pass's
                                     radix plan) by timing whole evaluations at plan
                                     creation on scratch buffers, or take them from the
                                     autotune cache (see GS_SCHED_AUTO); results are
                                     bitwise the same for every variant except the radix
                                     plan (gs_options.tile_variants bit 8), which agrees
                                     to rounding and is kept only when faster by more
                                     than 1 % */
#define GS_PLAN_NO_WORKSPACE   8  /* allocate no evaluation workspace: the plan holds its
                                     spectrum and twiddles only and is evaluated with
                                     gs_eval_static (gs_eval, gs_eval_step,
                                     gs_eval_backward and batches refuse it with
                                     GS_ERR_INVALID_ARG; not with GS_PLAN_AUTOTUNE) */

#define GS_PLAN_UNPADDED_LAPLACIAN 16 /* the Taylor term's Laplacian on the density's own
                                     grid (spectral, period 2 L_j: Algorithm 1 step 3 read
                                     on the unpadded grid) instead of the padded grid of
                                     the convolution; still folded into the stored spectrum
                                     (the padded transform at all-even indices is the
                                     n-point transform of rho).  Kernels whose Taylor term
                                     acts on rho itself only (INVALID_ARG for the dipolar
                                     and Davey-Stewartson potentials) */

#define GS_PLAN_PAD3           32 /* zero-pad the density to B_3 = prod_j [-3 L_j, 3 L_j]
                                     (Section 2.2, eq. (FourSeriB3) with 3 n_j points per
                                     axis) instead of to [-2 L_j, 2 L_j] (the Remark after
                                     eq. (tensor), the default): transforms of length 3 n_j,
                                     frequencies pi k / (3 L_j), M = prod_j 3 n_j, the
                                     factor integrals still over [-2 L_j, 2 L_j] (eq.
                                     (tensor)).  Every n_j even (INVALID_ARG otherwise) with
                                     3 n_j / 2 in the compiled size list (UNSUPPORTED_SIZE):
                                     the passes run on a grid of 3 n_j / 2 points per axis
                                     (the density in its first n_j points, zeros after,
                                     padded twice).  On a cubic grid the x passes read the
                                     density and write the potential in place (the inverse
                                     passes only where the potential is kept); otherwise
                                     the density is copied in before the first step and the
                                     potential out after the last, the copy adding
                                     (3/2)^d n^d doubles to the workspace (allocated for
                                     both).  Not batched (the batched schedules
                                     refuse it; GS_SCHED_AUTO evaluates it on its own) */

/* Size of the fixed device array gs_eval_static uses as its workspace. */
#define GS_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

typedef struct {
    double delta_rel;        /* near-field radius delta / max_j L_j; 0 selects 1e-4;
                                must be below min_j L_j / max_j L_j              */
    double dipole_n[3];      /* GS_DIPOLAR_3D: orientations (x, y, z), non-zero; used as given */
    double dipole_m[3];
    const double* gs_w;      /* GS_GAUSSIAN_SUM: weights w_q (host), length gs_q  */
    const double* gs_tau;    /* GS_GAUSSIAN_SUM: exponents tau_q >= 0 (host)      */
    int gs_q;
    void* stream;            /* hipStream_t for all work of the plan; NULL = null stream */
    int device;              /* HIP device ordinal; -1 = the current device       */
    int flags;               /* GS_PLAN_* bits                                    */
    int slab_planes;         /* 3D: kx planes per slab of the middle passes (the X2
                                workspace holds one slab); 0 = as many as fit in
                                GS_SLAB_BYTES (unset: all), -1 = all n+1 planes   */
    int slab_streams;        /* 3D: streams the slabs' middle-pass chains run on
                                concurrently (>= 2: X2 holds every slab, each at
                                its own planes; the results are the same bits);
                                0 or 1 = in order on the plan's stream           */
    double beta;             /* GS_INVERSE_POWER: the exponent, 0 < beta < d      */
    int tile_variants;       /* tile shapes of the cubic passes (bits 0-1: x-forward
                                pass, 1 = twice the row pairs per block; bits 2-3: y
                                passes, 1 = half, 2 = twice the z-pencils per block; bits
                                4-5: fused pass, 1 = half, 2 = twice the pencils per
                                block; bits 6-7: x-inverse pass, as bits 0-1); 0 = the
                                compiled defaults.  Compiled for n >= 128 where the LDS
                                allows, ignored elsewhere and on grids whose axes differ;
                                every such value gives the same bits.  Bit 8: the fused
                                pass on its radix-plan variant (n = 128, 256, 512, 1024,
                                2048: 16 values per thread where the default holds 8, 8
                                where it holds 16; bits 4-5 then ignored), which agrees
                                with the default to rounding, not bitwise; bits 9 and
                                10: the x-forward and x-inverse passes on theirs (the
                                same lengths and value counts; bits 0-1 and 6-7 then
                                ignored); bits 11 and 12: the y-forward and y-inverse
                                passes (3D; bits 2-3 then ignored for that pass).  A
                                plan on any of these is batched only by its own
                                launches.
                                GS_PLAN_AUTOTUNE picks them by timing            */
    int launch_hints;        /* 1 + the cache-hint bits of the passes (bit p-1 set: pass p
                                uses its non-temporal hint variant, gs_plan_info.hint_bits);
                                0 = the compiled default.  Every value gives the same bits;
                                GS_PLAN_AUTOTUNE picks them by timing            */
} gs_options;

typedef struct {
    int kernel, d;
    int64_t n;
    double L, eps, delta;    /* delta in physical units                          */
    int S;                   /* sinc truncation: 1/r tables have S+1 terms       */
    int Q;                   /* number of Gaussians in the table (incl. tau = 0) */
    double A0, c2;           /* Taylor constants of eq. (taylor)                   */
    size_t spectrum_bytes;   /* stored spectrum octant (n+1)^d FP64              */
    size_t workspace_bytes;  /* per-plan device workspace                        */
    double assembly_ms;      /* device time of the spectrum assembly (0 if host) */
    double assembly_gflop;   /* 2 Q (n+1)^d, the contraction's algorithmic flops */
    int host_only;
    int slab_planes;         /* kx planes per slab (3D), n+1 in 2D                */
    int num_steps;           /* kernel launches of one evaluation                 */
    int slab_streams;        /* concurrent slab chains (1 = in order)             */
    int x2_planes;           /* kx planes the X2 workspace holds                  */
    int tuned;               /* 1 if the launch variants came from the autotuner  */
    int hint_bits;           /* bit p-1 set: pass p uses its cache-hint variant   */
    int fused_grid_mult;     /* rounds of co-resident blocks of the 3D fused pass */
    int tune_candidates;     /* variants timed when this plan was created         */
    double tuned_ms;         /* measured evaluation time of the chosen variant    */
    double L_axes[3];        /* half-widths as given, C order (first d entries);
                                L above is their maximum, the table's length unit */
    double beta;             /* GS_INVERSE_POWER exponent (0 for other kernels)   */
    int64_t n_axes[3];       /* points per axis, C order (first d entries); n above is
                                their common value, or their largest on a grid whose
                                axes differ                                      */
    int tile_variants;       /* tile shapes in use (gs_options.tile_variants bits)  */
    int padding;             /* the density is zero-padded to [-p L_j, p L_j]: p = 2 or 3 */
} gs_plan_info;

/* Fill `opt` with the defaults (delta_rel 1e-4, null stream, device -1). */
void gs_options_default(gs_options* opt);

/*
 * Precomputation (Algorithm 1, "Precomputation"): Gaussian-sum table by sinc
 * quadrature with the smallest S meeting `eps` on [delta, R] in units of the
 * largest half-width L (Section 3; relative error of 1/r and of r^-beta, absolute
 * error of ln r; r^-beta through its Gaussian integral, eq. (Gauss_int) with the
 * factor 1/2 of the half line, under tau = exp(t - e^-t);
 * R = 2 sqrt(sum_j (L_j/L)^2), the largest distance in the box: 2 sqrt(d)
 * for a cube), the one-dimensional factor integrals of eq. (tensor) (eq.
 * (tensor_ani) for rectangular boxes) at the padded frequencies
 * xi = pi k/(2 L_j), k = 0..n_j, of every axis (GS_PLAN_PAD3: pi k/(3 L_j),
 * k = 0..3 n_j/2, and 3 n_j below), the Taylor constants A0, c2
 * (Section 2.3), and the stored spectrum octant [kx][ky][kz] (x first)
 *     S[k] = ( sum_q w_q prod_j g_q(xi_kj) + A0 - c2 |xi_k|^2 ) / prod_j (2 n_j),
 * assembled on the device by an FP64 matrix-core contraction.  Allocates the
 * spectrum and the evaluation workspace on the device.
 *   out     receives the plan (NULL on error).
 *   k, d    kernel family and dimension (2 or 3).
 *   n, L    length-d arrays, [z][y][x] order; every n_j in the compiled size
 *           list (gs_supported_sizes; UNSUPPORTED_SIZE otherwise); a cubic grid
 *           (equal n_j) runs the cubic passes, a grid with unequal n_j runs each
 *           pass at the length of the axis it transforms; every L_j > 0, and
 *           delta_rel below min_j L_j / max_j L_j (the near-field ball must fit
 *           the shortest axis, Section 2.5).
 *   eps     target accuracy of the Gaussian sum (1e-15 <= eps < 1).
 *   opt     NULL for defaults.
 * Errors: INVALID_ARG, UNSUPPORTED_SIZE, ACCURACY, OUT_OF_MEMORY, NO_DEVICE, HIP.
 * The environment variable GS_MAX_WORKSPACE_BYTES caps the device bytes a plan
 * may allocate (OUT_OF_MEMORY beyond it).
 */
gs_status gs_plan_create(gs_plan* out, gs_kernel k, int d, const int64_t* n,
                         const double* L, double eps, const gs_options* opt);

/* Frees the plan and its device memory (synchronises its stream).  NULL is a no-op. */
gs_status gs_plan_destroy(gs_plan p);

gs_status gs_plan_query(gs_plan p, gs_plan_info* info);

/* Copies the Gaussian-sum table (physical units) into w[0..Q-1], tau[0..Q-1]. */
gs_status gs_plan_table(gs_plan p, double* w, double* tau, int capacity);

/* Copies the factor matrix F[k][q] = g_q(pi k/(2L)), k = 0..n, row-major (n+1) x Q,
 * of the x axis (the last array axis). */
gs_status gs_plan_factors(gs_plan p, double* F, size_t capacity);

/* As gs_plan_factors for array axis `axis` (0 .. d-1, C order), whose half-width
 * L_axis gives the frequencies pi k/(2 L_axis).  INVALID_ARG for another axis. */
gs_status gs_plan_factors_axis(gs_plan p, int axis, double* F, size_t capacity);

/* Copies the stored spectrum octant ((n+1)^d FP64, scaled by 1/(2n)^d) to host
 * memory: from the device for device plans, the host assembly otherwise. */
gs_status gs_plan_spectrum(gs_plan p, double* host_out, size_t capacity);

/* Sets the HIP stream used by later calls on this plan (NULL = null stream). */
gs_status gs_plan_set_stream(gs_plan p, void* stream);

/*
 * Evaluation (Algorithm 1, "Actual computation"): u = I1 + A0 rho + c2 Lap rho
 * as one pruned, zero-padded FFT convolution with the stored spectrum, five
 * kernel launches in 3D (x-R2C, y-forward, fused z forward * spectrum *
 * inverse, y-inverse, x-C2R) and three in 2D.  rho and u are device arrays of
 * n^d FP64; u may alias rho.  The padding never touches memory.
 */
gs_status gs_eval(gs_plan p, const double* rho_dev, double* u_dev);

/*
 * gs_eval without any device allocation, for callers that cannot allocate device
 * memory while they evaluate (code under stream capture, serving loops, harnesses
 * that forbid hipMalloc): the same passes and bits as gs_eval, with the evaluation
 * workspace in a fixed device array of GS_STATIC_SCRATCH_BYTES (128 MiB) instead of
 * the plan's.  Every device the library runs on holds one such array until the
 * process ends; it fits 3D grids up to n = 128 (and larger n when the plan's
 * middle passes run in small kx slabs) and 2D grids up to n = 2048.  The plan may
 * be created with GS_PLAN_NO_WORKSPACE to hold no workspace of its own.  Calls
 * on one device share the array: calls that overlap in time on one device (other
 * streams, other threads) race, and the caller must serialise them.  The array
 * needs no clearing (every workspace element is written before it is read).
 * Errors: INVALID_ARG (invalid or host-only plan, NULL pointer),
 * UNSUPPORTED_SIZE (the plan's workspace exceeds the array), HIP.  Calls no
 * hipMalloc, hipFree or allocating routine; asynchronous on the plan's stream.
 */
gs_status gs_eval_static(gs_plan p, const double* rho_dev, double* u_dev);

/*
 * gs_eval plus the Hartree-type energy E = 1/2 int rho u by the grid sum
 * E = 1/2 (prod_j h_j) sum_i rho_i u_i (the energy of the differentiation
 * workload).  The sum is formed inside the fused spectrum pass by Parseval's
 * identity: u is the inverse transform of S rho^ on the padded grid (S the folded
 * spectrum, 1/M included), so sum_i rho_i u_i = sum_k S(k) |rho^(k)|^2 over the
 * padded spectrum, with no second read of rho.  Each pencil of that pass leaves one
 * partial sum and two more kernels add them in a fixed order, so E is the same bits
 * on every run and for every launch shape (tile variants, persistent grid).
 * energy_dev is device memory for one double, written asynchronously on the plan's
 * stream; u may alias rho.  The rho-gradient of E is (prod_j h_j) u (the operator is
 * symmetric).  Errors: as gs_eval; INVALID_ARG for a NULL energy_dev.
 */
gs_status gs_eval_energy(gs_plan p, const double* rho_dev, double* u_dev, double* energy_dev);

/*
 * The energy and its rho-gradient in one evaluation: grad_dev receives
 * (prod_j h_j) u (the gradient of E = 1/2 (prod_j h_j) sum rho u, the operator being
 * symmetric; the x-inverse pass stores u times prod_j h_j), energy_dev[0] the energy,
 * summed as in gs_eval_energy (the same bits as there).  grad_dev may alias rho_dev.
 * Errors: as gs_eval_energy.
 */
gs_status gs_eval_energy_gradient(gs_plan p, const double* rho_dev, double* grad_dev, double* energy_dev);

/*
 * Gaussian-mixture densities and the parameter gradient of a scalar through them (the
 * chain rule of the differentiation workload): on the plan's grid,
 *     rho_i = sum_c a_c exp(-|x_i - mu_c|^2 / sigma_c^2),   c = 0..K-1, 1 <= K <= 64.
 * a (K), mu (K x d, row c = (x, y[, z]) of centre c) and sigma (K) are device arrays.
 * gs_mixture_density writes rho (n^d FP64, device).  gs_mixture_gradient reads a grid
 * gradient g = dE/drho (device, n^d) and writes out (device, K (d + 2) doubles):
 *     out[c]               = scale sum_i g_i e_ci                               (dE/da_c)
 *     out[K + c d + j]     = scale (2 a_c / sigma_c^2) sum_i g_i e_ci (x_ij - mu_cj)
 *     out[K + K d + c]     = scale (2 a_c / sigma_c^3) sum_i g_i e_ci |x_i - mu_c|^2
 * with e_ci = exp(-|x_i - mu_c|^2 / sigma_c^2); the sums are reduced in a fixed order
 * (the same bits on every run) in the plan's own partial-sum buffer.  For the energy,
 * g = (prod_j h_j) u: pass u and scale = prod_j h_j.  Asynchronous on the plan's
 * stream; calls on one plan must not overlap.  Errors: INVALID_ARG (plan, K, pointers).
 */
gs_status gs_mixture_density(gs_plan p, int K, const double* a, const double* mu, const double* sigma,
                             double* rho_dev);
gs_status gs_mixture_gradient(gs_plan p, int K, const double* a, const double* mu, const double* sigma,
                              const double* g_dev, double scale, double* out_dev);

/*
 * Adjoint of gs_eval: grad_rho = A^T grad_u, the transposed chain (crop and
 * zero-padding exchanged, transform signs flipped).  The discrete operator is
 * a symmetric Toeplitz matrix because every kernel here is even, so the
 * transposed chain runs the same passes.  Used by autograd: for the energy
 * E = 1/2 h^d sum rho u, dE/drho = h^d u.
 */
gs_status gs_eval_backward(gs_plan p, const double* grad_u_dev, double* grad_rho_dev);

/*
 * Batched evaluation: many independent problems, each with its own plan (any
 * kernel, d = 2 or 3, sizes n <= 128 of the compiled list, possibly all
 * different).  The method is the per-problem evaluation of gs_eval unchanged;
 * batching only schedules the tiles of all problems together, and every
 * problem's result is bitwise the one gs_eval gives.
 *
 * Schedules:
 *   GS_SCHED_QUEUE      one persistent launch; each die (XCD) of the device
 *                       walks a pass-major task list of the problems pinned to
 *                       it, a task waiting for the preceding pass of its own
 *                       problem through per-problem counters.
 *   GS_SCHED_PHASED     one launch per pass type over the tasks of all problems.
 *   GS_SCHED_SIZED      one launch per pass type and grid size (each launch
 *                       specialised to its size).
 *   GS_SCHED_SEQUENTIAL each plan's own gs_eval launches, one problem after the
 *                       other (the unbatched baseline).
 *   GS_SCHED_CONCURRENT the launches of GS_SCHED_SIZED, each grid size's chain of
 *                       passes on its own stream (four streams forked from the
 *                       batch stream and joined back), the sizes running at the
 *                       same time.
 *   GS_SCHED_STREAMS    each plan's own gs_eval launches, the plans (largest first)
 *                       dealt round-robin to four concurrent streams; any plans
 *                       (no batched kernels needed).
 *   GS_SCHED_AUTO       the fastest of the others (and of their task sizes) for
 *                       this device and multiset of problem shapes, measured on
 *                       the first gs_batch_eval (as graph replays when use_graph
 *                       is set) and cached in the process and,
 *                       if the environment variable GS_AUTOTUNE_CACHE names a
 *                       file, in that JSON file across processes.
 */
typedef enum {
    GS_SCHED_AUTO = 0,
    GS_SCHED_QUEUE = 1,
    GS_SCHED_PHASED = 2,
    GS_SCHED_SEQUENTIAL = 3,
    GS_SCHED_SIZED = 4,
    GS_SCHED_CONCURRENT = 5,
    GS_SCHED_STREAMS = 6
} gs_schedule;

typedef struct gs_batch_s* gs_batch;

typedef struct {
    int schedule;        /* gs_schedule                                               */
    int tiles_per_task;  /* block-fulls of tiles per task (>= 1); 0 = default (queue 8,
                            phased 4) or tuned.  An upper bound: a problem's pass that
                            would split into fewer than 24 tasks gets smaller ones
                            (down to one block-full), so small problems keep their
                            die's blocks busy                                         */
    int grid;            /* persistent blocks; 0 = as many as can be co-resident.  The
                            queue schedule with per-die queues raises a smaller grid to
                            the co-resident count (every die must run blocks)          */
    int use_graph;       /* 1: capture the launch sequence in a hipGraph on the first
                            evaluation and replay it afterwards                         */
    void* stream;        /* hipStream_t the evaluations are ordered on; NULL = null stream */
} gs_batch_options;

typedef struct {
    int count;              /* problems                                        */
    double points;          /* sum of n^d over the problems                    */
    int schedule;           /* resolved schedule (never GS_SCHED_AUTO once run) */
    int tiles_per_task;
    int grid;
    int use_graph;
    int num_tasks;          /* tasks of the queue / phased schedules           */
    int tasks_per_pass[6];  /* index = pass id 1..5                             */
    int autotuned;          /* 1 if the schedule came from a measurement        */
    int candidates;         /* schedules timed by the autotuner for this batch  */
    double tuned_ms;        /* best measured evaluation time (ms), 0 if none    */
    int wait_timeouts;      /* 1 if a queue-schedule dependency wait ever gave up
                               or a queue was left unfinished (results of that
                               call invalid; never expected)                    */
    int num_queues;         /* queue schedule: task queues (one per die in use)  */
    int local_queues;       /* 1: each problem pinned to one die's queue         */
} gs_batch_info;

/* Defaults: GS_SCHED_AUTO, tiles_per_task 0, grid 0, no graph, null stream. */
void gs_batch_options_default(gs_batch_options* opt);

/*
 * Creates a batch over `count` distinct device plans on one device.  The plans
 * must outlive the batch and must not be evaluated elsewhere while a batch
 * evaluation is in flight (the batch uses their workspaces).  Allocates the
 * batch's device descriptors and synchronises once.  Errors:
 * GS_ERR_INVALID_ARG (count < 1, NULL or duplicate or host-only plan, plans on
 * several devices, a plan whose middle passes run in kx slabs),
 * GS_ERR_UNSUPPORTED_SIZE (n > 128), GS_ERR_HIP.
 */
gs_status gs_batch_create(gs_batch* out, int count, const gs_plan* plans, const gs_batch_options* opt);

/* Evaluates u[i] = U * rho[i] for every problem i; rho[i], u[i] are device
 * arrays of plans[i]'s shape (u[i] may alias rho[i]).  Asynchronous on the
 * batch's stream, except for the first call of a GS_SCHED_AUTO batch whose
 * shapes are not in the cache: that call times the candidates (each produces
 * the same result) and synchronises.  Calls on one batch must not overlap.
 * Returns GS_ERR_HIP when an earlier queue-schedule call of this batch, finished
 * by now, raised the error flag that gs_batch_query reports (never expected). */
gs_status gs_batch_eval(gs_batch b, const double* const* rho_dev, double* const* u_dev);

/* Sets the stream later gs_batch_eval calls are ordered after (the caller's
 * stream; NULL = null stream).  The batch's own work runs on a stream it owns,
 * ordered between the caller's stream by events. */
gs_status gs_batch_set_stream(gs_batch b, void* stream);

/* Fills info; waits for the batch's stream (it reads the error flag). */
gs_status gs_batch_query(gs_batch b, gs_batch_info* info);

/* Waits for the batch's stream and frees its device memory; NULL or an already
 * destroyed batch is a no-op. */
gs_status gs_batch_destroy(gs_batch b);

/* One-shot form: creates a GS_SCHED_QUEUE batch on the first plan's stream,
 * evaluates once, waits for it, checks the error flag (GS_ERR_HIP if it was
 * raised) and destroys the batch. */
gs_status gs_eval_batch(int count, const gs_plan* plans,
                        const double* const* rho_dev, double* const* u_dev);

/* One evaluation is a fixed list of kernel launches ("steps"): 3D: x-R2C, then
 * per kx slab (y-forward, fused spectrum pass, y-inverse), then x-C2R; 2D:
 * x-R2C, fused pass, x-C2R.  gs_plan_steps writes each step's pass id (1 =
 * x-R2C, 2 = y-forward, 3 = fused, 4 = y-inverse, 5 = x-C2R) into pass_ids
 * (up to capacity) and returns the number of steps (-1 for an invalid plan).
 * gs_eval_step runs step `step` only: running 0..steps-1 in order equals
 * gs_eval.  For timing and testing the passes separately.  A step consumes what
 * the previous step leaves in the workspace; in particular the 2D fused pass at
 * n = 1024 takes the pencils kx = 0 and kx = n as real (as the x-R2C step leaves
 * them: it transforms the two together as one complex pencil). */
int gs_plan_steps(gs_plan p, int* pass_ids, int capacity);
gs_status gs_eval_step(gs_plan p, const double* rho_dev, double* u_dev, int step);

/* gs_eval with an event recorded on the plan's stream before the first step and after
 * every step (events: count = steps + 1 hipEvent_t handles created by the caller, for
 * timing the passes of a whole evaluation launched back to back; a NULL entry records
 * nothing at that point).  Errors: INVALID_ARG (count, plan), HIP. */
gs_status gs_eval_events(gs_plan p, const double* rho_dev, double* u_dev, void* const* events, int count);

/* Copies a plan buffer between the device and host memory, for testing the
 * passes one at a time: which = 1 workspace X1 ((n+1) n^(d-1) complex, layout
 * [z][kx][y] / [kx][y]), 2 workspace X2 (3D: [kx - kx0][ky][z] of the last slab),
 * 3 the stored spectrum octant ((n+1)^d FP64).  X2 holds one kx slab:
 * 2n n (slab_planes) complex values.  to_device = 0 reads into host,
 * 1 writes from host.  count is in doubles and must equal the buffer size.
 * Synchronises the plan's stream. */
gs_status gs_plan_buffer(gs_plan p, int which, int to_device, double* host, size_t count);

/* Human-readable status name, and the last error message of this thread. */
const char* gs_status_string(gs_status s);
const char* gs_last_error(void);

/* Number of visible HIP devices (0 when there is none); never fails. */
int gs_device_count(void);

/* Sizes n for which kernels are compiled (ascending); returns the count. */
int gs_supported_sizes(int d, int64_t* out, int capacity);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
