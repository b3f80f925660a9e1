/*
 * fx.h -- C ABI of the free-flight expansion library (libfx.so, gfx950).
 *
 * The library evaluates the prescription (FF) of section 5.2 of Deuar,
 * "A tractable prescription for large-scale free flight expansion of
 * wavefunctions" (arXiv:1602.03395): a compact field Psi on an M-point
 * lattice (x_j = a_j + n_j dx_j, eq. (xj)) flies freely for a time t into
 * vacuum (eq. (vacuum)); the result is returned on the magnified lattice
 * xbar_j = abar_j + nbar_j lam_j dx_j (eq. (wbx)) with the same number of
 * points, as the sum over the lam = prod_j lam_j terms q of
 *
 *     Psibar[nbar] = sum_q f^(q)[nbar] B^(q)[n''(nbar)]            (FFpsi)
 *     f^(q)        = (1/lam) exp(i alpha_q.(xbar - a - alpha_q hbar t / 2m))   (presf)
 *     B^(q)        = FFT^-1[ A~^(q) exp(i k.(abar - a - (k + 2 alpha_q) hbar t / 2m)) ]   (presB)
 *     A~^(q)       = FFT[ Psi exp(-i alpha_q.(x - a)) ]            (presA)
 *     n''_j        = (nbar_j lam_j) mod M_j                        (FFaux)
 *
 * with alpha_j = q_j dk_j / lam_j, dk_j = 2 pi / L_j, the wavevectors of
 * eq. (kj) (Nyquist negative) and the odd-M umklapp rule stated after (FF).
 * The density rho = |Psibar|^2 is what is measured (section 2).
 *
 * Conventions shared by every call:
 *  - Arrays are C-ordered with the last axis contiguous; the output has the
 *    input's shape. Complex values are interleaved (re, im): complex128 for
 *    FX_PREC_C128 and complex64 for FX_PREC_C64_PHASE64. Densities are
 *    float64 resp. float32.
 *  - Every data pointer is a DEVICE pointer owned by the caller. The library
 *    never frees, retains or aliases caller memory beyond the call. Inputs
 *    and outputs must not overlap: every call checks the byte ranges on the
 *    host and returns FX_EINVAL when an output intersects an input or
 *    another output.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream). Work is
 *    enqueued on it and the call returns without synchronising; outputs are
 *    valid once the stream reaches that point. A plan must not be used on
 *    two streams at the same time; distinct plans are independent.
 *  - Arguments are validated on the host before anything is launched. On
 *    error a negative fx_status is returned, nothing is launched, outputs
 *    are unspecified, and fx_last_error() returns a message for the calling
 *    thread. No exception or abort crosses this interface.
 *  - Units: only hbar t / m enters; the caller passes m/hbar and t.
 */
#ifndef FX_H
#define FX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FX_MAX_DIM 3

typedef enum fx_status {
    FX_OK = 0,
    FX_EINVAL = -1,        /* invalid argument (shape, lambda, dx, t, pointers, ...) */
    FX_ENOMEM = -2,        /* device or host allocation failed, or workspace too small */
    FX_EDEVICE = -3,       /* a HIP runtime call or kernel launch failed */
    FX_EUNSUPPORTED = -4,  /* valid problem outside what this library supports (e.g. too long an axis) */
    FX_STATUS_RANGE_ = 0x7fffffff  /* not a status: makes every 32-bit value a valid fx_status, so that
                                      fx_status_string may be handed any int */
} fx_status;

typedef enum fx_precision {
    FX_PREC_C128 = 0,         /* plain method: complex128 data, FP64 arithmetic throughout */
    FX_PREC_C64_PHASE64 = 1   /* complex64 data, FP32 transforms and accumulation; every phase
                                 table (premultiply, chirp, twiddle f, FFT roots) is built in
                                 FP64 with exact reduction modulo 2 pi and rounded once to FP32 */
} fx_precision;

typedef enum fx_schedule {
    FX_SCHED_PAPER = 0,          /* the sum over all prod_j lam_j terms of (FF) */
    FX_SCHED_AXIS_FACTORISED = 1 /* the same operator applied as d successive 1-D expansions
                                    (sum_j lam_j terms); exact because the free propagator and
                                    every factor of (FF) factorise over axes (eq. (free0)) */
} fx_schedule;

/*
 * Problem statement (section 5.2). Only the first `ndim` entries of each
 * array are read.
 *   ndim        1..3
 *   shape[j]    M_j >= 1
 *   dx[j]       lattice spacing dx_j > 0, finite
 *   a[j]        input offset a_j; NaN selects the default -M_j dx_j / 2
 *   abar[j]     output offset abar_j; NaN selects the default
 *               a_j + (1 - lam_j) M_j dx_j / 2 (magnified box with the same centre)
 *   lambda[j]   integer magnification lam_j >= 1 (section 5.1 restricts to integers)
 *   m_over_hbar m / hbar > 0, finite
 *   t_flight    flight time, finite (negative values run the flight backwards)
 *   precision   an fx_precision
 *   schedule    an fx_schedule
 */
typedef struct fx_problem {
    int32_t ndim;
    int64_t shape[FX_MAX_DIM];
    double dx[FX_MAX_DIM];
    double a[FX_MAX_DIM];
    double abar[FX_MAX_DIM];
    int32_t lambda[FX_MAX_DIM];
    double m_over_hbar;
    double t_flight;
    int32_t precision;
    int32_t schedule;
} fx_problem;

typedef struct fx_plan fx_plan;
typedef struct fx_batch fx_batch;

/* Fills *p with a 1-D, 1-point, lam = 1, dx = 1, t = 0, FP64, paper-schedule
 * problem with default offsets. Host only; never fails for a non-NULL p. */
fx_status fx_problem_init(fx_problem* p);

/*
 * Builds a plan for one problem (host work + one upload): validates it,
 * computes the per-axis phase tables of (presA), (presB), (presf) and the FFT
 * roots in FP64 with exact reduction modulo 2 pi, rounds them to the data
 * precision, uploads them to the current HIP device and chooses the kernel
 * tiling. Allocates no workspace yet. *out is set only on FX_OK.
 * Errors: FX_EINVAL (bad problem or NULL pointers), FX_EUNSUPPORTED (an axis
 * longer than the library's in-LDS transform allows), FX_ENOMEM, FX_EDEVICE.
 */
fx_status fx_plan_create(const fx_problem* prob, fx_plan** out);

/*
 * Other spectra (section 7.4, generalisations): as fx_plan_create, but the free
 * evolution factor exp(-i hbar t k^2 / 2m) of eq. (free0) is replaced on every
 * axis j with phase[j] != NULL by exp(-i phase[j][i]), for a dispersion that is
 * a sum over axes, omega_k = sum_j omega_j(k_j). Only the chirp (presB) and the
 * final twiddle (presf) change; the vacuum assumption (eq. (vacuum)) still holds.
 *
 * phase[j] (host, read during the call only, not retained) holds lambda[j] *
 * shape[j] doubles: phase[j][i] = t * omega_j(kappa) in radians at the fine wave
 * number kappa = 2 pi l / (lambda[j] shape[j] dx[j]), l = i - floor(lambda[j]
 * shape[j] / 2) (ascending, the Nyquist value, for an even count, first).
 * phase has ndim entries; an entry NULL keeps the free-particle phase of
 * m_over_hbar and t_flight on that axis. The phases are reduced modulo 2 pi in
 * FP64, so their absolute accuracy is that of the caller's doubles.
 * Errors: as fx_plan_create; FX_EINVAL also for phase == NULL or a non-finite
 * table value.
 */
fx_status fx_plan_create_spectrum(const fx_problem* prob, const double* const* phase, fx_plan** out);

/* Releases the plan, its tables and any workspace it allocated itself. NULL is a no-op. */
fx_status fx_plan_destroy(fx_plan* plan);

/* Number of terms q of (FFpsi) the plan sums: prod_j lam_j. */
fx_status fx_plan_num_terms(const fx_plan* plan, int64_t* q_total);

/* Device bytes of scratch memory fx_expand / fx_expand_range / fx_expand_adjoint need. */
fx_status fx_plan_workspace_size(const fx_plan* plan, size_t* bytes);

/*
 * Hands the plan a caller-owned device buffer of at least
 * fx_plan_workspace_size() bytes (256-byte aligned). Without it the plan
 * allocates its own on first use. bytes == 0 with dev_ptr == NULL reverts to
 * plan-owned workspace. Error: FX_ENOMEM if bytes is too small, FX_EINVAL on
 * a misaligned pointer.
 */
fx_status fx_plan_set_workspace(fx_plan* plan, void* dev_ptr, size_t bytes);

/*
 * The whole expansion (FF) followed by the density: psi_out = Psibar,
 * rho_out = |Psibar|^2. psi0 is the input field (M complex values). Either
 * output may be NULL, not both. When psi_out is NULL the field is built in
 * workspace memory.
 */
fx_status fx_expand(fx_plan* plan, const void* psi0, void* psi_out, void* rho_out, void* stream);

/*
 * Partial sum of (FFpsi) over the terms q_begin <= q < q_end, where the term
 * index enumerates the q-vectors in C order of (q_{d-1}, ..., q_1, q_0), i.e.
 * the magnification index of the contiguous axis varies slowest. With
 * accumulate != 0 the partial sum is added to psi_acc, otherwise it replaces
 * it. Sums over disjoint ranges add up to fx_expand's field; the sequential
 * accumulation over q of section 7.1 is the use case (checkpointing long
 * runs, splitting the terms over devices). 0 <= q_begin <= q_end <= terms.
 */
fx_status fx_expand_range(fx_plan* plan, const void* psi0, void* psi_acc, int64_t q_begin,
                          int64_t q_end, int accumulate, void* stream);

/* rho = |psi|^2 elementwise over the plan's M points (FP64 or FP32 like the plan). */
fx_status fx_density(fx_plan* plan, const void* psi, void* rho, void* stream);

/*
 * Density image integrated along one axis of the magnified grid (section 6:
 * rho(x, y) = integral dz |Psi|^2): image = sum over that axis of rho times the
 * output spacing lam_axis dx_axis. image has the shape with `axis` removed.
 * 0 <= axis < ndim.
 */
fx_status fx_column_density(fx_plan* plan, const void* rho, int axis, void* image, void* stream);

/*
 * Hermitian adjoint of the expansion: grad_psi0 = U^H grad_psi_out, with U
 * the linear map psi0 -> Psibar of (FF). This is the inverse propagation of a
 * residual on the magnified grid back to the initial lattice, used for the
 * gradient of image-fitting losses (a derived operation: (FF) is linear in
 * Psi, so its adjoint reverses every step with conjugated factors).
 */
fx_status fx_expand_adjoint(fx_plan* plan, const void* grad_psi_out, void* grad_psi0, void* stream);

/*
 * Gradient of a real loss of the density: grad_psi0 = U^H (2 grad_rho * psibar), the
 * derivative dL/dRe psi0 + i dL/dIm psi0 for L a function of rho = |U psi0|^2 (a derived
 * operation, as fx_expand_adjoint). psibar (complex) is the expansion fx_expand returned,
 * grad_rho (real) dL/drho, both of the plan's shape; grad_psi0 receives the gradient.
 * Device pointers, asynchronous on `stream`. Errors: FX_EINVAL (NULL arguments), FX_ENOMEM,
 * FX_EDEVICE.
 */
fx_status fx_density_adjoint(fx_plan* plan, const void* psibar, const void* grad_rho, void* grad_psi0,
                             void* stream);

/* Bytes of the fixed scratch array fx_expand_noalloc works in, one per device. */
#define FX_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same result as fx_expand (same arguments, validation,
 * overlap checks and outputs), but the intermediates live in a scratch array of
 * FX_NOALLOC_SCRATCH_BYTES that is part of the library's device image (each device the library
 * runs on holds its own copy until the process ends) instead of a workspace: the call performs
 * no hipMalloc, hipFree or other allocation, and ignores any workspace set on the plan. The
 * outermost magnification index is blocked as much as needed to fit the array; a problem whose
 * intermediates exceed it even with blocks of one index returns FX_ENOMEM, with the size in
 * fx_last_error(), before anything is launched. Per-pass timing is not recorded in this call.
 * The first call on a device resolves the array's address there (a runtime symbol lookup, which
 * may load the library's device code on that device): make one call, or any other call of the
 * library, on each device before entering a region that must not allocate. All calls on one
 * device share its array, so calls that overlap in time on one device (several streams or
 * threads) race on it and give undefined results; sequential calls need no clearing between
 * them. Errors: as fx_expand, plus FX_ENOMEM as above.
 */
fx_status fx_expand_noalloc(fx_plan* plan, const void* psi0, void* psi_out, void* rho_out, void* stream);

/*
 * Stacks of fields (ensembles of realizations, section 1; batches of fields fitted to images):
 * `count` fields of the plan's shape stored back to back ([count][shape], C order), each
 * expanded independently, so fx_expand_many(p, count, psi0, psi_out, rho_out, s) gives for every
 * i < count the result fx_expand would give for field i, and fx_density_adjoint_many the gradient
 * fx_density_adjoint would give for field i (psibar, grad_rho, grad_psi0 all stacked alike).
 * The fields run as the leading slice dimension of every pass, in chunks of as many fields as
 * the plan's workspace budget (or the caller's workspace, fx_plan_set_workspace) holds.
 * count >= 1; pointers and outputs as for the single-field calls (psi_out or rho_out may be NULL,
 * not both). Errors: FX_EINVAL (count < 1, NULL arguments, overlapping inputs and outputs),
 * FX_EUNSUPPORTED (a single field's pass tensors reach 2^31 elements), FX_ENOMEM, FX_EDEVICE.
 */
fx_status fx_expand_many(fx_plan* plan, int64_t count, const void* psi0, void* psi_out, void* rho_out,
                         void* stream);
fx_status fx_density_adjoint_many(fx_plan* plan, int64_t count, const void* psibar, const void* grad_rho,
                                  void* grad_psi0, void* stream);

/*
 * Positive-P pairs (section 7.4, generalisations): the two independent fields
 * psi and psi^+ that stand for the annihilation and creation operators are
 * expanded together, as two slices of one run of the plan's passes. psi follows
 * the free evolution of the plan (Psibar = U psi), psi^+ the complex-conjugate
 * one (Psibar^+ = conj(U conj(psi^+)), i.e. the elementwise conjugate kernel),
 * and n = Psibar^+ * Psibar is the density estimator on the magnified grid
 * (complex; its real part estimates the mean density).
 *
 * psi, psi_plus: device, the plan's shape and complex type, read only.
 * psi_out, psi_plus_out, n_out: device, same shape and type; any may be NULL
 * but not all three. Needs fx_plan_pair_workspace_size() bytes of workspace
 * (allocated by the plan on first use unless the caller set a workspace, which
 * must then be at least that large: FX_ENOMEM otherwise). Works with either
 * schedule and with plans from fx_plan_create_spectrum (psi^+ then takes the
 * conjugate of that kernel too). Asynchronous on `stream`.
 * Errors: FX_EINVAL (NULL plan or input, all outputs NULL), FX_ENOMEM, FX_EDEVICE.
 */
fx_status fx_expand_pair(fx_plan* plan, const void* psi, const void* psi_plus, void* psi_out,
                         void* psi_plus_out, void* n_out, void* stream);

/* Device bytes of workspace fx_expand_pair needs (two slices plus input staging). */
fx_status fx_plan_pair_workspace_size(const fx_plan* plan, size_t* bytes);

/*
 * Far-field estimate (section 2.3, eq. (farfieldk)) on the plan's magnified output
 * lattice, the comparator the finite-time expansion replaces:
 *   amp[nbar] = (m / hbar t)^(d/2) Psi~(m xbar(nbar) / hbar t),   rho_ff = |amp|^2,
 * with Psi~ the norm-preserving transform of eq. (FT) summed over the input lattice as
 * in eq. (Psiwtm) but evaluated at the off-grid wave vectors m xbar / (hbar t). The
 * estimate carries no further phase information. Each axis is a dense complex matrix
 * (built on the host in FP64 on first use, kept by the plan) applied as a batched GEMM.
 * psi0: device input of the plan's shape and type; amp_out (complex) and rho_out (real)
 * are device outputs of the same shape, either may be NULL but not both.
 * Errors: FX_EINVAL (NULL plan or input, both outputs NULL, t_flight == 0),
 * FX_EUNSUPPORTED (a plan built with a caller spectrum), FX_ENOMEM, FX_EDEVICE.
 */
fx_status fx_far_field(fx_plan* plan, const void* psi0, void* amp_out, void* rho_out, void* stream);

/*
 * Brute-force comparator (the padded-lattice propagation of section 3 that the method
 * avoids, eq. (Psin) on the vacuum-padded lattice): per axis the field is zero-padded to
 * N_j = lam_j M_j points (eq. (vacuum)), transformed, multiplied by
 * exp(i k (abar - a) - i hbar t k^2 / 2m) for the N_j wave numbers of the padded lattice,
 * transformed back and sampled at every lam_j-th point. By the separability of the free
 * propagator this equals the full d-dimensional padded-lattice propagation; the result is
 * the same Psibar as fx_expand up to rounding. Padded lines longer than one workgroup's LDS
 * take two transform passes each way through a padded buffer of prod(shape) * lam_j
 * elements. Tables and buffers are built on first use and kept by the plan.
 * psi0: device input; psi_out (complex) and rho_out (real): device outputs of the same
 * shape, either may be NULL but not both.
 * Errors: FX_EINVAL (NULL plan or input, both outputs NULL), FX_EUNSUPPORTED (a plan
 * built with a caller spectrum, or a padded length with no factorisation into
 * workgroup-sized transforms), FX_ENOMEM, FX_EDEVICE.
 */
fx_status fx_brute_force(fx_plan* plan, const void* psi0, void* psi_out, void* rho_out, void* stream);

/*
 * Ragged batch of problems (ensembles of realizations, section 1; the terms q of each are
 * independent, section 7.1): problems equal up to their input field form a shape class with
 * one plan. A class is cut into work items of G realizations and one block of the outermost
 * magnification index (the q-block): the G fields run as the leading slice dimension of every
 * pass and the q-blocks accumulate into the item's output. Each class runs on a stream of its
 * own, forked from and joined back into the caller's stream, largest class first, so the
 * kernels of different classes overlap on the device. fx_batch_create autotunes each class
 * (G and the q-block, register or LDS transform family, fused or split accumulate, tile size,
 * persistent grids) and the class concurrency by timing eager runs, then launches every kernel
 * once; the first fx_batch_run on a stream captures the whole fork-join sequence into a HIP
 * graph, replayed with a single graph launch per run. All problems must have the same
 * precision. Errors: FX_EINVAL (NULL, n < 1, an invalid problem, mixed precisions),
 * FX_EUNSUPPORTED, FX_ENOMEM, FX_EDEVICE.
 */
fx_status fx_batch_create(const fx_problem* probs, int32_t n, fx_batch** out);
fx_status fx_batch_destroy(fx_batch* batch);

/*
 * Runs the batch: for each i < n, psi_out[i] = Psibar_i and rho_out[i] =
 * |Psibar_i|^2 (either array, or any entry of psi_out, may be NULL; rho_out
 * entries may be NULL only when psi_out[i] is not). The pointer arrays are
 * HOST arrays of DEVICE pointers; inputs may be shared between realizations,
 * outputs must be disjoint from each other and from every input (checked on
 * the host). The first run on a stream, or a run with different pointers,
 * re-captures the graph. While per-pass timing is enabled on a class plan
 * (fx_plan_set_timing on the plan from fx_batch_class), runs are issued
 * eagerly instead, so that the plan's events time every launch.
 */
fx_status fx_batch_run(fx_batch* batch, const void* const* psi0, void* const* psi_out,
                       void* const* rho_out, void* stream);

/*
 * Introspection of a created batch (profiling, tests). Classes are numbered in issue order
 * (largest first). fx_batch_class returns the class plan (owned by the batch: never destroy
 * it; it may be used with fx_plan_describe, fx_plan_set_timing and fx_plan_pass_times), the
 * number of realizations, the realizations per work item and the lane the class runs on; any
 * output pointer may be NULL. fx_batch_class_members writes the first min(max, members) batch
 * indices of the class's realizations (host array). Errors: FX_EINVAL (NULL batch, index out
 * of range).
 */
fx_status fx_batch_num_classes(const fx_batch* batch, int32_t* n);
fx_status fx_batch_class(fx_batch* batch, int32_t i, fx_plan** plan, int32_t* members, int64_t* group,
                         int32_t* lane);
fx_status fx_batch_class_members(const fx_batch* batch, int32_t i, int32_t* members, int32_t max);

/*
 * Overrides the number of lane streams the classes of a batch run on (profiling: lanes = 1 runs
 * every class on the caller's stream, one kernel at a time, so that per-pass timing measures each
 * kernel alone on the device; 0 restores the tuned value). Values above the number of classes are
 * clamped. Drops the captured graph (the next fx_batch_run captures again). Errors: FX_EINVAL
 * (NULL batch, negative lanes).
 */
fx_status fx_batch_set_lanes(fx_batch* batch, int32_t lanes);

/*
 * Per-pass timing (profiling aid). With enable != 0 every pass launch of this
 * plan is bracketed by two HIP events recorded on the stream the pass is
 * launched on. fx_plan_pass_times waits for the recorded events and returns,
 * for each pass of the schedule in order (at most max entries; *n_passes gets
 * the count), the number of timed launches and their summed duration in
 * milliseconds, then clears the counters. Entries 0.. are the passes of the
 * forward schedule ("passes" of fx_plan_describe); entries FX_ADJOINT_SLOT0..
 * are those of the adjoint schedule ("adjoint_passes"); entries that were not
 * run read 0 launches. Arrays are host memory.
 */
#define FX_ADJOINT_SLOT0 32
fx_status fx_plan_set_timing(fx_plan* plan, int enable);
fx_status fx_plan_pass_times(fx_plan* plan, int32_t* n_passes, int64_t* launches, double* ms, int32_t max);

/* Writes a one-line JSON description of the plan's schedule and tiling into buf. */
fx_status fx_plan_describe(const fx_plan* plan, char* buf, size_t len);

const char* fx_status_string(fx_status s);
const char* fx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FX_H */
