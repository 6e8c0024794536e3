/*
 * icr.h - C ABI of an MI355X (gfx950) implementation of Iterative Charted
 * Refinement (ICR), the Gaussian-process prior of NIFTy.re (section "Gaussian
 * Processes"; the method itself is defined in Edenhofer et al. 2022).
 *
 * A GP sample is s = L xi with xi ~ N(0, 1) (section "Standardization"). L is
 * applied level by level:
 *   level 0      s_0 = chol(K_00) xi_0 over the n_0^d coarsest pixels;
 *   level l->l+1 every interior coarse pixel c (1 <= c_a <= n_a - 2) spawns 2^d
 *                fine pixels  s_{l+1}[2(c-1)+b] = sum_w R_l[b,w] s_l[c+w]
 *                                              + sum_b' sqrtD_l[b,b'] xi_{l+1}[2(c-1)+b'],
 *   with R_l = K_fc K_cc^-1 and sqrtD_l the lower Cholesky factor of
 *   D_l = K_ff - K_fc K_cc^-1 K_cf (GP conditioning on the 3^d window).
 * Level sizes are n_{l+1} = 2 (n_l - 2) per axis. Windows w in {-1,0,1}^d and
 * children b in {0,1}^d are ordered lexicographically, last axis fastest.
 *
 * Conventions for every call below:
 *  - All calls return icr_status and never throw. On an argument error nothing
 *    is launched and no buffer is written; icr_last_error() describes it.
 *  - Buffers are caller-owned DEVICE pointers (hipMalloc / torch), C order, batch
 *    outermost. Their element type follows the plan's precision: double for
 *    ICR_F64, float for ICR_F32, bfloat16 (stored as uint16) for ICR_BF16_F32ACC.
 *    Pointers must be aligned to their element size; 16-byte alignment of every
 *    buffer enables the vectorised kernels.
 *  - xi-shaped buffers hold every level, level 0 first, each level a C-order grid
 *    of its shape, at the offsets reported by icr_plan_get_info (n_xi elements per
 *    sample). Output-shaped buffers hold the final level only (n_out per sample).
 *  - The hot calls (forward, adjoint, metric) are asynchronous on hip_stream
 *    (NULL = the default stream) and allocate nothing. A plan is read-only after
 *    it is built, so calls on different streams with different workspaces may
 *    run concurrently.
 *  - NaN/Inf in the inputs propagate; they are not checked.
 */
#ifndef ICR_H
#define ICR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ICR_MAX_DEPTH 15

typedef enum icr_status {
  ICR_OK = 0,
  ICR_ERR_INVALID_ARG = 1,   /* bad config, size, pointer or alignment */
  ICR_ERR_NOT_PD = 2,        /* a factorisation failed (K_cc always; D, K_00 with ICR_FLAG_NO_CLAMP) */
  ICR_ERR_HIP = 3,           /* a HIP runtime call or kernel launch failed */
  ICR_ERR_OUT_OF_MEMORY = 4, /* the plan's device matrices could not be allocated */
  ICR_ERR_UNSUPPORTED = 5    /* a valid but unimplemented combination */
} icr_status;

typedef enum icr_precision {
  ICR_F64 = 0,          /* storage and arithmetic in FP64 */
  ICR_F32 = 1,          /* storage and arithmetic in FP32 */
  ICR_BF16_F32ACC = 2   /* xi, fields and cotangents stored as bfloat16 (round to
                           nearest even), arithmetic and matrices in FP32 */
} icr_precision;

typedef enum icr_kernel {
  ICR_MATERN12 = 0,  /* sigma^2 exp(-r/l) */
  ICR_MATERN32 = 1,  /* sigma^2 (1 + sqrt3 r/l) exp(-sqrt3 r/l) */
  ICR_MATERN52 = 2,  /* sigma^2 (1 + sqrt5 r/l + 5 r^2/(3 l^2)) exp(-sqrt5 r/l) */
  ICR_SQEXP = 3      /* sigma^2 exp(-r^2 / (2 l^2)) */
} icr_kernel;

typedef enum icr_chart {
  ICR_CHART_REGULAR = 0,      /* pixels on a regular grid: one R, sqrtD per level */
  ICR_CHART_LOGRADIAL_2D = 1, /* index point (u, v) sits at (r cos t, r sin t) with
                                 r = p0 exp(p1 u), t = p2 v (chart_params p0..p2), ndim 2.
                                 Distances depend on u1, u2 and v1 - v2 only, so the plan
                                 keeps one R, sqrtD per interior coarse index along the
                                 first axis (radial shell), built at pixel (u, 1) */
  ICR_CHART_LOGRADIAL_CYL_3D = 2
                              /* index point (u, v, w) sits at (r cos t, r sin t, p3 w)
                                 with r = p0 exp(p1 u), t = p2 v (chart_params p0..p3),
                                 ndim 3. Distances depend on u1, u2, v1 - v2 and
                                 w1 - w2 only, so R and sqrtD are the same for every
                                 coarse pixel of one radial index u: the plan keeps one
                                 set per interior coarse index along the first axis
                                 (radial shell), built at that shell's pixel (u, 1, 1) */
} icr_chart;

/* Build flags */
#define ICR_FLAG_NO_CLAMP 1  /* fail with ICR_ERR_NOT_PD instead of clamping a pivot */
#define ICR_FLAG_HYPERGRAD 2 /* also build the length-scale derivatives of L_00, R and sqrtD
                                (FP64, on the device) for icr_hyper_grad; the build returns
                                ICR_ERR_NOT_PD if any pivot had to be clamped (the derivative
                                of a clamped factor is undefined) */

/*
 * Prior description. Index-space pixel i of level l sits at o_l + i delta_l per
 * axis with delta_l = distances0 / 2^l, o_0 = 0 and o_{l+1} = o_l + 3/4 delta_l
 * (children at +-delta_l/4 around their coarse pixel). Under a chart the kernel
 * sees the charted (physical) positions.
 */
typedef struct icr_config {
  int32_t ndim;        /* 1, 2 or 3 */
  int32_t shape0[3];   /* level-0 pixels per axis (first ndim used), each >= 3 if depth > 0 */
  int32_t depth;       /* number of refinement levels, 0..ICR_MAX_DEPTH */
  int32_t kernel;      /* icr_kernel */
  int32_t chart;       /* icr_chart */
  int32_t precision;   /* icr_precision */
  int32_t flags;       /* ICR_FLAG_* */
  int32_t reserved;    /* must be 0 */
  double distances0[3];/* level-0 pixel spacing per axis, > 0 */
  double scale;        /* sigma > 0: k(0) = sigma^2 */
  double length;       /* length scale l > 0 */
  double chart_params[4];
} icr_config;

typedef struct icr_plan icr_plan;  /* opaque; owns its device matrices */

typedef struct icr_plan_info {
  int32_t ndim;
  int32_t depth;
  int32_t precision;
  int32_t chart;
  int32_t elem_bytes;                         /* bytes per stored element */
  int32_t clamped_pivots[ICR_MAX_DEPTH + 1];  /* [0]: K_00, [l+1]: level l -> l+1 */
  int32_t level_shapes[ICR_MAX_DEPTH + 1][3]; /* unused axes are 1 */
  int64_t level_offsets[ICR_MAX_DEPTH + 2];   /* element offset of each level in xi; [depth+1] = n_xi */
  int64_t n_xi;                /* elements of xi per sample: sum_l prod(level shape) */
  int64_t n_out;               /* elements of the final level per sample */
  int64_t workspace_elems;     /* workspace per sample for forward and adjoint: n_xi - n_out */
  int64_t metric_workspace_elems; /* workspace per sample for icr_metric_apply: n_xi */
  int64_t device_bytes;        /* device memory held by the plan */
  int64_t level_sets[ICR_MAX_DEPTH]; /* matrix sets of refinement l -> l+1: 1 on a regular
                                        grid, n_l,0 - 2 (radial shells) under either chart */
  int64_t hypergrad_workspace_elems; /* doubles of workspace per sample for icr_hyper_grad
                                        (0 unless built with ICR_FLAG_HYPERGRAD) */
} icr_plan_info;

/*
 * Build the level-0 Cholesky factor and every level's R and sqrtD in FP64 on the
 * current HIP device, following the conditioning formulas above, and keep them
 * (FP64 plus a copy in the arithmetic type) in a new plan.
 *   cfg        host pointer, read only during the call.
 *   hip_stream stream for the build kernels (NULL = default stream).
 *   out_plan   receives the plan; *out_plan is set to NULL on failure.
 * The only synchronising call: it waits for the build to read back the status.
 * A pivot <= 3^d eps64 sigma^2 in K_00 or D is clamped (its column set to zero and
 * counted in icr_plan_info.clamped_pivots) unless ICR_FLAG_NO_CLAMP is set, in
 * which case ICR_ERR_NOT_PD is returned. A non-positive-definite K_cc always
 * returns ICR_ERR_NOT_PD.
 */
icr_status icr_build_matrices(const icr_config* cfg, void* hip_stream, icr_plan** out_plan);

/* Sizes, level shapes/offsets and clamp counts of a plan (host struct, caller-owned). */
icr_status icr_plan_get_info(const icr_plan* plan, icr_plan_info* info);

/*
 * Copy the FP64 build results to host memory (caller-owned, synchronous).
 *   level0:  l00 receives the lower Cholesky factor of K_00, N0 x N0 row-major
 *            with N0 = prod(shape0).
 *   level l: r receives R_l (2^d x 3^d row-major) and sqrtd sqrtD_l (2^d x 2^d);
 *            level_sets[l] pairs (icr_plan_info), set index outermost: under either
 *            chart one per radial shell u = 1 .. n_l,0 - 2. Either pointer may be NULL.
 */
icr_status icr_plan_copy_level0(const icr_plan* plan, double* l00);
icr_status icr_plan_copy_refinement(const icr_plan* plan, int32_t level, double* r, double* sqrtd);

/*
 * Replace a plan's matrices with caller-supplied FP64 values (host pointers, same
 * layouts as the copy calls above) and refresh the arithmetic-type copies the
 * kernels read. For matrices built elsewhere (another builder, precomputed or
 * learned values). A build-phase call: synchronous, and it must not run while a
 * hot call that uses the plan is in flight. Clamp counts are left as built.
 */
icr_status icr_plan_set_level0(icr_plan* plan, const double* l00, void* hip_stream);
icr_status icr_plan_set_refinement(icr_plan* plan, int32_t level, const double* r,
                                   const double* sqrtd, void* hip_stream);

/*
 * Forward: s = L xi for `batch` samples.
 *   xi        [batch][n_xi]  input excitations, every level.
 *   s         [batch][n_out] output, the final level.
 *   workspace [batch][workspace_elems] device scratch; after the call level l < depth
 *             of the sample sits at level_offsets[l] (the intermediate fields s_l).
 * batch == 0 is a no-op. xi, s and workspace must not overlap.
 */
icr_status icr_forward(const icr_plan* plan, int64_t batch, const void* xi, void* s,
                       void* workspace, void* hip_stream);

/*
 * Adjoint: xi_bar = L^T s_bar, the exact transpose of icr_forward. The coarse
 * cotangent of each level is gathered from the up to 3^d fine blocks that read
 * each coarse pixel, in a fixed order (no atomics: results are bitwise
 * reproducible).
 *   s_bar     [batch][n_out] input cotangent of the final level.
 *   xi_bar    [batch][n_xi]  output.
 *   workspace [batch][workspace_elems]; after the call level l < depth holds the
 *             coarse cotangent s_bar_l at level_offsets[l].
 */
icr_status icr_adjoint(const icr_plan* plan, int64_t batch, const void* s_bar, void* xi_bar,
                       void* workspace, void* hip_stream);

/*
 * Metric of a Gaussian likelihood in standardized coordinates, the Fisher metric
 * plus the identity (section "Performance of NIFTy.re compared to NIFTy"):
 *   out = L^T (w * (L v)) + v,   w = mask / sigma_n^2 per final pixel.
 *   w         [n_out] (w_batch_stride = 0) or [batch][w_batch_stride >= n_out],
 *             element type double for ICR_F64, float otherwise.
 *   v, out    [batch][n_xi]; must not overlap each other or the workspace.
 *   workspace [batch][metric_workspace_elems].
 */
icr_status icr_metric_apply(const icr_plan* plan, int64_t batch, const void* w,
                            int64_t w_batch_stride, const void* v, void* out,
                            void* workspace, void* hip_stream);

/*
 * icr_metric_apply for callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same computation with no workspace
 * argument. Its workspace is a static device array of the library, 64 MiB on every GPU
 * the library runs on, held until the process ends; the call allocates nothing.
 *   w, w_batch_stride, v, out as for icr_metric_apply (v and out must not overlap).
 * Returns ICR_ERR_INVALID_ARG, launching nothing, when batch * n_xi * elem_bytes exceeds
 * 64 MiB. All calls on one GPU share the array: calls that overlap in time on one GPU
 * (different streams or threads) race and give wrong results; serialise them.
 */
icr_status icr_metric_apply_static(const icr_plan* plan, int64_t batch, const void* w, int64_t w_batch_stride,
                                   const void* v, void* out, void* hip_stream);

/*
 * Gradient of E = <s_bar, L(theta) xi> with respect to the kernel hyperparameters
 * theta = (scale sigma, length), per sample, from the results of one icr_forward and
 * one icr_adjoint (the paper learns kernel parameters by differentiating the model,
 * section "Gaussian Processes"). With the level cotangents sbar_l of the adjoint sweep,
 *   dE/dlength = <sbar_0, dL_00 xi_0> + sum_l <sbar_{l+1}, dR_l s_l[window] + dsqrtD_l xi_{l+1}>,
 *   dE/dsigma  = <s_bar, s> / sigma   (R does not depend on sigma; L_00, sqrtD scale with it),
 * where dR, dsqrtD, dL_00 are the FP64 length derivatives built with ICR_FLAG_HYPERGRAD.
 * Chaining through a loss: pass the loss gradient with respect to s as s_bar.
 *   xi          [batch][n_xi]  the excitations of the forward call.
 *   s           [batch][n_out] its output.
 *   s_levels    [batch][workspace_elems] its workspace (levels s_0 .. s_{L-1}).
 *   s_bar       [batch][n_out] the adjoint's input cotangent.
 *   sbar_levels [batch][workspace_elems] the adjoint's workspace (sbar_0 .. sbar_{L-1}).
 *   grad        device double [batch][2]: (dE/dsigma, dE/dlength).
 *   workspace   device double [batch][hypergrad_workspace_elems] (partial sums).
 * Sums run in FP64 in a fixed order (bitwise reproducible); per-term products are in
 * the plan's arithmetic type. Returns ICR_ERR_UNSUPPORTED for a plan built without
 * ICR_FLAG_HYPERGRAD. Asynchronous on hip_stream; allocates nothing.
 */
icr_status icr_hyper_grad(const icr_plan* plan, int64_t batch, const void* xi, const void* s,
                          const void* s_levels, const void* s_bar, const void* sbar_levels,
                          double* grad, double* workspace, void* hip_stream);

/*
 * Conjugate gradients on the metric M = L^T (w * L .) + 1 for `batch` independent right-
 * hand sides, entirely on the device: step sizes stay in device memory, so the whole
 * run is enqueued without host round trips. CG is how MGVI/geoVI draw samples (section
 * "Variational Inference"); this runs exactly `iterations` steps from x_0 = 0 (no early
 * exit), the i-th step being the textbook update alpha = r.r/p.Mp, x += alpha p,
 * r -= alpha Mp, p = r + (r'.r'/r.r) p. Dots accumulate in FP64 in a fixed order.
 *   w, w_batch_stride as for icr_metric_apply.
 *   b         [batch][n_xi] right-hand sides; x [batch][n_xi] receives the solution.
 *   residual_norms  optional device array [batch][iterations + 1] (double): |r_k|.
 *   workspace device scratch of icr_cg_workspace_bytes(plan, batch) bytes, 256-byte aligned.
 * FP64 and FP32 plans only (ICR_ERR_UNSUPPORTED for BF16 storage).
 */
icr_status icr_cg_workspace_bytes(const icr_plan* plan, int64_t batch, int64_t* bytes);
icr_status icr_cg_metric(const icr_plan* plan, int64_t batch, const void* w, int64_t w_batch_stride,
                         const void* b, void* x, int32_t iterations, double* residual_norms,
                         void* workspace, void* hip_stream);

/*
 * The same CG with the energy-change stopping rule of the paper's sample-drawing CG
 * (section "Variational Inference": the linear samples are drawn by CG with an
 * absolute energy tolerance "absdelta" and at most 100 iterations). The CG energy is
 * E(x) = x.Mx / 2 - b.x; with the exact line search a step lowers it by
 * alpha (r.r) / 2. A sample stops after the first step whose decrease is below absdelta
 * (that step is kept), when its residual is exactly zero, or after maxiter steps; each
 * sample of the batch stops on its own and is left unchanged from then on.
 *   absdelta        > 0, in units of E (the paper's example: 1e-4 * n_xi / 10).
 *   maxiter         >= 0 steps at most.
 *   iterations_done optional device int32 [batch]: the steps each sample took.
 *   residual_norms  optional device double [batch][maxiter + 1]: |r_k|, a stopped sample's
 *                   last value repeated to the end.
 *   workspace       icr_cg_workspace_bytes(plan, batch) bytes, 256-byte aligned.
 * The iterations are enqueued without waiting on the device (no host round trip). Once
 * every sample has stopped, a flag in the workspace makes the kernels still queued
 * return at once, and the device raises a word of pinned host memory with it, which the
 * host reads (never waits on) before enqueuing each iteration: from then on no further
 * iteration is enqueued. FP64 and FP32 plans only; asynchronous on hip_stream. Allocates
 * no device memory; a call takes a 64-byte pinned host word from a process-wide pool,
 * allocating one when every word is still held by a call whose work has not finished
 * (the words are kept until the process ends).
 */
icr_status icr_cg_metric_sl(const icr_plan* plan, int64_t batch, const void* w, int64_t w_batch_stride,
                            const void* b, void* x, double absdelta, int32_t maxiter, int32_t* iterations_done,
                            double* residual_norms, void* workspace, void* hip_stream);

/*
 * Metric Gaussian Variational Inference around this prior with a Gaussian likelihood
 * (inverse noise variance w per final pixel), section "Variational Inference". MGVI
 * draws antithetic samples mean +- delta, delta = M^-1 r with r = eta + L^T (sqrt(w)
 * eta') for standard-normal eta (n_xi) and eta' (n_out), so that delta has covariance
 * M^-1 (solve with icr_cg_metric), and moves the expansion point by Newton-CG on the KL
 * divergence, whose gradient over antithetic pairs is M mean - L^T W d.
 *
 * icr_weighted_adjoint: out = L^T (w^p * y) + add with p = 1/2 (half != 0: the sample
 * right-hand side, add = eta, y = eta') or p = 1 (half == 0: b = L^T W d with y = d,
 * add = NULL).
 *   w, w_batch_stride as for icr_metric_apply; y [batch][n_out]; add NULL or
 *   [batch][n_xi]; out [batch][n_xi]; workspace [batch][metric_workspace_elems]
 *   (storage type; must not overlap the other buffers).
 * icr_mgvi_newton_step: mean <- mean - M^-1 (M mean - b) for `batch` independent
 * problems, M^-1 by `iterations` CG steps from 0 (icr_cg_metric's iteration);
 * residual_norms as for icr_cg_metric. FP64 and FP32 plans only.
 *   b, mean   [batch][n_xi]; workspace device, icr_mgvi_workspace_bytes, 256-byte aligned.
 * Random numbers are inputs: the caller draws eta, eta'. Asynchronous on hip_stream;
 * no allocation.
 */
icr_status icr_weighted_adjoint(const icr_plan* plan, int64_t batch, const void* w, int64_t w_batch_stride,
                                int32_t half, const void* y, const void* add, void* out, void* workspace,
                                void* hip_stream);
icr_status icr_mgvi_workspace_bytes(const icr_plan* plan, int64_t batch, int64_t* bytes);
icr_status icr_mgvi_newton_step(const icr_plan* plan, int64_t batch, const void* w, int64_t w_batch_stride,
                                const void* b, void* mean, int32_t iterations, double* residual_norms,
                                void* workspace, void* hip_stream);

/*
 * One level of the sweep, for callers that pipeline or shard levels themselves
 * (icr_forward and icr_adjoint are these calls in sequence). Strides are elements
 * between consecutive samples and must be >= the level's size.
 *   level >= 0: refinement level -> level+1.
 *     forward:  s_fine = R s_coarse[window] + sqrtD xi_fine;
 *     adjoint:  xi_bar_fine = sqrtD^T y_fine, s_bar_coarse = gathered R^T y_fine.
 *   level == -1: level 0. forward: s_fine = L00 xi_fine (s_coarse unused, may be
 *     NULL); adjoint: xi_bar_fine = L00^T y_fine (s_bar_coarse unused).
 * Same conventions as icr_forward (asynchronous, no allocation, no overlap).
 */
icr_status icr_forward_level(const icr_plan* plan, int32_t level, int64_t batch,
                             const void* s_coarse, int64_t coarse_stride,
                             const void* xi_fine, int64_t xi_stride,
                             void* s_fine, int64_t fine_stride, void* hip_stream);
icr_status icr_adjoint_level(const icr_plan* plan, int32_t level, int64_t batch,
                             const void* y_fine, int64_t y_stride,
                             void* xi_bar_fine, int64_t xi_bar_stride,
                             void* s_bar_coarse, int64_t coarse_stride, void* hip_stream);

/* Free the plan's device memory. NULL is a no-op. Not safe while calls using the
 * plan are still running on a stream. */
icr_status icr_plan_destroy(icr_plan* plan);

/* Message of the last failed call on this thread (thread-local, valid until the
 * thread's next icr_* call). "" after a successful call. */
const char* icr_last_error(void);

/* Library version as 10000*major + 100*minor + patch. */
int32_t icr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ICR_H */
