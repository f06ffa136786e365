/*
 * vfmm -- velocity of N regularised vortex particles by a uniform-quadtree Fast
 * Multipole Method on one AMD MI355X (gfx950) GPU.
 *
 * The method is the one characterised by F. A. Cruz and L. A. Barba,
 * "Characterization of the errors of the Fast Multipole Method approximation in
 * particle simulations" (2008):
 *   - the velocity of Gaussian vortex blobs, eq. 6-7 (direct sum, eq. 9);
 *   - a uniform quadtree of L levels (Section 3.3, Fig. 6) with local lists and
 *     interaction lists (Section 3.3.1);
 *   - p-term multipole and local expansions of the singular far-field kernel
 *     (eq. 14-22), translated by M2M (Section 3.3.2), M2L (eq. 22) and L2L
 *     (Section 3.3.3), evaluated by L2P; the near field is summed directly with
 *     the regularised kernel (eq. 10).
 *
 * Conventions shared by every entry point
 *   - Particles are given as structure-of-arrays float64: x[n], y[n], gamma[n]
 *     (position and circulation).  Velocities u[n], v[n] are float64 and are
 *     written in the caller's particle order.  Targets are the particles
 *     themselves; the self term is excluded (eq. 9), and coincident particles
 *     contribute zero.
 *   - Array arguments are DEVICE pointers unless marked (host).  The caller owns
 *     every input, output and workspace buffer; the library never allocates
 *     device memory.  The library owns only the opaque tree and batch handles,
 *     each with the HIP stream and events it creates (released with it).
 *   - Calls that take a `stream` (a hipStream_t passed as void*, NULL = the
 *     default stream) are asynchronous: they validate arguments on the host,
 *     enqueue kernels and return.  The caller synchronises before reading
 *     results.  A tree must not be used from two streams at once.
 *   - Every entry point returns a status; 0 (VFMM_OK) is success and negative
 *     values are errors.  On error nothing has been enqueued (argument errors)
 *     or the outputs are unspecified (HIP errors); vfmm_last_error() returns a
 *     thread-local message.  No entry point aborts or throws.  A HIP call that
 *     runs out of memory, or a host handle that cannot be allocated, gives
 *     VFMM_ERR_OUT_OF_MEMORY; NaN and infinite values are reported only by the
 *     opt-in check of vfmm_tree_set_check_finite (VFMM_ERR_NONFINITE).
 *
 * Tree conventions (the paper leaves them open; fixed here):
 *   - root box: the bounding square of the particles, side
 *     S = max extent * (1 + 2^-20), centred on the bounding-box midpoint
 *     (S = 1 for a zero extent), or a caller-given square;
 *   - leaf of a particle: ix = clamp(floor(((x - x0) / S) * 2^L), 0, 2^L - 1),
 *     likewise iy (a particle on a box edge belongs to the upper/right box);
 *   - expansion centres are geometric box centres; M2L starts at level 2;
 *     with L <= 1 every pair is near and the result equals the direct sum.
 */
#ifndef VFMM_H
#define VFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vfmm_status_t;

#define VFMM_OK 0
#define VFMM_ERR_INVALID_ARG (-1)
#define VFMM_ERR_OUT_OF_MEMORY (-2) /* a host handle or a HIP object could not be allocated */
#define VFMM_ERR_HIP (-3)
#define VFMM_ERR_UNSUPPORTED (-4)
#define VFMM_ERR_NONFINITE (-5)     /* opt-in finiteness check found NaN or infinity */
#define VFMM_ERR_WORKSPACE (-6)

/* Arithmetic of the evaluation (vfmm_fmm_velocity `precision`).
 *   VFMM_FP64      : every step in float64.
 *   VFMM_FP32      : P2M, M2M, M2L, L2L, L2P and P2P in float32 on scaled
 *                    coefficients; the P2P source loop keeps compensated float32
 *                    sums; output float64.  For p > 16 the shifts (P2M, M2M,
 *                    L2L) run in float64 and M2L stays float32 on the matrix
 *                    cores (so do the two modes below).
 *   VFMM_M2L_BF16  : as VFMM_FP32 but M2L on bfloat16 matrix cores with float32
 *                    accumulation.
 *   VFMM_M2L_FP16  : as VFMM_FP32 but M2L on float16 matrix cores with float32
 *                    accumulation. */
#define VFMM_FP64 0
#define VFMM_FP32 1
#define VFMM_M2L_BF16 2
#define VFMM_M2L_FP16 3

/* Which part of eq. 10 vfmm_fmm_velocity_parts writes. */
#define VFMM_PART_NEAR 1
#define VFMM_PART_FAR 2
#define VFMM_PART_ALL 3

#define VFMM_MAX_P 40
#define VFMM_MAX_LEVELS 12

typedef struct vfmm_tree_s* vfmm_tree_t;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t vfmm_version(void);

/* Human-readable name of a status code (static string). */
const char* vfmm_status_string(vfmm_status_t status);

/* Detail of the last error raised on the calling thread (static per thread). */
const char* vfmm_last_error(void);

/* Bytes of device workspace that vfmm_build_tree needs for n particles, a tree
 * of `levels` levels (leaf level L, 0 <= L <= 12) and expansions of up to p_max
 * terms (1 <= p_max <= 40).  `bytes` is a host pointer.  The workspace holds the
 * sorted particles, the leaf ranges, the multipole and local coefficients of
 * levels 2..L (Section 3.3: 4^l boxes per level) and the translation tables. */
vfmm_status_t vfmm_workspace_bytes(int64_t n, int32_t levels, int32_t p_max, size_t* bytes);

/* Builds the quadtree of Section 3.3 over the particles (x, y) (device, n each,
 * 1 <= n <= 2^31 - 1): root box, leaf of every particle, sort of the particles
 * by leaf (row-major leaf order; inside a leaf by the Morton index of the
 * particle's cell at level L + 4, ties in input order), leaf ranges, box-local
 * coordinates and the near-field target tiles.
 *   domain    (host, may be NULL): {x0, y0, S}, lower-left corner and side of the
 *             root square; NULL = bounding square of the particles.  Particles
 *             outside a given square are clamped into its edge boxes.
 *   workspace (device): at least vfmm_workspace_bytes(n, levels, p_max) bytes,
 *             256-byte aligned; owned by the caller, used by the tree until
 *             vfmm_tree_destroy.  x and y are read only during this call's
 *             kernels; they may change afterwards.
 *   out       (host): receives the tree handle.
 * Errors: VFMM_ERR_INVALID_ARG (null pointer, n, levels or p_max out of range,
 * non-finite or non-positive domain side), VFMM_ERR_WORKSPACE (too small or
 * misaligned), VFMM_ERR_HIP (launch failure). */
vfmm_status_t vfmm_build_tree(const double* x, const double* y, int64_t n, int32_t levels,
                              const double* domain, int32_t p_max, void* workspace,
                              size_t ws_bytes, void* stream, vfmm_tree_t* out);

/* FMM velocity of eq. 9 (the approximation of eq. 10): u[n], v[n] (device) at
 * every particle of the tree, in input order.
 *   gamma     (device, n): circulations, input order (eq. 2, 13).
 *   sigma     : Gaussian core size (eq. 3, 6), finite and > 0.
 *   p         : expansion terms, 1 <= p <= p_max of the tree (eq. 21).
 *   precision : VFMM_FP64, VFMM_FP32, VFMM_M2L_BF16 or VFMM_M2L_FP16.
 * Streams: the call is ordered on `stream` (after the work queued on it before
 * the call, before the work queued after it).  Inside, the gather of the
 * circulations and the expansion sweeps (tables, P2M, M2M, M2L + L2L) run on a
 * stream owned by the tree (created with it, default priority), concurrently
 * with the near-field schedule and the near field on `stream`; `stream` waits
 * for the gather (an event) before the near field and for the sweeps before
 * the far field is added.  Calls on one tree from different streams race, as
 * they share the tree's workspace.
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_HIP. */
vfmm_status_t vfmm_fmm_velocity(vfmm_tree_t tree, const double* gamma, double sigma, int32_t p,
                                int32_t precision, double* u, double* v, void* stream);

/* One call for one evaluation (eq. 9-10): vfmm_build_tree over (x, y) with the
 * bounding square and p_max = p, vfmm_fmm_velocity, then the tree handle is
 * released (the enqueued work still completes on `stream`).  workspace: at
 * least vfmm_workspace_bytes(n, levels, p) bytes, as for vfmm_build_tree.
 * Errors: those of the two calls. */
vfmm_status_t vfmm_fmm_velocity_oneshot(const double* x, const double* y, const double* gamma,
                                        int64_t n, double sigma, int32_t p, int32_t levels,
                                        int32_t precision, double* u, double* v, void* workspace,
                                        size_t ws_bytes, void* stream);

/* As vfmm_fmm_velocity, writing only the near part (P2P over the local list,
 * eq. 10 first sum), only the far part (the expansions, eq. 10 second sum) or
 * both (`parts` = VFMM_PART_NEAR, VFMM_PART_FAR or VFMM_PART_ALL). */
vfmm_status_t vfmm_fmm_velocity_parts(vfmm_tree_t tree, const double* gamma, double sigma,
                                      int32_t p, int32_t precision, int32_t parts, double* u,
                                      double* v, void* stream);

/* Bytes of device workspace that vfmm_fmm_velocity_at needs for n_targets
 * evaluation points (0 <= n_targets <= 2^31 - 1) of a tree with `levels`
 * levels.  `bytes` is a host pointer.  The workspace holds the points sorted
 * into the tree's leaves, their leaf-local coordinates and their tiles. */
vfmm_status_t vfmm_targets_workspace_bytes(int64_t n_targets, int32_t levels, size_t* bytes);

/* FMM velocity at separate evaluation points (eq. 8, as in the error maps of
 * Section 5.2) instead of at the particles: u[n_targets], v[n_targets]
 * (device) at the points (xt, yt) (device, n_targets each), in their order.
 * The particles' expansions are formed as in vfmm_fmm_velocity (and left in
 * the tree, as that call leaves them).  A point belongs to the leaf given by
 * the tree's floor-and-clamp rule; its near field sums the regularised kernel
 * (eq. 6) over the particles of that leaf's 3 x 3 local list (a particle at
 * the point itself contributes zero), its far field is the L2P of that leaf's
 * local expansion.  Points outside the closed root square of the tree (or
 * with NaN coordinates) receive NaN: no leaf expansion converges there; give
 * vfmm_build_tree a domain that covers them.
 *   gamma, sigma, p, precision, parts: as in vfmm_fmm_velocity_parts.
 *   workspace (device): at least vfmm_targets_workspace_bytes(n_targets,
 *             levels) bytes, 256-byte aligned, caller-owned, used only by
 *             this call's kernels (separate from the tree's workspace).
 * n_targets = 0 does nothing (xt, yt, u, v, workspace may then be NULL).
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_WORKSPACE, VFMM_ERR_HIP. */
vfmm_status_t vfmm_fmm_velocity_at(vfmm_tree_t tree, const double* gamma, double sigma, int32_t p,
                                   int32_t precision, int32_t parts, const double* xt,
                                   const double* yt, int64_t n_targets, void* workspace,
                                   size_t ws_bytes, double* u, double* v, void* stream);

/* FMM velocity on an adaptive quadtree (the paper uses uniform trees, Section
 * 3.3; this is the reading for leaves at different levels): a box is split
 * while it holds more than leaf_capacity particles, down to the tree's leaf
 * level L, so each particle's leaf lies at a level l <= L chosen by the local
 * density.  A particle's near field sums the regularised kernel (eq. 6) over
 * the particles of the 3 x 3 boxes of level l around its leaf (the local list
 * at the leaf's own level, Section 3.3.1); its far field is the L2P of its
 * leaf's local expansion, formed as in the uniform method (M2L over the
 * interaction lists of the leaf and its ancestors, L2L down the ancestors;
 * the multipoles are those of the tree's leaf-level boxes and their M2M
 * parents, whatever the adaptive tree does inside them).  With the tree's
 * near radius (vfmm_tree_set_near_radius) the cut-off uses the rings around
 * each adaptive leaf, the radius clamped to VFMM_NEAR_RINGS_MAX sides of that
 * leaf.  leaf_capacity = 0 puts every leaf at level L: the result is then
 * that of vfmm_fmm_velocity_parts, bit for bit.
 *   gamma, sigma, p, precision, parts: as in vfmm_fmm_velocity_parts.
 *   leaf_capacity: >= 0, the largest particle count of a leaf above level L.
 *   workspace (device): at least vfmm_adaptive_workspace_bytes(n, levels)
 *             bytes, 256-byte aligned, caller-owned (the particles sorted into
 *             the adaptive leaves, box counts, tiles, the near-field schedule).
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_WORKSPACE, VFMM_ERR_HIP. */
vfmm_status_t vfmm_adaptive_workspace_bytes(int64_t n, int32_t levels, size_t* bytes);
vfmm_status_t vfmm_fmm_velocity_adaptive(vfmm_tree_t tree, const double* gamma, double sigma,
                                         int32_t p, int32_t precision, int32_t parts,
                                         int64_t leaf_capacity, void* workspace, size_t ws_bytes,
                                         double* u, double* v, void* stream);

/* Float64 direct sum of eq. 7 / eq. 9 over all n particles, evaluated at the
 * particles listed in `targets` (device int64, n_targets entries, each in
 * [0, n)) or at all particles when targets is NULL (then n_targets must be n).
 * u, v (device) receive n_targets values, in the order of `targets`.
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_HIP. */
vfmm_status_t vfmm_direct_velocity(const double* x, const double* y, const double* gamma,
                                   int64_t n, double sigma, const int64_t* targets,
                                   int64_t n_targets, double* u, double* v, void* stream);

/* Float64 direct sum of eq. 8: the velocity induced by all n particles at
 * separate evaluation points (xt, yt) (device, n_targets each), written to
 * u, v (device, n_targets) in the points' order.  A particle at a point
 * contributes zero (the limit of eq. 6).  n_targets = 0 does nothing.
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_HIP. */
vfmm_status_t vfmm_direct_velocity_at(const double* x, const double* y, const double* gamma,
                                      int64_t n, double sigma, const double* xt, const double* yt,
                                      int64_t n_targets, double* u, double* v, void* stream);

/* Bytes of device scratch needed by vfmm_error_metrics. */
size_t vfmm_metrics_scratch_bytes(void);

/* Error of (u, v) against a reference (u_ref, v_ref), all device float64 [n]
 * (Section 5.1: errors normalised by the maximum velocity).  Writes out[3]
 * (device): max_i |dW_i|, sum_i |dW_i|^2, max_i |W_ref,i|, so that
 * e_max = out[0] / out[2] and e_rms = sqrt(out[1] / n) / out[2].
 *   scratch (device): vfmm_metrics_scratch_bytes() bytes.
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_HIP. */
vfmm_status_t vfmm_error_metrics(const double* u, const double* v, const double* u_ref,
                                 const double* v_ref, int64_t n, void* scratch, double* out,
                                 void* stream);

/* vfmm_error_metrics without the scratch argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The partial sums go to a device array of
 * the library (512 x 3 float64 = 12 KB per GPU, reserved when the library is
 * loaded and held until the process ends; its address is looked up on the
 * first call made with each device current), so the call itself allocates
 * nothing and any n >= 1 fits.  All calls on one GPU share that array and it
 * keeps the last call's partial sums: calls that overlap on one GPU (different
 * streams or threads) race.  Same output and errors as vfmm_error_metrics. */
vfmm_status_t vfmm_error_metrics_noalloc(const double* u, const double* v, const double* u_ref,
                                         const double* v_ref, int64_t n, double* out,
                                         void* stream);

/* Per-point error field behind the paper's spatial error maps (Section 5):
 * out[i] = log10(|dW_i| / max |W_ref|) (device, n), with |dW_i| the distance
 * between (u_i, v_i) and (u_ref_i, v_ref_i), floored at log10(1e-300) = -300;
 * NaN inputs give NaN.  `metrics` (device) is the out[3] of a previous
 * vfmm_error_metrics call on the same arrays (metrics[2] = max |W_ref|; a zero
 * maximum is read as 1).  n = 0 does nothing.
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_HIP. */
vfmm_status_t vfmm_error_field(const double* u, const double* v, const double* u_ref,
                               const double* v_ref, int64_t n, const double* metrics,
                               double* out, void* stream);

/* Copies tree arrays out of the workspace (device destinations, any may be
 * NULL): root[4] = {x0, y0, S, w_L}; perm[n] = input index of each sorted
 * particle; leaf_start[4^L + 1] = first sorted position of each leaf
 * (row-major leaf index iy * 2^L + ix). */
vfmm_status_t vfmm_tree_arrays(vfmm_tree_t tree, double* root, int32_t* perm,
                               int32_t* leaf_start, void* stream);

/* Copies the coefficients of the last vfmm_fmm_velocity call at `level`
 * (2 <= level <= L) out as float64 complex pairs: dst[(box * p + k) * 2 + {0,1}]
 * for the 4^level boxes in row-major order (device).  kind 0 = multipole
 * M_k = sum_i Gamma_i ((z_i - c)/w)^k; kind 1 = local L_n with the far-field
 * conjugate velocity W(z) = (-j / (2 pi w)) sum_n L_n ((z - c)/w)^n, where c is
 * the box centre and w the box side at that level.  Coefficients of an FP32
 * evaluation are widened to float64. */
vfmm_status_t vfmm_tree_expansions(vfmm_tree_t tree, int32_t kind, int32_t level, double* dst,
                                   void* stream);

/* Rebuilds an existing tree in place for new positions (same n, levels, p_max
 * and workspace), as a time-stepping loop does after moving the particles.
 * Same conventions and errors as vfmm_build_tree. */
vfmm_status_t vfmm_tree_rebuild(vfmm_tree_t tree, const double* x, const double* y,
                                const double* domain, void* stream);

/* Phase timing.  Phases of one vfmm_fmm_velocity call:
 * 0 gather circulations (and, for vfmm_fmm_velocity_at, the sort of the
 * evaluation points), 1 translation tables, 2 P2M, 3 M2M (levels L-1..2),
 * 4 M2L + L2L (levels 2..L), 5 near-field work schedule, 6 near field (P2P
 * kernel), 7 L2P (after waiting for phases 1-4: sums the parts of split
 * near-field tiles, adds the far field and writes the result).  When a call
 * evaluates both parts, phases 1-4 run on the tree's stream while 5-6 run on
 * the caller's (after the gather), so their times overlap.
 * After vfmm_tree_enable_timing(tree, max_calls) (max_calls >= 1; 0 disables), the
 * next max_calls evaluations record HIP events at the beginning and end of
 * each phase on the stream that runs it (no synchronisation).  In
 * evaluations captured into a hipGraph these records only order the captured
 * work and take no timestamps when the graph is replayed: time captured work
 * from outside the graph.
 * vfmm_tree_read_timing waits for the recorded events, writes
 * ms[call * VFMM_N_PHASES + phase] (host, max_calls * VFMM_N_PHASES doubles)
 * and *n_calls (host), and starts a new recording.  Phases skipped by a call
 * read 0. */
#define VFMM_N_PHASES 8
vfmm_status_t vfmm_tree_enable_timing(vfmm_tree_t tree, int32_t max_calls);
vfmm_status_t vfmm_tree_read_timing(vfmm_tree_t tree, double* ms, int32_t* n_calls);

/* ---------------------------------------------------------------------------
 * (p, levels) selector.  The paper measures how the FMM error depends on N, the
 * number of levels and the truncation p (Sections 4-5); a 10 -> 64 -> 64 -> 1
 * GELU network learns log10 of the maximum error (normalised by the maximum
 * velocity, Section 5.1) from runs of this library, and the cheapest (p, L)
 * whose prediction meets a tolerance is chosen.
 *
 * Network parameters: VFMM_MLP_PARAMS float32 values (device), laid out as
 * W1[10][64] (row = input feature), b1[64], W2[64][64] (row = input unit),
 * b2[64], W3[64], b3.  Activations: GELU, tanh form.  Inputs are the
 * VFMM_N_FEATURES features of vfmm_selector_features, standardised by the
 * caller (x - mean) / std.  With bf16 != 0 the weights, inputs and
 * activations are rounded to bfloat16 and products accumulate in float32;
 * gradients, master weights and Adam moments are float32. */
#define VFMM_MLP_PARAMS 4929
#define VFMM_N_FEATURES 10

/* Device scratch needed by vfmm_mlp_gradient for `batch` samples. */
size_t vfmm_mlp_scratch_bytes(int64_t batch);

/* y[b] = network(x[b]) for b < batch (device arrays; x is [batch][10]). */
vfmm_status_t vfmm_mlp_forward(const float* params, int32_t bf16, const float* x, int64_t batch,
                               float* y, void* stream);

/* grad[VFMM_MLP_PARAMS] = d/dparams of mean_b (y_b - target_b)^2 and, if loss is
 * not NULL, loss[0] = that mean (device arrays).  Deterministic: per-block
 * partial gradients are summed in a fixed order.  scratch: device,
 * vfmm_mlp_scratch_bytes(batch) bytes. */
vfmm_status_t vfmm_mlp_gradient(const float* params, int32_t bf16, const float* x,
                                const float* target, int64_t batch, float* grad, float* loss,
                                void* scratch, size_t scratch_bytes, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step >= 1)
 * on params, with first/second moments m, v (device, VFMM_MLP_PARAMS each). */
vfmm_status_t vfmm_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                            float lr, void* stream);

/* Device scratch needed by vfmm_particle_stats and vfmm_select_params for n. */
size_t vfmm_select_scratch_bytes(int64_t n);

/* Particle statistics (float64, host out[12]): sum x, sum x^2, sum y, sum y^2,
 * sum Gamma, sum Gamma^2, sum |Gamma|, max |Gamma|, min x, max x, min y,
 * max y.  Synchronises `stream`. */
vfmm_status_t vfmm_particle_stats(const double* x, const double* y, const double* gamma,
                                  int64_t n, void* scratch, size_t scratch_bytes, double* stats,
                                  void* stream);

/* Host function: the 10 selector features of (p, levels, near_radius) for
 * particles with these statistics (out[10], host): p, L, log2 N, log2 N - 2L,
 * log2(max(w_L, a) / sigma) (w_L the leaf side; a the near radius of the
 * distance cut-off clamped to VFMM_NEAR_RINGS_MAX w_L, 6 sigma for
 * VFMM_NEAR_RADIUS_AUTO, none for 0: the distance below which every pair uses
 * the regularised kernel), log2(sigma / h) with h = S / sqrt(N), mean Gamma /
 * rms Gamma, log10(sum |Gamma| / max |Gamma|), std x / S, std y / S, where S is
 * the root side of vfmm_build_tree's bounding square. */
vfmm_status_t vfmm_selector_features(const double* stats, int64_t n, double sigma, int32_t p,
                                     int32_t levels, double near_radius, float* out);

/* Chooses (p, levels, near radius) for an FP32 evaluation of these particles
 * with max error <= tol: candidates p = 4..20, L = 2..min(10, level with ~4
 * particles per leaf) and near radius 0 (the paper's split),
 * VFMM_NEAR_RADIUS_AUTO or sigma sqrt(2 ln(1/tol)) (the distance cut-off, only
 * where VFMM_NEAR_RINGS_MAX leaf sides reach 6 sigma); the network (params,
 * device; bf16) predicts log10 of each candidate's error from its standardised
 * features (feat_mean, feat_std: host, 10 each); among those with prediction +
 * margin <= log10(tol) the one with the least modelled cost (near-field and
 * ring pairs counted from the leaf occupancy, expansion and translation work)
 * is returned.  If none qualifies: p = 20, L = deepest level with leaf side
 * >= 8 sigma, radius 0, *used_fallback = 1.
 * Outputs are host pointers; the call synchronises `stream`.
 * scratch: device, vfmm_select_scratch_bytes(n) bytes. */
vfmm_status_t vfmm_select_params(const double* x, const double* y, const double* gamma, int64_t n,
                                 double sigma, double tol, const float* params,
                                 const float* feat_mean, const float* feat_std, double margin,
                                 void* scratch, size_t scratch_bytes, int32_t* p, int32_t* levels,
                                 double* near_radius, double* predicted_log10,
                                 int32_t* used_fallback, void* stream);

/* Selection with audit (Section 5: the error of an evaluation measured against
 * the direct sum, eq. 7, on sampled targets and normalised by the maximum
 * velocity, Section 5.1).  Steps:
 *   1. the network's choice (vfmm_select_params; its near radius is used
 *      only with VFMM_SELECT_CUTOFF, else the paper's split);
 *   2. with VFMM_SELECT_AUDIT: that (p, L, radius) evaluated in FP32 at all particles
 *      and its e_max taken on the n_audit targets (device int64 particle
 *      indices) against (u_ref, v_ref) (device, n_audit each; NULL = the FP64
 *      direct sum there, computed now).  The choice passes if
 *      e_max <= slack * tol (a NaN or infinite error fails).  While it fails, p
 *      is raised by 2 (up to 20) at the same L and radius.  If p = 20 still fails, the
 *      conservative choice (p = 20, deepest L <= max_levels with leaf side
 *      >= 8 sigma) is evaluated in FP64 and returned (used_fallback = 1);
 *   3. with VFMM_SELECT_CUTOFF as well, for a passing FP32 choice: its
 *      neighbours, the same p at levels L - 1 .. L + 1 (>= 2, <= max_levels,
 *      at most about four particles per leaf), each with the paper's split and
 *      with the distance cut-off of the near field (Section 4.1's distance a)
 *      at VFMM_NEAR_RADIUS_AUTO and at sigma sqrt(2 ln(1/tol)) (where one
 *      pair's kernel difference falls to the tolerance; the cut-off only where
 *      VFMM_NEAR_RINGS_MAX leaf sides reach 6 sigma), each audited; the passing
 *      ones and the choice of step 2 are timed (median of time_reps tree
 *      rebuild + evaluation runs between HIP events on `stream`); the
 *      fastest neighbour is returned if it is more than 3 % faster than the
 *      choice of step 2 (the spread of repeated timings), else that choice.
 *      The trial trees take the process-wide tuning (vfmm_set_tuning).
 * Every evaluation is recorded in out->steps (at most VFMM_SELECT_TRAIL_MAX).
 *   params, feat_mean, feat_std, margin: as in vfmm_select_params.
 *   max_levels: deepest tree the workspace is sized for (<= 0: the default,
 *             min(10, deepest L with 4^L <= 4n)); deeper candidates are
 *             skipped and a deeper network choice is clamped to it.
 *   workspace (device): vfmm_select_audit_workspace_bytes(n, n_audit,
 *             max_levels) bytes, 256-byte aligned, caller-owned: the trial
 *             trees, their velocities and the audit's buffers.
 *   out (host): the choice (p, levels, precision VFMM_FP32 or VFMM_FP64,
 *             near_radius 0 / > 0 / VFMM_NEAR_RADIUS_AUTO), the network's own
 *             choice and prediction, the audited e_max of the returned choice
 *             and the steps.  Trees are built with the process-wide tuning.
 * Synchronises `stream` (many times).
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_WORKSPACE, VFMM_ERR_HIP and those of
 * the calls above. */
#define VFMM_SELECT_AUDIT 1
#define VFMM_SELECT_CUTOFF 2
#define VFMM_SELECT_TRAIL_MAX 16
typedef struct vfmm_audit_step {
  int32_t p, levels, precision;
  double near_radius;
  double emax;  /* e_max on the audit targets */
  double ms;    /* median timed rebuild + evaluation, -1 if not timed */
} vfmm_audit_step;
typedef struct vfmm_selection {
  int32_t p, levels, precision;
  double near_radius;
  int32_t used_fallback;
  int32_t network_p, network_levels, network_fallback;
  double network_radius;   /* the network's near radius (0 without VFMM_SELECT_CUTOFF) */
  double predicted_log10;  /* the network's prediction for its choice (NaN for its fallback) */
  double audit_emax;       /* audited e_max of the returned choice (NaN without audit) */
  int32_t n_steps;
  vfmm_audit_step steps[VFMM_SELECT_TRAIL_MAX];
} vfmm_selection;
vfmm_status_t vfmm_select_audit_workspace_bytes(int64_t n, int64_t n_audit, int32_t max_levels,
                                                size_t* bytes);
vfmm_status_t vfmm_select_and_audit(const double* x, const double* y, const double* gamma,
                                    int64_t n, double sigma, double tol, const float* params,
                                    const float* feat_mean, const float* feat_std, double margin,
                                    const int64_t* targets, int64_t n_audit, const double* u_ref,
                                    const double* v_ref, int32_t flags, double slack,
                                    int32_t time_reps, int32_t max_levels, void* workspace,
                                    size_t ws_bytes, vfmm_selection* out, void* stream);

/* ---------------------------------------------------------------------------
 * Batched evaluation of many independent instances (uneven n, p, levels), the
 * parameter sweeps of Section 5 run together.  Each phase runs once for all
 * instances (a global sort on (instance, leaf, sub-cell) keys, one launch per
 * phase or per level), so the launch count does not grow with the number of
 * instances, and the sequence can be captured in a hipGraph and replayed.
 * Arithmetic: near field in FP32 (compensated sums, series for close pairs);
 * expansions in FP32 for p <= 16; for p > 16 P2M, M2M, L2L and L2P in FP64 with
 * the M2L in FP32 on the matrix cores. */
typedef struct vfmm_instance {
  const double* x;      /* device, n: positions */
  const double* y;
  const double* gamma;  /* device, n: circulations */
  double* u;            /* device, n: velocity out (input order) */
  double* v;
  int64_t n;            /* >= 1; sum over instances <= 2^31 - 1 */
  double sigma;         /* > 0 */
  int32_t p;            /* 1 .. 24 */
  int32_t levels;       /* 0 .. 6 */
} vfmm_instance;

typedef struct vfmm_batch_s* vfmm_batch_t;

/* Device workspace for a batch of `count` instances (1 .. 4096), host array. */
vfmm_status_t vfmm_batch_workspace_bytes(const vfmm_instance* inst, int32_t count, size_t* bytes);

/* Plans a batch: validates the instances, lays out the workspace (256-byte
 * aligned, caller-owned) and uploads the per-instance offset tables
 * (synchronous).  The instance pointers are recorded: later runs read and
 * write the same buffers, whose contents may change between runs. */
vfmm_status_t vfmm_batch_create(const vfmm_instance* inst, int32_t count, void* workspace,
                                size_t ws_bytes, vfmm_batch_t* out);

/* Evaluates every instance.  use_graph = 0: enqueue the kernels on `stream`.
 * use_graph = 1: the first call captures the sequence in a hipGraph on
 * `stream` (which must not be the NULL stream) and every call replays it.
 * The first call also builds the translation tables (outside any capture).
 * Streams: once the particles are sorted into their leaves, the expansion
 * sweeps (P2M, M2M, M2L, L2L) run on a stream owned by the plan (created with
 * it, default priority) beside the near-field tiles and the near field on
 * `stream`, which waits for them (events) before L2P; captured,
 * the two become branches of the graph.  The call behaves as one ordered
 * sequence on `stream`; runs of one plan from different streams race. */
vfmm_status_t vfmm_batch_run(vfmm_batch_t batch, int32_t use_graph, void* stream);

/* Releases the plan with its graph, stream and events (not the workspace).
 * NULL is ignored. */
void vfmm_batch_destroy(vfmm_batch_t batch);

/* Kernel-substitution floor of every instance (as vfmm_substitution_bound
 * with the instance's bounding square, levels and sigma, the paper's split):
 * bound (host, count) receives 1 / (exp(w_L^2 / 2 sigma^2) - 1) per instance,
 * for the bounding squares of the last run, which the call waits for.
 * Errors: VFMM_ERR_INVALID_ARG (NULL pointer, no run yet), VFMM_ERR_HIP. */
vfmm_status_t vfmm_batch_substitution_bounds(vfmm_batch_t batch, double* bound);

/* One call for one batched evaluation (Sections 3.1-3.3 per instance):
 * vfmm_batch_create, vfmm_batch_run without a graph on `stream`, then the plan
 * is released (the enqueued work still completes).  workspace: at least
 * vfmm_batch_workspace_bytes(inst, count) bytes.  The plan's tables are
 * uploaded synchronously, so this call blocks the host briefly.
 * Errors: those of the two calls. */
vfmm_status_t vfmm_fmm_velocity_batched(const vfmm_instance* inst, int32_t count, void* workspace,
                                        size_t ws_bytes, void* stream);

/* Distance cut-off of the near field (Section 4.1: the error of taking the
 * singular kernel for a far pair is bounded through the distance a of the
 * pair).  For later evaluations of this tree (vfmm_fmm_velocity*,
 * vfmm_fmm_velocity_at), a particle outside the target's local list but
 * closer than the radius a also interacts through the regularised kernel
 * (eq. 6): Gamma (K_sigma - K') is added to the expansion result.
 *   radius = 0 (the default): the paper's split (local list only);
 *   radius > 0: a = min(radius, VFMM_NEAR_RINGS_MAX w_L), w_L the leaf side;
 *               the rings of leaves at Chebyshev distance 2 .. D are
 *               searched, D the smallest with D w_L >= a (every particle
 *               closer than D w_L lies in the local list or in those rings);
 *   radius < 0 (VFMM_NEAR_RADIUS_AUTO): a = min(r_p, VFMM_NEAR_RINGS_MAX w_L)
 *               with r_p the distance beyond which exp(-r^2 / 2 sigma^2) is
 *               below half an ulp of the evaluation's precision (6 sigma in
 *               FP32, sqrt(76) sigma in FP64), so that up to a no kernel
 *               substitution error remains at that precision.
 * The batched evaluation always uses the paper's split.
 * Errors: VFMM_ERR_INVALID_ARG (NULL tree, radius not finite). */
#define VFMM_NEAR_RADIUS_AUTO (-1.0)
#define VFMM_NEAR_RINGS_MAX 4
vfmm_status_t vfmm_tree_set_near_radius(vfmm_tree_t tree, double radius);

/* Floor of the kernel substitution (eq. 6 against eq. 15; Section 4.1).  The
 * far field sums the singular kernel K' for every pair it carries; K' differs
 * from K_sigma by exp(-r^2 / 2 sigma^2) |K'| at distance r.  Every pair closer
 * than d = max(w_L, a) is summed with K_sigma: w_L = root_side / 2^levels (two
 * leaves that are not neighbours are at least one leaf side apart), a the near
 * radius as vfmm_tree_set_near_radius resolves it for `precision` (0: none;
 * VFMM_NEAR_RADIUS_AUTO: 6 sigma in the three float32 modes, sqrt(76) sigma in
 * FP64), clamped to VFMM_NEAR_RINGS_MAX w_L.
 *   *distance (host, may be NULL) = d;
 *   *bound    (host) = |K' - K_sigma| / |K_sigma| at r = d
 *             = 1 / (exp(d^2 / 2 sigma^2) - 1),
 * the largest relative kernel error of any pair in the far field: an error
 * floor that no expansion order removes.  Above about 1e-3 the far field is
 * not a useful approximation of eq. 7 (leaves narrower than a few sigma).
 * Host only: no device work, no GPU needed.
 * Errors: VFMM_ERR_INVALID_ARG (root_side or sigma not finite and > 0, levels
 * outside 0 .. VFMM_MAX_LEVELS, radius not finite, unknown precision). */
vfmm_status_t vfmm_substitution_bound(double root_side, int32_t levels, double sigma,
                                      double near_radius, int32_t precision, double* distance,
                                      double* bound);

/* Advection of the particles with their own velocity (eq. 5, dx_i/dt = u(x_i);
 * the viscous diffusion of eq. 1 is not included).  Heun's explicit two-stage
 * Runge-Kutta method, `steps` times:
 *   x* = x + dt u(x),   x <- x + (dt / 2) (u(x) + u(x*)),
 * each stage's velocity being a vfmm_fmm_velocity evaluation (order p,
 * `precision`, the tree's near radius) after vfmm_tree_rebuild of the tree on
 * the stage's positions (root = their bounding square).
 *   x, y      (device, n each, in/out): positions in input order, advanced in
 *             place.  gamma (device, n): circulations (unchanged).
 *   workspace (device): at least vfmm_advect_workspace_bytes(n) bytes (six
 *             float64 arrays of n: both stages' velocities and the predictor
 *             positions), 256-byte aligned, caller-owned.
 * On return the tree is built on the last predictor positions.  steps = 0
 * does nothing.
 * Errors: VFMM_ERR_INVALID_ARG, VFMM_ERR_WORKSPACE, VFMM_ERR_HIP. */
vfmm_status_t vfmm_advect_workspace_bytes(int64_t n, size_t* bytes);
vfmm_status_t vfmm_advect(vfmm_tree_t tree, double* x, double* y, const double* gamma,
                          double sigma, int32_t p, int32_t precision, double dt, int32_t steps,
                          void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Tuning (process-wide settings chosen by the autotuner).  Both are read when a
 * tree is built (vfmm_build_tree); the tree keeps them for its lifetime, so
 * trees tuned differently can be evaluated side by side.
 *   VFMM_TUNE_P2P_TILE : particles per near-field tile: 64, 32 or 16 (one, two
 *                        or four lanes per target; also the source-chunk size
 *                        of the far-pair test).
 *   VFMM_TUNE_P2P_WAVES: waves per workgroup of the near-field launch: 1, 2, 4, 8.
 *   VFMM_TUNE_M2L_TILE : float32 matrix-core M2L for p <= 16: 0 = a 32-box tile
 *                        per workgroup of 4 waves with the operands loaded into
 *                        registers one offset ahead (default); 1 / 2 = the
 *                        tile's source multipoles first staged in LDS
 *                        (coalesced row loads), 4 / 8 waves per workgroup.
 *   VFMM_TUNE_P2P_SYMMETRIC: 0 (default) or 1, for trees with 64-particle
 *                        tiles (ignored otherwise): the near field at the
 *                        particles evaluates each pair of two different tiles
 *                        of the local list that hold 96 or more particles
 *                        together once, both directions from one kernel value
 *                        (K_sigma is odd: K(-r) = -K(r)); the opposite
 *                        contributions are added to float64 sums of the source
 *                        particles with atomic additions, whose order varies
 *                        from run to run (results reproducible to float64
 *                        rounding of those sums, not bit for bit).
 *                        Evaluation points and the adaptive tree always take
 *                        both directions separately.  vfmm_batch_create reads
 *                        it too: a batch planned with it uses it for the
 *                        instances with at least 48 particles per leaf on
 *                        average (a symmetric pair of chunks always takes 64
 *                        steps, which sparse leaves do not fill).
 * Results do not depend on the settings beyond float32 summation order. */
#define VFMM_TUNE_P2P_TILE 1
#define VFMM_TUNE_P2P_WAVES 2
#define VFMM_TUNE_M2L_TILE 3
#define VFMM_TUNE_P2P_SYMMETRIC 4
vfmm_status_t vfmm_set_tuning(int32_t param, int32_t value);
int32_t vfmm_get_tuning(int32_t param); /* -1 for an unknown parameter */
/* The setting a tree was built with (-1 for a NULL tree or an unknown parameter). */
int32_t vfmm_tree_get_tuning(vfmm_tree_t tree, int32_t param);

/* Opt-in finiteness check (enable != 0; 0 turns it off, the default).  After
 * every later evaluation of this tree (vfmm_fmm_velocity*, vfmm_fmm_velocity_at,
 * vfmm_advect's evaluations) the library counts NaN and infinite values among
 * the circulations, the particle positions the tree was built on, and the
 * velocities written, synchronises `stream` and returns VFMM_ERR_NONFINITE
 * (with both counts in vfmm_last_error) if any was found; the outputs are
 * written either way.  Points of vfmm_fmm_velocity_at outside the root square
 * receive NaN by definition and therefore fail the check.  Because it
 * synchronises, an evaluation on a stream under graph capture is refused
 * (VFMM_ERR_INVALID_ARG) while the check is on.  The first enable allocates two
 * counters of pinned host memory, freed with the tree.
 * Errors: VFMM_ERR_INVALID_ARG (NULL tree), VFMM_ERR_OUT_OF_MEMORY. */
vfmm_status_t vfmm_tree_set_check_finite(vfmm_tree_t tree, int32_t enable);

/* Releases the tree handle (not the caller's workspace).  NULL is ignored. */
void vfmm_tree_destroy(vfmm_tree_t tree);

#ifdef __cplusplus
}
#endif

#endif /* VFMM_H */
