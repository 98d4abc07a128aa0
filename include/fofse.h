/*
 * fofse.h - C ABI of the MI355X (gfx950) implementation of fast orthogonality
 * deficiency compensated frequency selective extrapolation (FOFSE).
 *
 * Seiler & Kaup, "Fast orthogonality deficiency compensation for improved
 * frequency selective image extrapolation".  Problem statement (Section 2,
 * Fig. 1): an area L = A u B of M x N samples; the samples of f are known on
 * the support area A, and the model g (eq. 1) built over L by K iterations
 * (eqs. 2-9 with the constant compensation of eq. 14) is the estimate of f on
 * the missing area B.  Weighting w = rho on A, 0 elsewhere (eq. 4), with the
 * isotropic model rho = rho_hat ** dist(centre) (eq. 15).  Basis functions:
 * the T x T two-dimensional DFT (Results section) or, by fofse_set_basis, the
 * T x T two-dimensional DCT (Section 2), handled entirely in the transform
 * domain.
 *
 * Conventions shared by every entry point:
 *   - "device" pointers are HIP device memory of the plan's device; "host"
 *     pointers are ordinary host memory.  The library never frees caller memory.
 *   - All calls taking a stream are asynchronous on that stream (a hipStream_t
 *     passed as void*; NULL = the null stream).  Argument errors are detected on
 *     the host, return synchronously and enqueue nothing.
 *   - Data-dependent per-block problems never abort a batch: they are reported
 *     in the per-block status word and the block's outputs are zero.
 *   - A plan may be used from one host thread and one stream at a time.
 */
#ifndef FOFSE_H
#define FOFSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fofse_plan_s* fofse_plan;   /* opaque; owned by the library */

typedef enum {
    FOFSE_OK = 0,
    FOFSE_ERR_ARG = 1,          /* invalid argument (NULL, size, range)       */
    FOFSE_ERR_UNSUPPORTED = 2,  /* valid but not built (e.g. an FFT size)     */
    FOFSE_ERR_NOMEM = 3,        /* device allocation failed                   */
    FOFSE_ERR_DEVICE = 4,       /* a HIP call or a kernel launch failed       */
    FOFSE_ERR_LIMIT = 5         /* batch beyond the fixed scratch of
                                   fofse_extrapolate_batch_noalloc            */
} fofse_status;

/* Per-block status bits written to d_status (0 = block processed normally). */
#define FOFSE_BLOCK_NO_SUPPORT   1  /* sum of weights W0 <= 0 (no usable sample)  */
#define FOFSE_BLOCK_NONFINITE    2  /* a known sample is NaN or infinite          */
#define FOFSE_BLOCK_BAD_PARAM    4  /* rho_hat not in (0,1] or gamma not in (0,1] */

/*
 * Geometry of one class of areas (Fig. 1).
 *   area_h, area_w : M, N, the area size (1 <= M, N <= fft_size).  The isotropic
 *                    model is centred at ((M-1)/2, (N-1)/2) (eq. 15).
 *   fft_size       : T, the DFT size (the paper's FFT size, Section 3).
 *                    Supported: 16, 32, 64 and 128 (128: area at most
 *                    64 x 64; no adjoint).
 *   iterations     : K >= 0, the number of iterations (the paper's I, Table 1),
 *                    at most 4096.
 *   target_mask    : host, M*N bytes row-major, non-zero on the missing area B.
 *                    Copied at creation; at least one non-zero byte.
 */
typedef struct {
    int32_t area_h;
    int32_t area_w;
    int32_t fft_size;
    int32_t iterations;
    const uint8_t* target_mask;
} fofse_geometry;

/*
 * Create a plan for one geometry on HIP device `device`.  Uploads the target
 * pixel list and the DFT twiddle table to the device (the plan owns them).
 * Returns FOFSE_ERR_ARG for an invalid geometry or NULL out, FOFSE_ERR_UNSUPPORTED
 * for an FFT size that is not built, FOFSE_ERR_NOMEM / FOFSE_ERR_DEVICE on HIP
 * failures.  *out is set only on FOFSE_OK.
 */
fofse_status fofse_create(const fofse_geometry* geometry, int32_t device,
                          fofse_plan* out);

/* Number of samples of the missing area B of the plan's geometry (0 if NULL). */
int32_t fofse_target_count(fofse_plan plan);

/*
 * Kernel organisation used by fofse_extrapolate_batch and fofse_backward
 * (results are the same up to rounding of the shared transform; each path is
 * deterministic):
 *   FOFSE_PATH_AUTO    (default) grouped when supported and the batch holds at
 *                      least 8 blocks per compute unit, split otherwise;
 *   FOFSE_PATH_SPLIT   one workgroup per block, the block's rows spread over
 *                      several wavefronts (lowest latency for few blocks);
 *   FOFSE_PATH_GROUPED blocks with identical support masks grouped on the device;
 *                      one shared W per workgroup (highest throughput).
 *                      fft_size 64: four blocks per workgroup, one wavefront
 *                      each; fft_size 128: two blocks per workgroup, four
 *                      wavefronts each.  The adjoint takes it for fft_size 64
 *                      and K <= 256 (one workgroup per block otherwise).
 * Returns FOFSE_ERR_ARG for a NULL plan or unknown path, FOFSE_ERR_UNSUPPORTED
 * if the grouped path cannot run this geometry.
 */
#define FOFSE_PATH_AUTO    0
#define FOFSE_PATH_SPLIT   1
#define FOFSE_PATH_GROUPED 2
fofse_status fofse_set_path(fofse_plan plan, int32_t path);

/*
 * Set of basis functions (Section 2: the DFT and the DCT both let the whole
 * iteration run in the transform domain, after eq. 9):
 *   FOFSE_BASIS_DFT (default) the T x T two-dimensional DFT, conjugate pairs
 *                   (everything below describes this basis unless stated);
 *   FOFSE_BASIS_DCT the orthonormal T x T DCT-II, phi_{k,l}[m,n] = a_k a_l
 *                   cos(pi k (2m+1)/(2T)) cos(pi l (2n+1)/(2T)), a_0 = sqrt(1/T),
 *                   a_k = sqrt(2/T), the area at the grid's origin.  Every
 *                   iteration picks the basis function with the largest |R_w|
 *                   among all T*T (eq. 9; ties to the smallest k*T + l), sets
 *                   c = gamma R_w[u] / sum_A w phi_u^2 (eqs. 5, 14; the
 *                   denominator depends on u) and removes c <w phi_u, phi_k> from
 *                   every R_w[k] (eq. 3).  fofse_extrapolate_batch then writes
 *                   keys k*T + l in [0, T*T) to d_sel and (c, 0) to d_coef;
 *                   blocks with identical support masks share a workgroup,
 *                   whatever the path setting.  fft_size 16, 32 or 64; no
 *                   adjoint.
 * Results of one basis never depend on the other's settings.  Selecting the
 * DCT uploads a T x T cosine table on first use (synchronous).
 * Returns FOFSE_ERR_ARG for a NULL plan or unknown basis,
 * FOFSE_ERR_UNSUPPORTED for the DCT with fft_size 128,
 * FOFSE_ERR_NOMEM / FOFSE_ERR_DEVICE if the table cannot be uploaded.
 */
#define FOFSE_BASIS_DFT 0
#define FOFSE_BASIS_DCT 1
fofse_status fofse_set_basis(fofse_plan plan, int32_t basis);

/*
 * Orthogonality deficiency compensation (Section 2):
 *   FOFSE_COMP_CONSTANT (default) the constant factor of eq. 14,
 *                       c = gamma p_u (FOFSE);
 *   FOFSE_COMP_FULL     the full compensation of eqs. 10-13 (OFSE):
 *                       c = gamma_u p_u with gamma_u = 1 / sum_l (p_l / p_u)
 *                       Khat_{u,l}.  With the DFT basis Khat_{u,l} = W[u-l] / W0,
 *                       so c = R_w[u]^2 / (R_w (*) W)[u] (cyclic convolution over
 *                       the full T x T spectrum, evaluated at the selected class
 *                       only); c is 0 when R_w[u] or the convolution is 0, and
 *                       real for a self-conjugate class.  gamma in d_rho_gamma
 *                       is not used (only rho_hat is checked).  Built with
 *                       the DFT basis for fft_size 64 (always the grouped
 *                       organisation, whatever the path setting) and for
 *                       fft_size 16 and 32 (one wavefront per block, whatever
 *                       the fofse_set_waves setting); no adjoint.
 * Returns FOFSE_ERR_ARG for a NULL plan or unknown mode, FOFSE_ERR_UNSUPPORTED
 * for FOFSE_COMP_FULL with fft_size 128, or 64 with an area or B beyond the
 * grouped organisation's limits (fofse_extrapolate_batch and
 * fofse_backward return it for FOFSE_COMP_FULL with the DCT basis, and for the
 * adjoint of FOFSE_COMP_FULL).
 */
#define FOFSE_COMP_CONSTANT 0
#define FOFSE_COMP_FULL     1
fofse_status fofse_set_compensation(fofse_plan plan, int32_t mode);

/*
 * Extrapolate n_blocks areas of the plan's geometry (Sections 2 and 3).
 *
 * For every block b, K iterations of FOFSE run in the DFT domain: the weighted
 * known samples w*f are transformed once (eqs. 7, 8); each iteration picks the
 * conjugate class with the largest |R_w| (eq. 9), estimates its coefficient
 * c = gamma * R_w[u] / W0 (eqs. 5 and 14), adds c phi_u + conj(c) phi_-u to the
 * model (eq. 2) and removes it from the weighted residual spectrum via the
 * shifted transform of w (eq. 3); the model is synthesised on B (eq. 1).
 * Arithmetic is IEEE double precision on the device.
 *
 *   d_areas      device float [n_blocks][M*N], row-major samples of f.  Samples
 *                outside A are ignored (they may hold anything finite or not).
 *   d_known      device uint8 [n_blocks][M*N], non-zero where the sample is in
 *                the support area A; bytes on B are ignored (B is never known).
 *                NULL: every block's A is the complement of B.
 *   d_rho_gamma  device double [2] = {rho_hat, gamma}, read when the kernel
 *                runs (so a captured graph sees updated values).  rho_hat in
 *                (0,1], gamma in (0,1]; otherwise every block reports
 *                FOFSE_BLOCK_BAD_PARAM.
 *   d_out        device float [n_blocks][nB] with nB = fofse_target_count():
 *                g on the samples of B in row-major order of the area.
 *   d_sel        device int32 [n_blocks][K] or NULL: canonical key u*T+v of the
 *                class selected in each iteration (u,v with v in [0,T/2], and
 *                u in [0,T/2] when v is 0 or T/2).
 *   d_coef       device double [n_blocks][K][2] or NULL: coefficient c (re, im)
 *                added for that class (im = 0 for a self-conjugate class).
 *   d_status     device int32 [n_blocks] or NULL: FOFSE_BLOCK_* bits.
 *   stream       hipStream_t (as void*), NULL for the null stream.
 *
 * The model on B is synthesised from the selection record, so when d_sel or
 * d_coef is NULL the plan keeps a record of its own (12 B per block and
 * iteration).  The grouped path and the DCT basis with per-block masks
 * (d_known non-NULL) use a plan-owned grouping workspace (about 40 B per
 * block).  Both grow when a larger batch arrives, to at least twice their
 * previous size; the buffers they replace stay allocated until fofse_destroy,
 * so a graph captured before the growth stays valid.  No buffer is allocated
 * while `stream` is being captured into a graph: a captured call must find the
 * plan's buffers large enough (make one eager call with at least as many
 * blocks first), or use fofse_extrapolate_batch_noalloc.
 *
 * Returns FOFSE_ERR_ARG (NULL plan or required pointer, n_blocks < 0),
 * FOFSE_ERR_NOMEM if a plan-owned buffer cannot be allocated,
 * FOFSE_ERR_UNSUPPORTED if one would have to grow while the stream is being
 * captured, FOFSE_ERR_DEVICE if a launch fails, FOFSE_OK otherwise.
 * n_blocks == 0 is a no-op.
 */
fofse_status fofse_extrapolate_batch(fofse_plan plan, int32_t n_blocks,
                                     const float* d_areas, const uint8_t* d_known,
                                     const double* d_rho_gamma, float* d_out,
                                     int32_t* d_sel, double* d_coef,
                                     int32_t* d_status, void* stream);

/*
 * fofse_extrapolate_batch for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, meaning and results (the same kernels, the same
 * bits) as fofse_extrapolate_batch, with two differences:
 *   - d_sel and d_coef are required (the record the model is synthesised from
 *     is the caller's);
 *   - n_blocks is at most FOFSE_NOALLOC_MAX_BLOCKS.
 * The grouping workspace lives in a fixed 5 MiB device array of the library,
 * one per device, held from the first call on that device until the process
 * ends.  Every call on a device shares it: calls that overlap on one device
 * (concurrent streams, or several host threads) race and give undefined
 * results.  The plan, and with the DCT basis its cosine table
 * (fofse_set_basis), are created beforehand; the call allocates nothing.
 * Returns FOFSE_ERR_LIMIT for n_blocks > FOFSE_NOALLOC_MAX_BLOCKS,
 * FOFSE_ERR_ARG for a NULL plan, n_blocks < 0 or a NULL required pointer
 * (d_areas, d_rho_gamma, d_out, d_sel, d_coef), FOFSE_ERR_DEVICE if the
 * array's address cannot be obtained or a launch fails, otherwise as
 * fofse_extrapolate_batch.  n_blocks == 0 is a no-op.
 */
#define FOFSE_NOALLOC_MAX_BLOCKS 65536
fofse_status fofse_extrapolate_batch_noalloc(fofse_plan plan, int32_t n_blocks,
                                             const float* d_areas, const uint8_t* d_known,
                                             const double* d_rho_gamma, float* d_out,
                                             int32_t* d_sel, double* d_coef,
                                             int32_t* d_status, void* stream);

/*
 * Wavefronts per block of the split path (FOFSE_PATH_SPLIT, and AUTO when it
 * picks the split path); 0 restores the default.  Built: T = 16: 1 (default),
 * 2; T = 32: 1, 2 (default), 4; T = 64: 2, 4 (default), 8; T = 128: 8 (default),
 * 16.  More wavefronts hold fewer rows of R each (fewer registers,
 * more exchange per iteration).  Results are the same bits for every choice of
 * a given FFT size except for the order of the transform's rounding.
 * Returns FOFSE_ERR_ARG for a NULL plan or a negative count,
 * FOFSE_ERR_UNSUPPORTED for a count not built for the plan's FFT size.
 */
fofse_status fofse_set_waves(fofse_plan plan, int32_t waves);

/*
 * Resident workgroups per compute unit of the persistent grouped kernels
 * (FOFSE_PATH_GROUPED, and AUTO when it picks the grouped path): the grid is
 * that many workgroups per compute unit, each taking a contiguous range of the
 * work items.  0 restores the default: 2 for fft_size 64 (forward and
 * adjoint: two workgroups of four blocks fit a compute unit), 1 for fft_size
 * 128.  Built: 1 or 2 for fft_size 64, 1 otherwise.  The DCT basis always runs
 * one workgroup per compute unit.  Results do not depend on it (every block is
 * computed the same way whatever its work item).
 * Returns FOFSE_ERR_ARG for a NULL plan or a negative count,
 * FOFSE_ERR_UNSUPPORTED for a count not built for the plan's FFT size.
 */
fofse_status fofse_set_occupancy(fofse_plan plan, int32_t wg_per_cu);

/*
 * Profiling hook.  With timing enabled, every fofse_extrapolate_batch and
 * fofse_backward call records a pair of HIP events on its stream around its
 * main kernel (the iteration kernel, or the adjoint kernel; the weight,
 * grouping, synthesis and summation kernels are outside; with the DCT basis
 * the one kernel iterates and synthesises).
 * The plan keeps the pairs of the last 256 calls.
 *   fofse_set_timing    enable (non-zero) or disable; enabling clears the ring.
 *                       FOFSE_ERR_ARG for a NULL plan, FOFSE_ERR_DEVICE if the
 *                       events cannot be created.
 *   fofse_kernel_times  waits for those events and writes the main-kernel
 *                       durations in milliseconds of up to `max` most recent
 *                       calls (oldest first) to host ms_out; returns how many
 *                       were written (0 for a NULL plan or ms_out, or when
 *                       timing is off).
 */
fofse_status fofse_set_timing(fofse_plan plan, int32_t enable);
int32_t fofse_kernel_times(fofse_plan plan, float* ms_out, int32_t max);

/*
 * Adjoint of fofse_extrapolate_batch with the selection held fixed.
 *
 * The paper does not differentiate the extrapolation; this is the exact
 * derivative of the forward steps (eqs. 1-5, 7, 8, 14, 15) for the classes
 * recorded by a forward call.  Given that record the model g on B is linear in
 * the known samples f, and smooth in rho_hat and gamma.  For a loss L with
 * dL/dg = d_grad_out it returns dL/df, dL/drho_hat and dL/dgamma.  Arithmetic is
 * IEEE double precision on the device.
 *
 *   d_areas, d_known, d_rho_gamma : the forward call's inputs (same layout and
 *                    meaning as in fofse_extrapolate_batch).
 *   d_sel, d_coef  : device int32 [n_blocks][K] and double [n_blocks][K][2], the
 *                    record written by the forward call on these inputs (class
 *                    keys u*T+v and coefficients c).  Keys are read modulo the
 *                    grid, so any key yields a defined result; the imaginary
 *                    part of a self-conjugate class's coefficient is taken as
 *                    0, as the forward writes it.
 *   d_grad_out     : device float [n_blocks][nB], dL/dg on the samples of B
 *                    (layout of the forward's d_out).
 *   d_grad_areas   : device float [n_blocks][M*N] or NULL: dL/df, 0 off the
 *                    support area A.
 *   d_grad_rho_gamma : device double [2] or NULL: {dL/drho_hat, dL/dgamma}
 *                    summed over the blocks in a fixed order (overwritten, not
 *                    accumulated).
 *   d_grad_block   : device double [n_blocks][2] or NULL: the same per block.
 *   stream         : hipStream_t (as void*), NULL for the null stream.
 *
 * Blocks whose forward status would be non-zero (non-finite known sample,
 * W0 <= 0, rho_hat or gamma out of range) get zero gradients.
 *
 * The plan's path (fofse_set_path) applies as in the forward: the grouped
 * adjoint (T = 64 and K <= 256) shares W and its rho_hat derivative between
 * the blocks of one support mask and runs one wavefront per block; otherwise
 * one workgroup per block.  For fft_size 128 (K <= 512) the workgroup keeps
 * the Hermitian half of W, then of D = DFT(dw/drho_hat), in LDS.  Both give the same gradients up to the order of
 * FP64 rounding, and each is deterministic: the same inputs give the same bits,
 * whatever other blocks share the batch.
 *
 * Plan-owned buffers (the per-block gradients, 16 B per block, used when
 * d_grad_block is NULL, and the grouped path's workspace) grow as in
 * fofse_extrapolate_batch, and never while the stream is being captured.
 *
 * Returns FOFSE_ERR_ARG for a NULL plan or a NULL required pointer (d_areas,
 * d_rho_gamma, d_sel, d_coef, d_grad_out) or n_blocks < 0,
 * FOFSE_ERR_UNSUPPORTED when K exceeds 2048 (512 for fft_size 128), the plan's basis is
 * the DCT (FOFSE_BASIS_DCT has no adjoint) or its compensation is
 * FOFSE_COMP_FULL, or when a plan-owned buffer would have to grow under
 * stream capture, FOFSE_ERR_NOMEM if a plan-owned buffer cannot be
 * allocated, FOFSE_ERR_DEVICE if a launch fails, FOFSE_OK otherwise.
 * n_blocks == 0 is a no-op (d_grad_rho_gamma is not written).
 */
fofse_status fofse_backward(fofse_plan plan, int32_t n_blocks,
                            const float* d_areas, const uint8_t* d_known,
                            const double* d_rho_gamma, const int32_t* d_sel,
                            const double* d_coef, const float* d_grad_out,
                            float* d_grad_areas, double* d_grad_rho_gamma,
                            double* d_grad_block, void* stream);

/* Release the plan and its device memory.  NULL is ignored. */
void fofse_destroy(fofse_plan plan);

/*
 * Several geometries in one call (Section 2's problem for areas, missing areas
 * and FFT sizes that differ from block to block).
 *
 * fofse_create_multi creates one plan per geometry (as fofse_create, with the
 * same errors; at most FOFSE_MULTI_MAX_GEOMS geometries).
 * fofse_multi_geometry_plan returns the plan of geometry g (owned by the
 * multi plan; NULL for a bad index), on which fofse_set_path, fofse_set_waves,
 * fofse_set_occupancy, fofse_set_basis, fofse_set_compensation and
 * fofse_set_timing act as on any plan.
 *
 * fofse_extrapolate_multi runs n_blocks blocks of mixed geometries:
 *   d_geom_id    device int32 [n_blocks]: geometry index of every block.
 *   d_areas      device float, packed areas: block b's M_g x N_g samples,
 *                row-major, start at element d_area_off[b].
 *   d_area_off   device int64 [n_blocks]: element offset of every block (in
 *                d_areas, d_known and d_out alike); areas may sit anywhere.
 *   d_known      device uint8, the same layout as d_areas, or NULL (every
 *                block's A is the complement of its B).
 *   d_rho_gamma  device double [2], as in fofse_extrapolate_batch.
 *   d_out        device float, the same layout as d_areas: g is written on the
 *                samples of each block's B; every other element is left as it
 *                was (d_out may be d_areas itself).
 *   d_status     device int32 [n_blocks] or NULL: FOFSE_BLOCK_* bits.
 * Every block gets exactly the result of fofse_extrapolate_batch on its
 * geometry's plan.  The blocks are sorted by geometry on the device; the call
 * then waits for the per-geometry counts (a few bytes copied to the host)
 * before it enqueues the per-geometry work, so it cannot be captured into a
 * graph (FOFSE_ERR_UNSUPPORTED under capture: use one plan per geometry
 * there).  The selection records are plan-owned.  Staging for the gathered
 * areas grows as in fofse_extrapolate_batch.
 * Returns FOFSE_ERR_ARG for a NULL plan or required pointer, n_blocks < 0,
 * or a geometry index out of range (found on the device; nothing is run
 * then), FOFSE_ERR_NOMEM, FOFSE_ERR_DEVICE, or what a geometry's
 * fofse_extrapolate_batch returns.  n_blocks == 0 is a no-op.
 *
 * fofse_destroy_multi releases the multi plan and its geometries' plans.
 */
#define FOFSE_MULTI_MAX_GEOMS 16
typedef struct fofse_multi_plan_s* fofse_multi_plan;   /* opaque; owned by the library */
fofse_status fofse_create_multi(const fofse_geometry* geometries, int32_t n_geoms, int32_t device,
                                fofse_multi_plan* out);
fofse_plan fofse_multi_geometry_plan(fofse_multi_plan plan, int32_t geom);
fofse_status fofse_extrapolate_multi(fofse_multi_plan plan, int32_t n_blocks, const int32_t* d_geom_id,
                                     const float* d_areas, const int64_t* d_area_off,
                                     const uint8_t* d_known, const double* d_rho_gamma, float* d_out,
                                     int32_t* d_status, void* stream);
void fofse_destroy_multi(fofse_multi_plan plan);

/* Static string for a status code (never NULL). */
const char* fofse_status_str(fofse_status status);

#ifdef __cplusplus
}
#endif

#endif /* FOFSE_H */
