/*
 * rsc.h -- rotational sparse coding on gfx950 (MI355X): C ABI.
 *
 * Implements the encoding path of "Fast Rotational Sparse Coding" (McCann,
 * Andrearczyk, Unser, Depeursinge; arXiv 1806.04374): patches are mapped to
 * coordinates in a discrete steerable basis (Sec. II-D, II-E step 2) and coded
 * by orthogonal matching pursuit over every rotation of every atom, with the
 * rotation R_r replaced by the diagonal steering matrix S_r (eq. (8); Sec. II-C,
 * Fig. 2; Sec. II-E step 3).  Codes map back to pixels with Phi (Sec. II-E step 4).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns rsc_status: 0 on success, a negative code on error.
 *    Nothing aborts or prints.  rsc_last_error() gives a thread-local message for
 *    the last failure on the calling thread.
 *  - Device faults are sticky per handle: once a launch, copy or synchronisation on a
 *    handle fails, every later call on that handle (and rsc_sync with it) returns
 *    RSC_E_DEVICE with the first fault's message.  Such a handle can only be destroyed.
 *  - Device pointers are HIP device (or managed) addresses owned by the caller.
 *    The library owns only the handle and its resident copies of the basis,
 *    dictionary and tables.  Host arrays are copied before the call returns.
 *  - "stream" is a hipStream_t passed as void*; NULL is the default stream.  The
 *    compute calls only enqueue work and return; argument errors are reported
 *    synchronously, launch errors as RSC_E_DEVICE.  rsc_sync() is the call that waits.
 *  - Compute calls never allocate device memory.
 *  - Calls that use the dictionary (encode, reconstruct, synthesis, autotuning,
 *    encoder info) return RSC_E_NOT_READY until rsc_set_dictionary succeeds.
 *  - A handle may be used from one thread at a time; distinct handles are
 *    independent.
 *  - Geometry: odd patch side N; pixel (row i, col j) sits at x = j - c,
 *    y = c - i with c = (N-1)/2 (y up); angles are counter-clockwise.  The patch
 *    is the disk of radius N/2 (97 pixels at N = 11, as in Sec. III-A); pixels
 *    outside it are ignored on input and written as 0 on output.
 *  - Hat coordinates are packed real, B = S(2T+1) per patch, harmonic-major:
 *    [k=0: s=0..S-1], then for k = 1..T: [Re: s=0..S-1][Im: s=0..S-1].  A pair
 *    (a, b) of harmonic k stands for the complex coefficient (a + i b)/sqrt(2)
 *    of the circular harmonic of order k and its conjugate for order -k.
 *  - Angle index r in [0, R) means a rotation by 2*pi*r/R counter-clockwise:
 *    harmonic k of a coefficient is multiplied by exp(-i k 2 pi r / R) (eq. (6),
 *    eq. (8)).  Atom index m is in [0, M).
 */
#ifndef RSC_H
#define RSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RSC_OK = 0,
  RSC_E_INVALID = -1,      /* bad argument: null pointer, size out of range, wrong state */
  RSC_E_NOMEM = -2,        /* the library could not allocate its own resident copies */
  RSC_E_DEVICE = -3,       /* a HIP call or kernel launch failed */
  RSC_E_UNSUPPORTED = -4,  /* valid request that the library does not implement */
  RSC_E_NOT_READY = -5     /* the handle has no dictionary yet (rsc_set_dictionary) */
} rsc_status;

typedef enum {
  RSC_FP32 = 0,            /* projection and correlation in FP32 on MFMA */
  RSC_BF16 = 1,            /* correlation operands in BF16, FP32 accumulation, FP32 re-score */
  RSC_FP16 = 2             /* correlation operands in FP16, FP32 accumulation, FP32 re-score */
} rsc_precision;

/* Tile shape of the encoder (both give identical codes up to FP32 rounding order). */
typedef enum {
  RSC_TILE_AUTO = 0,       /* the library's choice: RSC_TILE_32 where it is compiled and
                              R > 32, else RSC_TILE_16 */
  RSC_TILE_16 = 1,         /* 16 patches x 8 atoms per MFMA tile (v_mfma_f32_16x16x4f32) */
  RSC_TILE_32 = 2          /* 32 patches x 16 atoms per MFMA tile (v_mfma_f32_32x32x2f32);
                              S = T = 5, K <= 4 and R <= 64 only */
} rsc_tile;

typedef struct rsc_handle rsc_handle;
typedef struct rsc_rotation_plan rsc_rotation_plan;

/*
 * Build the discrete steerable basis on the host in FP64 and upload it
 * (Sec. II-D, eq. (5)-(7); Sec. II-E step 1).
 *
 * Columns are phi_{s,k}(rho, theta) = g_s(rho) exp(i k theta) for s = 0..S-1 and
 * k = 0..T, sampled on the disk grid, with g_s(rho) = exp(-(rho - centres[s])^2 /
 * (2 sigma^2)) in place of the annulus indicator of eq. (5).  The centre pixel is
 * 0 for k != 0.  Each column is normalised (eq. (7)) and the S columns of every
 * harmonic are then made orthonormal by symmetric (Loewdin) orthonormalisation.
 * The biorthogonal partner (Phi^T Phi)^{-1} Phi^T (Sec. II-D) is formed by a
 * Cholesky factorisation.
 *
 *   N        odd patch side, 3 <= N <= 31
 *   S, T     radial profiles and largest harmonic; B = S(2T+1) <= min(n_pix, 128),
 *            T <= 15.  The pursuit (rsc_set_dictionary and everything that needs a
 *            dictionary) is compiled for (S, T) = (5, 5) and (7, 7); handles of other
 *            geometries (FP32 only) serve projection, steering and synthesis
 *   centres  host array [S] of profile centres in pixels, or NULL for
 *            centres[s] = (s+1) (N/2)/S
 *   sigma    profile width in pixels, or <= 0 for (N/2)/S (used only when
 *            centres is NULL or sigma > 0)
 *   prec     arithmetic of the encoder's correlation (rsc_precision); see
 *            rsc_omp_encode for what the 16-bit forms compute
 *   out      receives the new handle
 * Errors: RSC_E_INVALID (bad sizes, null out, singular basis), RSC_E_UNSUPPORTED
 * (geometry or precision not compiled), RSC_E_NOMEM, RSC_E_DEVICE.
 */
rsc_status rsc_create(int N, int S, int T, const double* centres, double sigma,
                      rsc_precision prec, rsc_handle** out);

/*
 * The same FP64 basis construction as rsc_create, on the host only (no device
 * needed): for inspection and host-side tests.
 *   phi   host [N*N, B] or NULL;  pinv  host [B, N*N] or NULL (layouts as in
 *   rsc_get_basis); n_pix, B, cond_gram may be NULL.  Callers size phi/pinv with
 *   B = S(2T+1).  Any S >= 1, T >= 0 is accepted here.
 */
rsc_status rsc_basis_host(int N, int S, int T, const double* centres, double sigma,
                          double* phi, double* pinv, int* n_pix, int* B, double* cond_gram);

/*
 * A handle on the paper's own discrete steerable basis (eq. (5)-(7), Sec. II-D): S =
 * floor(N/2) annuli N(s-1)/(2S) <= r < N s/(2S) on the disk grid, harmonics
 * exp(i t theta), |t| <= T_s, on annulus s, T_s = half the annulus' circumference,
 * floor(pi r_mid) (Sec. II-D's anti-aliasing rule), lowered to the largest value whose
 * 2 T_s + 1 harmonic columns are linearly independent on the annulus' pixels (as printed,
 * the 8-pixel second annulus at N = 11 would get 11 columns and Phi^T Phi would be
 * singular).  lowpass != 0 halves the cut-offs (the low-pass basis of Sec. III-C).  The
 * centre pixel is 0 for t != 0; columns are normalised; packed real coordinates are
 * harmonic-major with the annuli whose T_s >= k in block k ([Re][Im] for k >= 1, the
 * convention of rsc_create).  B = sum_s (2 T_s + 1) (81 at N = 11, 39 low-pass).
 * The handle is FP32 and serves rsc_project, rsc_steer, rsc_synthesize_hat,
 * rsc_basis_info and rsc_get_basis.  The pursuit (rsc_set_dictionary, rsc_omp_encode,
 * rsc_reconstruct) runs on the full basis at N = 11 (B = 81, T_s = 1, 3, 8, 11, 15) and
 * N = 15 (B = 153, T_s = 1, 3, 8, 11, 13, 18, 19) with even R <= 64 and K <= 4, on the
 * 16x16 encoder tile; other annular handles get RSC_E_UNSUPPORTED from
 * rsc_set_dictionary.  The dictionary update (rsc_rksvd_update, rsc_rksvd_train) runs in
 * the annular layout for B <= 160 (the full basis at N = 11 and 15).  Image projection
 * serves the full and low-pass annular bases at N = 11 and 15 (the limits of
 * rsc_project_images), and rsc_classify takes annular class handles; image stamping
 * returns RSC_E_UNSUPPORTED for every annular handle.
 *   N      odd, 3 <= N <= 31;  out  receives the handle
 * B <= 192 and T_s <= 31 are handled (N <= 15 for the full basis: B = 153 at N = 15).
 * Errors: RSC_E_INVALID (N, null out), RSC_E_UNSUPPORTED (B > 192 or some T_s > 31),
 * RSC_E_NOMEM, RSC_E_DEVICE.
 */
rsc_status rsc_create_annular(int N, int lowpass, rsc_handle** out);

/*
 * The same annular basis on the host only (no device needed).
 *   phi   host [N*N, B] or NULL;  pinv  host [B, N*N] or NULL;  Ts  host [N/2] or NULL
 *   (the cut-off of each annulus);  B, cond_gram may be NULL.  Call once with phi and
 *   pinv NULL to learn B.  N odd, 3 <= N <= 63.
 */
rsc_status rsc_annular_basis_host(int N, int lowpass, double* phi, double* pinv, int* Ts, int* B,
                                  double* cond_gram);

/* Release the handle and its device copies.  NULL is accepted. */
rsc_status rsc_destroy(rsc_handle* h);

/*
 * Sizes of the basis: disk pixel count, packed hat dimension B = S(2T+1), and the
 * 2-norm condition number of Phi^T Phi (FP64).  Any output pointer may be NULL.
 */
rsc_status rsc_basis_info(const rsc_handle* h, int* n_pix, int* B, double* cond_gram);

/*
 * Host copies of the FP64 basis for inspection: phi [N*N, B] (row = pixel in
 * row-major grid order, zero rows outside the disk) and pinv [B, N*N] (zero
 * columns outside the disk).  Either pointer may be NULL.
 */
rsc_status rsc_get_basis(const rsc_handle* h, double* phi, double* pinv);

/*
 * Load the dictionary D_hat (Sec. II-C; hat coordinates, Sec. II-E step 3) and the
 * angle grid size R.
 *   d_hat   HOST array [M, B] float32, packed hat coordinates, each row of unit
 *           Euclidean norm (|1 - ||d_m||| <= 1e-5, else RSC_E_INVALID); copied before
 *           the call returns
 *   M       1 <= M <= 256 (BF16 / FP16 handles: M <= 128)
 *   R       1 <= R <= 128 (BF16 / FP16 handles: R <= 64)
 *   stream  the upload is enqueued on it (hipStream_t as void*)
 * Stream-ordered, without a device-wide wait: the handle keeps two device copies of its
 * tables and the upload fills the one not in use.  Launches enqueued before this call
 * (on any stream) keep the previous dictionary; launches enqueued after it return use
 * the new one (on another stream they are ordered after the upload by the library).  The
 * upload waits on the device for the launches that read the copy it overwrites (the
 * dictionary before the previous one).  A HIP graph keeps the tables bound when it was
 * captured: capture again after an upload.  Blocks the host only when a copy must grow
 * or its staging buffer still feeds an earlier upload.
 * On any error the handle keeps its previous dictionary.
 * Errors: RSC_E_INVALID (arguments), RSC_E_UNSUPPORTED (sizes beyond the compiled
 * limits of the handle's precision, tables beyond the 160 KiB LDS of a CU, an annular
 * handle other than the full basis at N = 11 or 15 or with odd R or R > 64, or a geometry
 * the pursuit is not compiled for), RSC_E_NOMEM, RSC_E_DEVICE (sticky).
 */
rsc_status rsc_set_dictionary(rsc_handle* h, const float* d_hat, int M, int R, void* stream);

/*
 * Select the encoder tile shape for later rsc_omp_encode calls on this handle.
 * RSC_TILE_32 on a geometry or K it does not support makes rsc_omp_encode fall
 * back to RSC_TILE_16.  Errors: RSC_E_INVALID for an unknown value.
 */
rsc_status rsc_set_tile(rsc_handle* h, rsc_tile tile);

/*
 * Encoder launch shape: tile shape and persistent blocks per compute unit
 * (0 = as many as fit; larger requests are capped at what fits), counted in blocks
 * of 4 waves: where the FP32 16x16 encoder runs 8-wave blocks (both of its
 * dictionary tables fit a CU and the launch has at least 8 tiles of 16 patches per
 * CU) each counts as two, and a cap below two still admits one.  Codes do not
 * depend on blocks_per_cu; the tile shape changes only FP32 rounding order.
 * Errors: RSC_E_INVALID for an unknown tile or blocks_per_cu outside 0..16.
 */
rsc_status rsc_set_launch(rsc_handle* h, rsc_tile tile, int blocks_per_cu);

/*
 * The encoder kernel rsc_omp_encode would run for K on this handle: its tile shape
 * (RSC_TILE_16 or RSC_TILE_32, after resolving RSC_TILE_AUTO and fallbacks) and the
 * matrix-core floating-point operations it executes per patch when all K steps run
 * (padding included).  Either output pointer may be NULL.  For BF16 / FP16 handles
 * the count covers the 16-bit instructions only (the FP32 re-score of candidates
 * depends on the data; see rsc_precision_stats) and the tile is RSC_TILE_32.
 */
rsc_status rsc_encode_info(const rsc_handle* h, int K, int* tile, double* mfma_flops_per_patch);

/* Current encoder tile shape and blocks per CU (either pointer may be NULL). */
rsc_status rsc_get_launch(const rsc_handle* h, int* tile, int* blocks_per_cu);

/*
 * Autotuner: times rsc_omp_encode on a representative sample for every usable tile
 * shape and blocks_per_cu = 1..4 (median of reps runs, HIP events on the stream),
 * then keeps the fastest in the handle.  Blocking; not for a hot loop.
 *   xhat              device [P, B] sample, P >= 1
 *   atom, angle, coef device [P, K] scratch outputs (overwritten)
 *   reps              1..100
 *   report            host [8][3] or NULL: (tile, blocks_per_cu, median ms) per candidate
 *   n_report          host, number of rows written (may be NULL)
 * Errors: RSC_E_INVALID (arguments), RSC_E_NOT_READY (no dictionary), RSC_E_DEVICE.
 */
rsc_status rsc_autotune_encode(rsc_handle* h, const float* xhat, int64_t P, int K, int32_t* atom,
                               int32_t* angle, float* coef, int reps, double* report, int* n_report,
                               void* stream);

/*
 * Projection onto the basis (Sec. II-E step 2): xhat_p = (Phi^T Phi)^{-1} Phi^T x_p.
 *   patches  device [P, N, N] float32 row-major; off-disk pixels ignored (they must be
 *            finite: a few kernels read one of them with a zero weight)
 *   P        number of patches, >= 0 (0 is a no-op)
 *   xhat     device [P, B] float32 row-major, written
 * Asynchronous on stream.  16-byte aligned patches take the fastest kernels.
 */
rsc_status rsc_project(const rsc_handle* h, const float* patches, int64_t P, float* xhat,
                       void* stream);

/*
 * Device workspace that rsc_omp_encode needs for P patches and K atoms per patch: always
 * 0 bytes, because every per-patch value of the pursuit (residual, Cholesky factor,
 * coefficients, selections) stays in registers; admission and graph-capture code query it
 * like the other workspace sizes.  Errors: RSC_E_INVALID (null h or bytes, P < 0, K
 * outside 1..min(8, B)).
 */
rsc_status rsc_encode_workspace_size(const rsc_handle* h, int64_t P, int K, size_t* bytes);

/*
 * Rotational OMP over the augmented dictionary [S_0 D, ..., S_{R-1} D]
 * (Fig. 2 with R_r replaced by S_r; Sec. II-C and II-E step 3), K atoms per patch.
 * Each step selects the (atom, angle) of largest |<S_r d_m, residual>| (exact ties:
 * smallest m, then smallest r), refits all selected coefficients by least squares
 * and updates the residual.  A patch stops early when ||residual||^2 <=
 * 1e-10 ||xhat||^2 or when the best column is already selected.
 *   xhat         device [P, B] float32 (output of rsc_project)
 *   P            >= 0
 *   K            1 <= K <= 8 and K <= B
 *   workspace    device scratch of ws_bytes >= rsc_encode_workspace_size(h, P, K) bytes
 *                (that size is 0, so NULL with ws_bytes = 0 is the usual call)
 *   atom, angle  device [P, K] int32, slots in selection order; empty slots -1
 *   coef         device [P, K] float32; empty slots 0
 *   resid2       device [P] float32 squared hat-domain residual norm, or NULL
 * Requires rsc_set_dictionary first (else RSC_E_NOT_READY).
 *
 * BF16 / FP16 handles: the correlations of every (atom, angle) are formed with
 * 16-bit operands and FP32 accumulation; every atom whose 16-bit maximum over the
 * angles lies within 8.5u ||residual|| of the largest one (u = 2^-8 for BF16, 2^-11
 * for FP16; above twice a worst-case bound, 4.02u ||residual||, on the 16-bit error of
 * a score, so the atom with the exact maximum is always among them) is re-scored over
 * all angles in FP32, and the selection is taken from the FP32 scores.  BF16 handles
 * re-score the atom with the largest 16-bit maximum first and then only the candidates
 * whose 16-bit maximum reaches its FP32 maximum minus 4.25u ||residual|| (the atom with
 * the largest FP32 maximum always does).
 *
 * Least squares (every handle): a Cholesky update in FP32 while an upper bound on the
 * condition number of the selected columns' Gram matrix, k ||L^{-1}||_F^2, stays at or
 * below 1e3 (FP32 handles) or 1e6 (BF16 / FP16 handles) and the new pivot is above 1e-6 of
 * the column's squared norm; otherwise the patch's least squares are re-solved from scratch
 * in FP64 for this and every later step.  A column whose FP64 pivot is at most 1e-14 of its
 * squared norm (numerically inside the span of the selected ones) ends the patch's
 * pursuit.  rsc_precision_stats counts the FP64 steps.
 */
rsc_status rsc_omp_encode(const rsc_handle* h, const float* xhat, int64_t P, int K,
                          void* workspace, size_t ws_bytes,
                          int32_t* atom, int32_t* angle, float* coef, float* resid2,
                          void* stream);

/*
 * Pixels of coded patches (Sec. II-E step 4): x_p = Phi sum_i coef[p,i] S_{angle[p,i]}
 * d_{atom[p,i]}; slots with atom < 0 are skipped.
 *   atom, angle, coef  device [P, K] (as written by rsc_omp_encode)
 *   out                device [P, N, N] float32, 0 outside the disk
 * Slots with atom >= M or angle outside [0, R) are treated as empty.
 */
rsc_status rsc_reconstruct(const rsc_handle* h, const int32_t* atom, const int32_t* angle,
                           const float* coef, int64_t P, int K, float* out, void* stream);

/*
 * Synthetic patches at continuous angles: out_p = Phi sum_j weight[p,j]
 * S(theta[p,j]) d_{atom[p,j]} + noise_p, where S(theta) multiplies harmonic k by
 * exp(-i k theta) (eq. (6)).  Used to build inputs on the device.
 *   atom    device [P, J] int32 (entries outside [0, M) are skipped)
 *   theta   device [P, J] float32 radians
 *   weight  device [P, J] float32
 *   noise   device [P, N, N] float32 added to every pixel, or NULL
 *   out     device [P, N, N] float32
 *   1 <= J <= 16
 */
rsc_status rsc_synthesize(const rsc_handle* h, const int32_t* atom, const float* theta,
                          const float* weight, int64_t P, int J, const float* noise,
                          float* out, void* stream);

/*
 * Bytes of device workspace rsc_project_images needs for n_images images
 * (two int64 prefix-sum arrays of n_images + 1 entries).
 */
rsc_status rsc_images_workspace_size(int n_images, size_t* bytes);

/*
 * Projection of every stride-1 N x N window of a batch of images of uneven sizes
 * (Sec. II-E step 2 applied to all patches of each image, as in the sliding-window
 * coding of Sec. III-A).  Window p of image i has its top-left pixel at (y, x),
 * 0 <= y <= H_i - N, 0 <= x <= W_i - N; windows are numbered image by image, then
 * row-major by (y, x), and only the disk pixels of each window are used.
 *   pixels      device float32, image i row-major at pixels + img_offset[i]
 *   img_offset  device int64 [n_images];  H, W  device int32 [n_images]
 *   n_images    0 <= n_images <= 2^20 (0 is a no-op)
 *   P_total     host: sum over images of max(0, H-N+1) * max(0, W-N+1); windows past
 *               P_total are not written, so it must equal that sum
 *   workspace   device, >= rsc_images_workspace_size bytes, 8-byte aligned; holds the
 *               per-image prefix sums computed on the device (no host round trip)
 *   xhat        device [P_total, B] float32
 * Everything is enqueued on the stream without allocation or host synchronisation,
 * so a batch (with rsc_omp_encode after it) can be captured in a HIP graph.
 * Compiled for 11x11 windows with B <= 96 (the S = T = 5 grid or the annular basis) and
 * 15x15 windows with 64 < B <= 160 (the S = T = 7 grid or the annular basis);
 * RSC_E_UNSUPPORTED otherwise.
 */
rsc_status rsc_project_images(const rsc_handle* h, const float* pixels, const int64_t* img_offset,
                              const int32_t* H, const int32_t* W, int n_images, int64_t P_total,
                              void* workspace, size_t ws_bytes, float* xhat, void* stream);

/*
 * rsc_project_images without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the per-image plan lives in a static device array of the library
 * (1 MiB per device, held until the process ends), so this call allocates nothing.
 * Arguments, numbering and results as rsc_project_images; n_images <= 65535
 * (RSC_E_INVALID above).  Every call on one device shares that array: calls that overlap
 * on one device (concurrent streams or threads) race and must be ordered by the caller.
 */
rsc_status rsc_project_images_noalloc(const rsc_handle* h, const float* pixels, const int64_t* img_offset,
                                      const int32_t* H, const int32_t* W, int n_images, int64_t P_total,
                                      float* xhat, void* stream);

/*
 * Adds synthetic stamps to images: for stamp s, amplitude[s] * Phi S(theta[s]) d_{atom[s]}
 * (an N x N patch, zero off the disk) is added with its centre pixel at
 * centre[s] = (row, col) of image image[s], clipped at the image borders.  pixels must be
 * initialised by the caller (for instance with noise).  Overlapping stamps are summed
 * with atomic adds, so the rounding order of overlaps is not fixed.
 *   atom int32 [n], theta float32 [n] radians, amplitude float32 [n], centre int32 [n, 2],
 *   image int32 [n]; img_offset, H, W as in rsc_project_images; all device arrays.
 */
rsc_status rsc_synthesize_images(const rsc_handle* h, const int32_t* atom, const float* theta,
                                 const float* amplitude, const int32_t* centre, const int32_t* image,
                                 int64_t n_stamps, const int64_t* img_offset, const int32_t* H,
                                 const int32_t* W, int n_images, float* pixels, void* stream);

/*
 * Workspace bytes for rsc_rksvd_update and rsc_rksvd_train on P patches coded with K
 * slots (1 <= K <= 8), with the handle's current dictionary sizes (M, B): the pair
 * buckets (8 bytes per slot), per-chunk partial covariances (about (4096 + M) B^2
 * doubles) and small tables.  Requires a dictionary (RSC_E_NOT_READY).
 */
rsc_status rsc_rksvd_workspace_size(const rsc_handle* h, int64_t P, int K, size_t* bytes);

/*
 * Dictionary update of rotational K-SVD (Fig. 2, the loop over atoms; Sec. II-C), in hat
 * coordinates (Sec. II-E) of the handle's basis (the (S, T) grid or the annular basis),
 * from codes computed with the handle's current dictionary D.
 * Every atom is updated from the same codes and the same D (the augmented dictionary
 * of Fig. 2 is built once per outer iteration).  For atom m, each patch p whose code
 * uses m contributes the column S_{-r0}(xhat_p - D b_p): r0 is the angle of the first
 * slot (selection order) holding m and b_p the code without that entry.  The new atom
 * is the first left singular vector of those columns, with the sign that agrees with
 * the old atom (<new, old> > 0; on 0, largest-magnitude coordinate positive).  Atoms used
 * by no patch take, in index order, the directions xhat_p / ||xhat_p|| of the patches
 * with the largest coding error resid2 (positive errors only, distinct patches, ties to
 * the smaller p); with none left they keep their value.
 *   xhat                device [P, B] float32
 *   atom, angle, coef   device [P, K] codes as written by rsc_omp_encode (K <= 8)
 *   resid2              device [P] float32 coding error of each patch
 *   workspace           device, >= rsc_rksvd_workspace_size bytes, 256-byte aligned
 *   d_new               device [M, B] float32 output, unit rows
 *   usage               device [M] int32 output, patches using each atom
 *   reset               device [M] int32 output (reset patch or -1), or NULL
 * Enqueued on the stream; the handle's dictionary is not changed (pass d_new to
 * rsc_set_dictionary).  Errors: RSC_E_INVALID, RSC_E_NOT_READY, RSC_E_UNSUPPORTED
 * (B > 160, or tables of the update beyond the 160 KiB LDS of a CU: the single-value
 * dictionary 4 M B bytes plus 16 R (T + 1) bytes of rotation table), RSC_E_DEVICE.
 */
rsc_status rsc_rksvd_update(const rsc_handle* h, const float* xhat, int64_t P, int K, const int32_t* atom,
                            const int32_t* angle, const float* coef, const float* resid2, void* workspace,
                            size_t ws_bytes, float* d_new, int32_t* usage, int32_t* reset, void* stream);

/*
 * Rotational K-SVD learning loop (Fig. 2 with R_r -> S_r; Sec. II-C, II-E): loads d_init,
 * then n_iter times rsc_omp_encode + rsc_rksvd_update + rsc_set_dictionary, then one
 * more rsc_omp_encode so that the codes belong to the final dictionary.
 *   xhat                       device [P, B] float32
 *   d_init                     host [M, B] float32, unit rows; R the angle grid
 *   workspace, ws_bytes        as for rsc_rksvd_update (size queried after a dictionary
 *                              of the same M is loaded)
 *   atom, angle, coef, resid2  device outputs: codes of the final pursuit
 *   d_out                      host [M, B] float32: the learned dictionary
 *   history                    host [n_iter + 1] float64 or NULL: sum of resid2 after
 *                              each pursuit
 * Blocking (the dictionary returns to the host each iteration to rebuild the tables).
 * Errors as rsc_rksvd_update and rsc_set_dictionary; a refused call leaves the handle's
 * dictionary as it was.
 */
rsc_status rsc_rksvd_train(rsc_handle* h, const float* xhat, int64_t P, int K, int n_iter, const float* d_init,
                           int M, int R, void* workspace, size_t ws_bytes, int32_t* atom, int32_t* angle,
                           float* coef, float* resid2, float* d_out, double* history, void* stream);

/* ------------------------------------------------------------------ texture classifier
 * Sec. III-B ("Classifier"): one dictionary per class codes every patch; a patch's
 * label is the class whose pursuit leaves the smallest squared error (the pursuit's
 * hat-domain residual norm, ties to the smaller class index); an image's feature is
 * the histogram of its patches' labels as frequencies; a test image takes the class
 * of its chi^2-nearest training image, d(a, b) = sum_i (a_i - b_i)^2 / (a_i + b_i).
 */

/*
 * Workspace bytes of rsc_classify for P patches and K atoms per patch (one class's
 * codes: atom, angle, coef [P, K] and the residual norms [P]).
 */
rsc_status rsc_classify_workspace_size(int64_t P, int K, size_t* bytes);

/*
 * Labels of P patches against C class dictionaries: for c = 0..C-1 the pursuit of
 * rsc_omp_encode runs with classes[c]'s dictionary, and every patch keeps the class of
 * smallest squared error.
 *   classes     host array of C handles, each with a dictionary (RSC_E_NOT_READY
 *               otherwise) and the same basis: the same (N, S, T) grid, or the same
 *               annular basis (RSC_E_INVALID otherwise); their precisions and
 *               dictionary sizes may differ
 *   C           1 <= C <= 1024
 *   xhat        device [P, B] float32 (rsc_project of any of the handles)
 *   P, K        as rsc_omp_encode (K <= 8 and K <= B)
 *   workspace   device, >= rsc_classify_workspace_size(P, K) bytes, 256-byte aligned
 *   label       device [P] int32, written: the class index
 *   sse         device [P] float32, written: that class's squared residual norm
 * Everything is enqueued on the stream; nothing is allocated.
 */
rsc_status rsc_classify(const rsc_handle* const* classes, int C, const float* xhat, int64_t P, int K,
                        void* workspace, size_t ws_bytes, int32_t* label, float* sse, void* stream);

/*
 * Label frequencies of groups of consecutive patches (an image's windows, numbered
 * as rsc_project_images numbers them):
 *   label       device [P] int32; labels outside 0..C-1 are not counted (they still
 *               count in the group size)
 *   offset      device int64 [n_groups + 1], nondecreasing; group g is patches
 *               offset[g] .. offset[g+1]-1 (clamped into 0..P)
 *   n_groups    >= 0 (0 is a no-op);  C  1 <= C <= 4096
 *   hist        device [n_groups, C] float32: count / group size (0 for an empty group)
 */
rsc_status rsc_label_histogram(const int32_t* label, int64_t P, const int64_t* offset, int n_groups, int C,
                               float* hist, void* stream);

/*
 * chi^2 nearest neighbour: for every test histogram, the training histogram at the
 * smallest d(a, b) (computed in FP64; bins with a_i + b_i = 0 add nothing; ties to the
 * smaller training index).
 *   train       device [n_train, C] float32, n_train >= 1
 *   test        device [n_test, C] float32, n_test >= 0 (0 is a no-op)
 *   nearest     device [n_test] int32, written
 *   dist        device [n_test] float32, written (or NULL)
 */
rsc_status rsc_chi2_nearest(const float* train, int n_train, const float* test, int n_test, int C,
                            int32_t* nearest, float* dist, void* stream);

/* ------------------------------------------------------------------ patch rotation
 * Sec. III-C (rotation speed): a batch of N x N patches turned by one angle, either by
 * interpolation (the paper's sparse N^2 x N^2 matrices R_nearest and R_bicubic) or by
 * steering the hat coordinates (x_hat <- S x_hat, then Phi x_hat).  Angles are in
 * radians, counter-clockwise, about the centre pixel.
 */

/*
 * Plan of an interpolated rotation: the rows of R (1 tap per output pixel for nearest
 * neighbour, 16 for bicubic) built on the host in FP64 and uploaded to the current
 * device.  Output pixel (x, y) reads the input at R_{-theta}(x, y); nearest rounds the
 * coordinates half up; bicubic is Keys' cubic convolution (a = -1/2) over the 4 x 4
 * neighbours; input pixels outside the patch count as 0.
 *   N      odd, 3 <= N <= 25;  mode  0 = nearest, 1 = bicubic
 *   plan   written; release with rsc_rotation_plan_destroy
 */
rsc_status rsc_rotation_plan_create(int N, double theta, int mode, rsc_rotation_plan** plan);

/*
 * Rotation of 11x11 pixel patches through the steerable basis in one pass (eq. (6)-(8):
 * project onto the handle's basis, steer by theta, synthesize).  The plan holds
 * Phi S_theta Phi^+ as one 121 x 97 operator from the disk pixels to the grid (zero off the
 * disk, built in FP64 on the host, applied in FP32 on the matrix cores by rsc_rotate_interp);
 * the result equals rsc_project, rsc_steer and rsc_synthesize_hat in turn up to rounding.
 *   h      a handle of rsc_create with N = 11 (only its basis is used; it may be destroyed
 *          after this call)
 *   plan   written; release with rsc_rotation_plan_destroy
 * rsc_rotate_interp with such a plan needs 16-byte aligned patches (RSC_E_INVALID otherwise).
 * Errors: RSC_E_INVALID (arguments, non-finite theta), RSC_E_UNSUPPORTED (N != 11 or the
 * annular basis), RSC_E_NOMEM, RSC_E_DEVICE.
 */
rsc_status rsc_rotation_plan_create_steer(const rsc_handle* h, double theta, rsc_rotation_plan** plan);

/* Releases a plan's device tables (NULL is a no-op). */
rsc_status rsc_rotation_plan_destroy(rsc_rotation_plan* plan);

/*
 * R x for every patch: patches and out device float32 [P, N, N] (distinct buffers); R is the
 * plan's interpolation matrix, or Phi S_theta Phi^+ for a plan of
 * rsc_rotation_plan_create_steer (whose patches must be 16-byte aligned).  P = 0 is a no-op.
 * Asynchronous on stream.  Errors: RSC_E_INVALID (arguments, alignment), RSC_E_DEVICE.
 */
rsc_status rsc_rotate_interp(const rsc_rotation_plan* plan, const float* patches, int64_t P, float* out,
                             void* stream);

/*
 * Steering of hat coordinates (the diagonal S_theta of eq. (8) at any angle): harmonic k
 * of every patch multiplied by exp(-i k theta).
 *   xhat, out   device [P, B] float32, distinct buffers (RSC_E_INVALID if equal)
 *   theta       device float32 [P] per-patch angles, or NULL to use theta0 for all
 * Needs the handle's basis only (no dictionary); in the layout of the handle's basis (the
 * full (S, T) grid, or the annular basis' harmonic-major blocks of rsc_create_annular).
 * Asynchronous on stream.  Errors: RSC_E_INVALID (arguments, non-finite theta0),
 * RSC_E_UNSUPPORTED (a harmonic above 31), RSC_E_DEVICE.
 */
rsc_status rsc_steer(const rsc_handle* h, const float* xhat, int64_t P, const float* theta, double theta0,
                     float* out, void* stream);

/*
 * Phi x_hat on the N x N grid (zero off the disk), for any hat coordinates (Sec. II-E
 * step 4 without the dictionary).
 *   xhat    device [P, B] float32;  pixels  device [P, N, N] float32, written
 * Asynchronous on stream.  Errors: RSC_E_INVALID (arguments), RSC_E_UNSUPPORTED (B > 192),
 * RSC_E_DEVICE.
 */
rsc_status rsc_synthesize_hat(const rsc_handle* h, const float* xhat, int64_t P, float* pixels, void* stream);

/*
 * Counters of the encoder, accumulated over its launches on this handle (the FP32
 * re-scoring of candidates of the 16-bit forms and the FP64 least-squares fallback
 * described at rsc_omp_encode):
 *   out[0]  pursuit steps (patch x step) that re-scored candidates (16-bit handles; else 0)
 *   out[1]  candidates re-scored in FP32, summed over those steps (16-bit handles; else 0)
 *   out[2]  largest number of candidates in one step (16-bit handles; else 0)
 *   out[3]  steps whose least squares went to the FP64 solve (every handle)
 *   out     host [4] int64, or NULL; reset != 0 clears the counters after reading.
 * Blocking: waits for the whole device first.  Launches that overlap the call may
 * or may not be counted.
 */
rsc_status rsc_precision_stats(rsc_handle* h, int64_t* out, int reset);

/*
 * Wait for all work on the stream.  RSC_E_DEVICE if the wait reports a failed kernel (the
 * fault then becomes sticky on h) or if h already carries a sticky fault.  h may be NULL
 * (only the stream is checked).
 */
rsc_status rsc_sync(rsc_handle* h, void* stream);

/*
 * Message for the last failure on this thread; when there is none and h carries a sticky
 * fault, that fault's message; else "".  h may be NULL.  Valid until the next call.
 */
const char* rsc_last_error(const rsc_handle* h);

/*
 * Marks h as failed, as a device fault on it would (for callers that detect a fault of
 * their own on work that shares the handle's streams, and for tests of error handling):
 * every later call on h returns RSC_E_DEVICE with msg (NULL: a generic message).  A
 * handle that already carries a fault keeps its first message.  Errors: RSC_E_INVALID
 * (null h).
 */
rsc_status rsc_set_fault(rsc_handle* h, const char* msg);

#ifdef __cplusplus
}
#endif

#endif /* RSC_H */
