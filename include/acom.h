/* acom.h — C ABI of the MI355X (gfx950) sparse-correlation orientation matcher.
 *
 * Method: Ophus et al., "Automated crystal orientation mapping in py4DSTEM using
 * sparse correlation matching" (arXiv 2111.00171).  Every call names the passage
 * of the paper that defines the operation it performs.
 *
 * Conventions
 *   - Pointers are DEVICE pointers unless marked [host].  Device buffers are
 *     plain global memory (hipMalloc or a framework allocator); the library
 *     never retains a caller pointer after a call returns.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *     acom_match, acom_polar_*, acom_correlate, acom_score, acom_score_grad and
 *     acom_refine are asynchronous on `stream` and allocate nothing: scratch
 *     memory is the caller's workspace.  acom_build_plan allocates the plan and
 *     synchronises `stream` before returning.
 *   - Every entry point returns an acom_status_t.  Problems the host can see
 *     (null pointers, sizes, workspace too small) return ACOM_E_INVALID or
 *     ACOM_E_WORKSPACE synchronously with a message in acom_last_error()
 *     (thread-local).  Data problems inside the peak lists (non-finite values,
 *     negative intensity, an empty pattern) are never fatal: that pattern gets
 *     zone = -1 and score = 0.  No C++ exception crosses this boundary.
 *   - Reciprocal-space quantities are spatial frequencies in 1/Angstrom (no 2 pi),
 *     angles are radians unless the name says _deg.
 *   - Orientation matrices m are 3x3 row-major with d = m d0 (sample -> crystal);
 *     columns u, v, w are the in-plane x, y axes and the zone axis
 *     (Methods > Generation of an Orientation Plan, Eq. rotation_matrices).
 */
#ifndef ACOM_H
#define ACOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ACOM_OK = 0,
  ACOM_E_INVALID = 1,     /* bad argument (see acom_last_error) */
  ACOM_E_NOMEM = 2,       /* device allocation failed (acom_build_plan only) */
  ACOM_E_HIP = 3,         /* a HIP runtime call failed */
  ACOM_E_UNSUPPORTED = 4, /* valid request the library does not support */
  ACOM_E_WORKSPACE = 5    /* workspace smaller than acom_*_workspace_size */
} acom_status_t;

/* Correlation kernel K(d) shared by the plan and the image.
 * CONE is the paper's max(1 - d/delta, 0) (plan expression and Eq. image_polar);
 * GAUSS is exp(-d^2 / 2 sigma^2) cut at d < 3 sigma (an option, not the paper's). */
typedef enum { ACOM_KERNEL_CONE = 0, ACOM_KERNEL_GAUSS = 1 } acom_kernel_t;

/* Radial axis q_s.  SHELLS: the unique |g| of the phases (the paper's radii);
 * UNIFORM: bin centres (s + 1/2) k_max / n_radial, each g reaching the bins
 * near |g| through rho = |g| - q_s inside the kernel distance. */
typedef enum { ACOM_RADIAL_UNIFORM = 0, ACOM_RADIAL_SHELLS = 1 } acom_radial_t;

/* Precision of the plan-image contraction operands (accumulation is FP32). */
typedef enum { ACOM_FP32 = 0, ACOM_BF16 = 1, ACOM_FP16 = 2 } acom_precision_t;

/* One crystal phase (Methods > Structure Factor Calculations): unit cell and
 * atomic basis, plus the zone axes to sample (Methods > Generation of an
 * Orientation Plan: a SLERP grid over one or two spherical triangles, or an
 * explicit list). */
typedef struct {
  double lattice[3][3];        /* rows a, b, c in Cartesian Angstrom */
  int32_t n_atoms;
  const double* frac_xyz;      /* [host] n_atoms x 3 fractional positions in [0,1) */
  const int32_t* species;      /* [host] n_atoms rows into f_tab, or NULL (all 0) */
  int32_t n_f;                 /* number of f_q knots; 0 -> f_n == 1 for every atom */
  const double* f_q;           /* [host] n_f knots (1/A), increasing */
  const double* f_tab;         /* [host] n_species x n_f scattering factors, linear interp. */
  int32_t n_triangles;         /* 1 or 2 (ignored when n_zones_explicit > 0) */
  double triangles[2][3][3];   /* per triangle the corner directions v0, v1, v2 (crystal Cartesian) */
  int32_t n_zones_explicit;    /* > 0: use zones_explicit instead of the triangles */
  const double* zones_explicit;/* [host] n x 3 zone-axis directions */
} acom_phase_t;

typedef struct {
  double k_max;          /* maximum scattering vector, 1/A (reflections with 0 < |g| < k_max) */
  double delta;          /* correlation kernel size delta, 1/A (paper: 0.08) */
  double gamma;          /* radial power-law weight (paper default 1) */
  double omega;          /* amplitude power-law weight (paper default 1) */
  double accel_kV;       /* beam energy for the Ewald sphere (300) */
  double zone_step_deg;  /* SLERP angular step between zone axes */
  double gauss_sigma;    /* GAUSS kernel sigma; <= 0 -> delta / 2 */
  double sigma_exc;      /* excitation tolerance of the continuous score, 1/A; <= 0 -> 0.02 */
  int32_t n_radial;      /* N_r for UNIFORM (ignored for SHELLS) */
  int32_t n_angular;     /* N_phi: even, >= 8, only prime factors 2, 3, 5, <= 1024 */
  int32_t radial;        /* acom_radial_t */
  int32_t kernel;        /* acom_kernel_t */
  int32_t precisions;    /* bit mask of (1 << acom_precision_t) operand copies to build; FP32 is always built */
  int32_t keep_f64;      /* nonzero: keep the FP64 angular plan for acom_plan_copy_f64 */
  int32_t bound_exact_freqs;  /* split bound of acom_match with FP32 operands: frequencies k < Kc bounded
                                 by their exact correlogram spectra; 0 -> Kc = min(N_phi/2 + 1, 28) */
  int32_t bound_block_radii;  /* radii per block of the Cauchy-Schwarz bound for k >= Kc: 2, 4, 8 or 16
                                 (0 -> 16) */
  int32_t bound_exact_freqs_16bit;  /* Kc for BF16 / FP16 operands; 0 -> min(N_phi/2 + 1, 48) */
} acom_plan_params_t;

typedef struct acom_plan_s* acom_plan_t;

/* Ragged peak lists, CSR (the py4DSTEM PointListArray as one flat array):
 * pattern p owns peaks offsets[p] .. offsets[p+1]-1.  (qx, qy) in 1/A with the
 * pattern centre at the origin, intensity >= 0 (Methods > Correlation Pattern
 * Matching: the M peaks (q_m, gamma_m, I_m)). */
typedef struct {
  int64_t n_patterns;    /* [host] value */
  int64_t total_peaks;   /* [host] value; must equal offsets[n_patterns] */
  const int64_t* offsets;/* n_patterns + 1, offsets[0] = 0, nondecreasing */
  const float* qx;
  const float* qy;
  const float* intensity;
} acom_peaks_t;

/* Per pattern, top_k entries ordered by decreasing score (ties: smaller zone).
 * zone is the global zone index over the concatenated phases, -1 for no match. */
typedef struct {
  int32_t* zone;         /* n x top_k */
  int32_t* phase;        /* n x top_k */
  int32_t* bin;          /* n x top_k: winning in-plane bin n (phi3 = -n 2pi/N_phi before refinement) */
  int32_t* mirror;       /* n x top_k: 1 when the mirror correlogram won */
  float* score;          /* n x top_k: correlation value C at the winning bin */
  float* phi3;           /* n x top_k: -(n + parabolic offset) 2 pi / N_phi */
  float* orient;         /* n x top_k x 9, or NULL */
  int32_t* n_evaluated;  /* n, or NULL: zones whose correlogram was evaluated exactly */
} acom_matches_t;

/* ---------------------------------------------------------------- plan ---- */

/* Build the orientation plan (Methods > Structure Factor Calculations; Methods >
 * Generation of an Orientation Plan): reflections and structure factors F_hkl,
 * zone-axis grid and rotations, P0 from the excitation error (Eq. excitation
 * error) and the kernel, per-zone normalisation A = 1/sqrt(sum P0^2) (A = 0 for a
 * zone with no excited reflection), and the 1-D FFT of P along phi3.  FP64 on
 * the GPU; the frequency-domain plan is kept in FP32 plus the requested
 * low-precision copies.  Phases are concatenated in order.  Synchronous. */
acom_status_t acom_build_plan(const acom_phase_t* phases, int32_t n_phases,
                              const acom_plan_params_t* params, void* stream, acom_plan_t* out);

/* Sizes of a built plan.  q_s [host, N_r] (the radial axis), zones [host, Z x 3],
 * zone_phase [host, Z] and norm_A [host, Z] may each be NULL. */
acom_status_t acom_plan_info(acom_plan_t plan, int32_t* n_zones, int32_t* n_radial,
                             int32_t* n_angular, int32_t* n_phases, double* q_s, double* zones,
                             int32_t* zone_phase, double* norm_A);

/* The split of the contraction pass's bound (see acom_match) for operands of
 * `precision`: Kc exact frequencies and the radii per block of the
 * Cauchy-Schwarz part; either pointer may be NULL. */
acom_status_t acom_plan_bound_split(acom_plan_t plan, int32_t precision, int32_t* exact_freqs, int32_t* block_radii);

/* Copy the FP64 angular plan P[z][a][s] (Z x N_phi x N_r) to host memory.
 * Requires keep_f64 at build time, else ACOM_E_UNSUPPORTED. */
acom_status_t acom_plan_copy_f64(acom_plan_t plan, double* host_P);

acom_status_t acom_plan_destroy(acom_plan_t plan);

/* --------------------------------------------------------------- match ---- */

/* Workspace bytes for acom_match with this many patterns per internal chunk
 * (<= 0 -> default 16384).  The size does not depend on n_patterns. */
acom_status_t acom_match_workspace_size(acom_plan_t plan, int32_t precision, int32_t chunk,
                                        size_t* bytes);

/* Match every pattern against the plan (Methods > Correlation Pattern Matching):
 * sparse polar image X (Eq. image_polar), its FFT along phi3, the per-frequency
 * contraction sum_s FFT{P}^* FFT{X} for C and FFT{P}^* FFT{X}^* for C_mirror, the
 * inverse FFT, and the maximum over zones, in-plane bins and the two branches.
 * Every reported score is computed exactly in FP32 from the FP32 plan; a zone is
 * skipped only when an upper bound of both its correlograms is below the
 * current top_k-th exact score.  The bound, computed in `precision` on MFMA
 * and widened by a precision-dependent margin, is
 *   U = (1/N) sum_k w_k T_k  (half spectrum; w_k = 1 at k = 0 and N/2, else 2),
 *   T_k = max(|G_k|, |G_m,k|)                     for k < Kc,
 *   T_k = sum_b ||FFT{P}_k,b|| ||FFT{X}_k,b||     for k >= Kc (Cauchy-Schwarz
 *         on blocks b of bound_block_radii radii),
 * with Kc (per operand precision) and the block size set at plan build
 * (acom_plan_bound_split).
 * Adds a 3-point parabolic sub-bin offset and the orientation matrix.
 * top_k in [1, 16]; `chunk` must equal the value given to the size query. */
acom_status_t acom_match(acom_plan_t plan, const acom_peaks_t* peaks, int32_t top_k,
                         int32_t precision, int32_t chunk, void* workspace, size_t workspace_bytes,
                         const acom_matches_t* out, void* stream);

/* acom_match for callers that cannot allocate or pass a workspace (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and results as acom_match without the workspace: the scratch
 * memory is a 128 MiB array in the library's device code, one per GPU, held
 * until the process ends.  The call allocates nothing and runs in chunks of
 * acom_match_noalloc_chunk patterns (the largest multiple of 64, at most
 * 16384, whose workspace fits 128 MiB: several hundred at 1081 zones x 128 x
 * 360 bins).  ACOM_E_UNSUPPORTED when not even 64 patterns fit (a plan of
 * tens of thousands of zones); use acom_match then.  Every call on a GPU uses
 * that GPU's one array: calls that overlap in time on one GPU (on different
 * streams or host threads) race and must be serialised by the caller. */
acom_status_t acom_match_noalloc(acom_plan_t plan, const acom_peaks_t* peaks, int32_t top_k, int32_t precision,
                                 const acom_matches_t* out, void* stream);
acom_status_t acom_match_noalloc_chunk(acom_plan_t plan, int32_t precision, int32_t* chunk);

/* Matching of overlapping diffraction patterns (Methods > Matching of
 * Overlapping Diffraction Patterns): n_orient rounds per pattern.  Round 0 is
 * the top-1 match of acom_match.  After each round the forward kinematical
 * pattern of the matched orientation (Methods > Calculation of Kinematical
 * Diffraction Patterns: reflection g at the (x, y) of orient^T g, intensity
 * |F_g|^2 exp(-s_g^2 / 2 sigma_exc^2), kept when above rel_cut times the phase's
 * largest |F|^2) is compared with the peaks: a peak within deletion_radius of
 * the nearest simulated peak gets intensity 0, one at a distance d below the
 * correlation kernel's reach r_k (delta for the cone kernel, 3 sigma for the
 * Gaussian) has its intensity multiplied by (d - deletion_radius) /
 * (r_k - deletion_radius); the edits accumulate and the next round matches the
 * edited peaks.  The score reported for every round is the correlogram value of
 * the ORIGINAL peaks at that round's (zone, bin, branch).  A round whose match
 * is empty or whose score is <= 0 or below min_score reports zone -1 and ends
 * the search for that pattern (later rounds report -1 too).
 * out arrays are n x n_orient (orient n x n_orient x 9, may be NULL; n_evaluated
 * is not written).  deletion_radius in [0, r_k), rel_cut in (0, 1], n_orient in
 * [1, 16].  `chunk` must equal the value given to the size query. */
acom_status_t acom_match_multi_workspace_size(acom_plan_t plan, int32_t precision, int32_t chunk,
                                              int64_t total_peaks, size_t* bytes);
acom_status_t acom_match_multi(acom_plan_t plan, const acom_peaks_t* peaks, int32_t n_orient,
                               float deletion_radius, float rel_cut, float min_score, int32_t precision,
                               int32_t chunk, void* workspace, size_t workspace_bytes,
                               const acom_matches_t* out, void* stream);

/* Autotuner of the contraction launch shape (block tile 64 x 64 or large,
 * radii per LDS step for BF16/FP16 operands, block order) for `precision` on
 * this plan: runs the polar pass on the first chunk of `peaks`, times every
 * candidate shape of the contraction on it with HIP events (one warm-up and two
 * timed launches each), and keeps the fastest in the calling host thread's
 * launch settings (see acom_set_tuning), where that thread's later calls for
 * this precision use it.  The plan is not modified.  Results of acom_match do
 * not depend on the shape.  Synchronous.  `workspace` as for
 * acom_match with the same `chunk`.  shape [host, 3] (tile: 0 = 64 x 64,
 * 1 = large; radii per LDS step, 16 or 32 for FP32 operands and 32, 64 or 128
 * for 16-bit ones; order) and ms [host] (one launch of the fastest shape) may
 * be NULL. */
acom_status_t acom_autotune(acom_plan_t plan, const acom_peaks_t* peaks, int32_t precision, int32_t chunk,
                            void* workspace, size_t workspace_bytes, void* stream, int32_t* shape, float* ms);

/* Intermediate outputs, for verification (same arithmetic as acom_match).
 * acom_polar_image: X[p][a][s] (n x N_phi x N_r, FP32), Eq. image_polar.
 * acom_polar_spectrum: FFT of X along phi3, Xr/Xi[p][k][s] (n x (N_phi/2+1) x N_r).
 * acom_correlate: C[p][z][b][n] (n x Z x 2 x N_phi, FP32), b = 0 correlogram,
 *   b = 1 mirror, computed by the FFT route in FP32.
 * All three need workspace >= acom_debug_workspace_size(plan, n_patterns). */
acom_status_t acom_debug_workspace_size(acom_plan_t plan, int64_t n_patterns, size_t* bytes);
acom_status_t acom_polar_image(acom_plan_t plan, const acom_peaks_t* peaks, float* X,
                               void* workspace, size_t workspace_bytes, void* stream);
acom_status_t acom_polar_spectrum(acom_plan_t plan, const acom_peaks_t* peaks, float* Xr, float* Xi,
                                  void* workspace, size_t workspace_bytes, void* stream);
acom_status_t acom_correlate(acom_plan_t plan, const acom_peaks_t* peaks, float* C,
                             void* workspace, size_t workspace_bytes, void* stream);
/* Upper bounds U[p][z] = (1/N) sum_k w_k max(|G_k|, |G_m,k|) (k over the half
 * spectrum, w_k = 1 at k = 0 and N/2, else 2) as computed by the contraction
 * pass in `precision` (n x Z, FP32), without margin. */
acom_status_t acom_bound(acom_plan_t plan, const acom_peaks_t* peaks, int32_t precision, float* U,
                         void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------ score / refine ---- */

/* Continuous correlation score of pattern p at orientation m = base_orient[p]
 * Exp(theta[p]) with respect to the reflections of phase[p] (an extension of the
 * polar correlation, not in the paper):
 *   S = sum_m sum_g w_m v_g K_mg / sqrt(sum_g v_g^2),
 *   w_m = q_m^gamma I_m^(omega/2) (Eq. image_polar),
 *   v_g = |g|^gamma (|F_g|^2 exp(-s_g^2 / 2 sigma_exc^2))^(omega/2)
 *         (Eq. excitation error, Eq. shape_gaussian),
 *   K_mg = exp(-|q_m - (x_g, y_g)|^2 / (2 (delta/2)^2)), (x_g, y_g, z_g) = m^T g.
 * For omega > 0, reflections whose |s_g| at the scored orientation is at least
 * 10 sigma_exc / sqrt(omega) + 0.035 1/A are left out (v_g below exp(-25) of its
 * peak value even after a 1 degree rotation).  At most 1024 reflections may take
 * part: a pattern with more gets S = NaN (and NaN gradients), never a truncated
 * sum.  A phase index outside the plan or a malformed CSR row also gives NaN.
 * base_orient n x 9, theta n x 3, phase n (int32) or NULL (phase 0); S n. */
acom_status_t acom_score(acom_plan_t plan, const acom_peaks_t* peaks, const float* base_orient,
                         const float* theta, const int32_t* phase, float* S, void* stream);

/* Backward of acom_score: given dS (n), dtheta = dS dS/dtheta (n x 3) and, when
 * dqx / dqy are not NULL, dS dS/dqx and dS dS/dqy per peak (total_peaks). */
acom_status_t acom_score_grad(acom_plan_t plan, const acom_peaks_t* peaks, const float* base_orient,
                              const float* theta, const int32_t* phase, const float* dS,
                              float* dtheta, float* dqx, float* dqy, void* stream);

/* Gradient-ascent refinement of n_cand candidate orientations per pattern
 * (init_orient n x n_cand x 9, cand_phase n x n_cand or NULL): per candidate,
 * steps of length l along grad S / |grad S| from the current orientation (l starts
 * at 0.25 deg, doubles after an improving step up to 0.5 deg, halves otherwise),
 * at most max_iter trials or until l < 1e-4 deg; the best candidate wins.  The
 * reflections taking part (as for acom_score) are chosen at the start
 * orientation and again whenever the next trial could lie more than 1 deg from
 * the orientation they were chosen at (the accepted steps since then plus the
 * trial's own step bound that rotation).
 * out_orient n x 9, out_score n, out_cand n (index of the winner) or NULL.
 * A candidate with an invalid phase or non-finite matrix is skipped (out_cand
 * = -1 and score 0 when none is left); a candidate whose reflection set exceeds
 * 1024 makes the pattern an error: out_cand = -2, out_score = NaN.
 * out_work (n x 2, or NULL) counts the kernel's work per pattern: the (peak,
 * reflection) pairs evaluated for S alone (trial steps) and for S with its
 * gradient (start and accepted orientations). */
acom_status_t acom_refine(acom_plan_t plan, const acom_peaks_t* peaks, int32_t n_cand,
                          const float* init_orient, const int32_t* cand_phase, int32_t max_iter,
                          float* out_orient, float* out_score, int32_t* out_cand, int32_t* out_work,
                          void* stream);

/* ------------------------------------------------------------ profile ---- */

/* Kernel timing with HIP events recorded on the launch stream around every
 * kernel that acom_match launches (measurement support).  The records belong to
 * the calling host thread: they cover that thread's launches only.
 * acom_profile_begin creates `capacity` event pairs and starts recording;
 * acom_profile_read synchronises the recorded events and returns, for kernel
 * kind 0 (polar image + FFT), 1 (bound contraction) or 2 (exact pass), the
 * summed duration in milliseconds and the number of launches; records beyond
 * the capacity are dropped.  acom_profile_end stops recording and frees the
 * events. */
acom_status_t acom_profile_begin(int32_t capacity);
acom_status_t acom_profile_read(int32_t kind, double* total_ms, int32_t* launches);
acom_status_t acom_profile_end(void);

/* Launch-shape tuning of the calling host thread (results do not depend on it;
 * every thread starts from the defaults below, so calls made from different
 * threads on different streams share no mutable state):
 * key 0: contraction block order, 0 = pattern tiles fastest,
 *        1 = zone tiles fastest with the tiles of one pattern group on one XCD (default);
 * key 1: radii staged per LDS step by the BF16/FP16 contraction: 32, 64 (default), 128 (the largest dividing Rp is used);
 * key 2: exact-pass pattern order, 1 = XCD-grouped (default), 0 = plain;
 * key 3: polar-pass order, 1 = consecutive patterns grouped on one XCD,
 *        0 = pattern index fastest (default);
 * key 4: contraction block tile, 0 = 64 x 64, 1 = large (128 x 128; 128 x 64 for FP32 operands),
 *        2 = large for BF16/FP16 operands when it gives at least two tiles per compute unit,
 *        else 64 x 64 (default);
 * key 5: 1 = the contraction skips the leading radii where the plan is zero in every zone
 *        (exact: those terms are zeros; default), 0 = it runs over all radii;
 * key 6: radii staged per LDS step by the FP32 contraction: 16 (default) or 32;
 * key 7: radial columns per pass of the polar (splat + FFT) kernel: 16 or 32 (default; 16 when
 *        Rp is not a multiple of 32).  The image and spectrum are bit-identical either way;
 * key 8: largest zone count (0 .. 32768, default 16384) whose per-pattern bound row the exact
 *        pass copies to LDS; larger plans select zones in place in the workspace;
 * key 9: 1 = the exact pass runs on persistent workgroups that take patterns from XCD-local
 *        work queues in the workspace, 0 = one workgroup per pattern (default).  Results are
 *        identical either way;
 * key 10: with key 2 = 1, the exact pass's patterns per XCD run (0 .. 2^20, default 1024):
 *        XCD x takes the x-th run of that many consecutive patterns out of each group of
 *        8 runs, so the device works on neighbouring patterns; 0 = one contiguous range
 *        per XCD.  Results are identical for every value.
 * A shape found by acom_autotune takes precedence over keys 0, 1, 4 and 6 for its precision
 * until one of those keys is set again. */
acom_status_t acom_set_tuning(int32_t key, int32_t value);

/* Fiber-texture zone sets (the paper's alternative orientation plans: zone
 * axes within theta_max of a fiber axis, optionally an azimuthal wedge about it)
 * for acom_phase_t.zones_explicit.  Rings of polar angle i*step about the axis
 * (i = 0 .. floor(theta_max / step)); ring i holds ceil(360 sin(theta_i) / step)
 * points evenly around a full circle (phi1 - phi0 = 360), or
 * ceil((phi1 - phi0) sin(theta_i) / step) intervals of the wedge [phi0, phi1]
 * with both ends; the axis itself comes first.  Azimuth 0 is unit(f x e) with e
 * the coordinate axis least aligned with f.  Host call, no GPU work: writes up
 * to `capacity` directions (n x 3, unit) into `zones` (may be NULL to query the
 * count) and the number needed into *count; ACOM_E_INVALID when capacity is
 * too small. */
acom_status_t acom_fiber_zones(const double* axis, double theta_max_deg, double phi0_deg, double phi1_deg,
                               double step_deg, double* zones, int32_t capacity, int32_t* count);

/* ---------------------------------------------------- forward patterns ---- */
/* Forward kinematical diffraction patterns (Methods > Calculation of
 * Kinematical Diffraction Patterns) for n orientations: a reflection g of the
 * phase (the plan's reflections, 0 < |g| < k_max) appears at the (x, y) of
 * orient^T g with intensity |F_g|^2 exp(-s_g^2 / 2 sigma_exc^2) (Eq. excitation
 * error, Gaussian shape factor) when that exceeds rel_cut (0, 1] times the
 * phase's largest |F|^2.  orient n x 9 (sample -> crystal, row-major), phase n
 * (int32) or NULL for phase 0; n in [0, 2^24].  Device pointers, asynchronous.
 * acom_simulate_count writes counts (n, int32) and the CSR offsets (n + 1,
 * int64, offsets[0] = 0); after reading offsets[n] the caller sizes the peak
 * arrays, and acom_simulate_fill writes qx, qy, intensity (offsets[n] each) in
 * the plan's reflection order within each pattern.  A phase index outside the
 * plan gives an empty pattern. */
acom_status_t acom_simulate_count(acom_plan_t plan, int64_t n, const float* orient, const int32_t* phase,
                                  float rel_cut, int32_t* counts, int64_t* offsets, void* stream);
acom_status_t acom_simulate_fill(acom_plan_t plan, int64_t n, const float* orient, const int32_t* phase,
                                 float rel_cut, const int64_t* offsets, float* qx, float* qy, float* intensity,
                                 void* stream);

/* ------------------------------------------------- Bragg disk detection ---- */
/* The peak list of each pattern comes from correlating its raw detector frame
 * with the image of the probe over vacuum (Methods > Correlation Pattern
 * Matching; Methods > Software Implementation): disk positions are the
 * correlation maxima, and a peak's intensity is the correlation value there.
 * The paper cites this step without defining it; the library computes:
 *   C[y][x] = sum_{u,v} f[(y+u) mod N][(x+v) mod N] t[u][v]   (circular, FP32 FFTs)
 * with t the probe image shifted so that its centre pixel is at the origin;
 * candidates are interior pixels (at least `edge` from every border, not
 * within `exclusion_radius` of the optical axis) whose C is strictly above all
 * 8 neighbours; kept are those with C > max(min_abs, min_rel * largest
 * candidate C), taken in order of decreasing C (ties: lower raster index
 * y*N+x first) when no kept peak is closer than `min_spacing` pixels, at most
 * `max_peaks`; each is placed at the vertex of the parabola through C at the
 * peak and its two neighbours, per axis, and reported as
 * qx = (x + dx - center_x) * pixel_size, qy = (y + dy - center_y) * pixel_size,
 * intensity = C[y][x], strongest first. */
typedef struct {
  int32_t size;            /* N: frames are N x N float32, row-major (y, x); 64 or 128 */
  int32_t edge;            /* in [1, N/2) */
  float min_rel, min_abs;  /* threshold relative to the largest candidate (>= 0), and absolute */
  int32_t min_spacing;     /* pixels, in [0, 2N]; 0 or 1 = no spacing rule */
  int32_t max_peaks;       /* in [1, 256]: slots per frame */
  float center_y, center_x;   /* optical axis, pixels */
  float exclusion_radius;     /* pixels (>= 0; 0 = none), compared as radius^2 in FP32 */
  float pixel_size;           /* 1/A per pixel (> 0) */
} acom_disk_params_t;

/* Conjugate spectrum of the probe template, scaled by 1/N^2: spectrum is
 * N x (N/2 + 1) complex (interleaved float pairs, device), computed from the
 * device probe image (N x N float32) with its centre pixel (cy0, cx0) moved to
 * the origin.  Asynchronous on stream; INVALID for other sizes or a centre
 * outside the frame. */
acom_status_t acom_disk_template(const float* probe, int32_t size, int32_t cy0, int32_t cx0, float* spectrum,
                                 void* stream);

/* Detection on n frames (device, n x N x N float32, 16-byte aligned): writes
 * counts[n] (peaks found per frame), offsets[n + 1] (exclusive prefix sum of
 * counts, int64) and per frame max_peaks slots of slot_qx, slot_qy, slot_I
 * (and slot_pixel = y*N + x when not null; all n x max_peaks, slot t of frame p
 * at p*max_peaks + t, slots beyond the count untouched).  flags (n, nullable):
 * 1 when more than 1024 candidates passed the threshold, in which case the
 * first 1024 in raster order were ranked.  One workgroup per frame (about
 * 77 KiB of LDS at N = 128), no workspace.  Asynchronous on stream; host
 * checks return INVALID (sizes, ranges, nulls, alignment, n beyond 2^26). */
acom_status_t acom_detect_disks(const float* frames, int64_t n, const float* spectrum, const acom_disk_params_t* p,
                                int32_t* counts, int64_t* offsets, float* slot_qx, float* slot_qy, float* slot_I,
                                int32_t* slot_pixel, int32_t* flags, void* stream);

/* Compacts the slots of acom_detect_disks (counts, offsets and slots as that
 * call wrote them) into CSR peak arrays qx, qy, intensity (device, `capacity`
 * entries each; offsets[n] are written, n * max_peaks always suffice) usable
 * as acom_peaks_t with these offsets.  Entries that would land outside
 * [0, capacity) are dropped, so inconsistent offsets never write out of
 * bounds.  Asynchronous on stream; INVALID for bad sizes or null pointers. */
acom_status_t acom_gather_peaks(int64_t n, int32_t max_peaks, const int32_t* counts, const int64_t* offsets,
                                const float* slot_qx, const float* slot_qy, const float* slot_I, float* qx, float* qy,
                                float* intensity, int64_t capacity, void* stream);

/* ------------------------------------------------------------- errors ---- */
const char* acom_status_string(acom_status_t s);
const char* acom_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ACOM_H */
