/*
 * bh.h -- C ABI of the MI355X ball-harmonic rotational-alignment library.
 *
 * Kruse, Kishore, Debarnot, Dokmanic, "Beyond Exhaustive Sampling: Efficient
 * Rotational Matching via Ball Harmonics" (arXiv 2509.01180).
 *
 * The library computes, for a template t and a batch of subtomograms f,
 * the rotation g maximising the zero-shift cross-correlation of Eq. (1),
 *     C(g) = int t(x) [R_g f](x) dx,   (R_g f)(x) = f(g^{-1} x),
 * through the ball-harmonic expansion (Sec. II-A) and the rotational
 * correlation of Eq. (2), maximised by frequency marching and gradient
 * ascent (Sec. II-C).
 *
 * Conventions (shared by every entry point)
 * -----------------------------------------
 * Volumes: N^3 FP32 samples on the cell-centred grid of [-1,1]^3,
 *   x_i = (i - (N-1)/2) * 2/N, vols[b][i][j][k] = f_b(x_i, y_j, z_k)
 *   (x slowest).  Only samples with |x| < 1 enter (the indicator of psi).
 * Basis (Sec. II-A): psi_klm = c_lk j_l(lambda_lk r) Y_l^m(theta, phi),
 *   lambda_lk the k-th zero of j_l, c_lk = sqrt(2)/|j_{l+1}(lambda_lk)|
 *   (L2-orthonormal on the ball), Y_l^m complex orthonormal with the
 *   Condon-Shortley phase.
 * Band L: the frequency-ordered prefix {(k,l,m) : lambda_lk < lambda_{L+1,1}}.
 * Coefficient layout: radial entries (l,k) in ascending lambda (ties by
 *   (l,k)), each followed by m = -l..l; C(L) complex coefficients, stored
 *   interleaved (re, im) as float[2*C], 8-byte aligned (the kernels read
 *   each (re, im) pair at once; a misaligned coefficient pointer is
 *   BH_EINVAL).  bh_index_table lists the order.
 * Coefficients: a_klm = h^3 sum_{|x_v|<1} conj(psi_klm(x_v)) f(x_v), h = 2/N
 *   (voxel quadrature of the L2 inner product).
 * Rotations: ZYZ Euler triples (alpha, beta, gamma), active,
 *   R = R_z(alpha) R_y(beta) R_z(gamma); FP64.
 * Cross-power (Eq. (2)): xi^l_{mn} = sum_{k in band} conj(b_klm) a_kln,
 *   b = template, a = particle; score C(g) = Re sum_l sum_{mn} xi^l_{mn}
 *   D^l_{mn}(g), D^l_{mn} = e^{-i m alpha} d^l_{mn}(beta) e^{-i n gamma},
 *   d^l(beta) = exp(-i beta J_y).
 *
 * Memory: every pointer named "dev" is device memory owned by the caller;
 * the library never frees caller memory.  A plan owns its basis matrix,
 * tables and scratch.  All device work is enqueued on the caller's HIP
 * stream (NULL = default stream) and is asynchronous; results are valid
 * after the stream is synchronised.  A plan must not be used from two
 * threads at once.
 *
 * Errors: every entry point returns BH_OK (0) or a negative code and sets a
 * thread-local message readable with bh_last_error().  No C++ exception
 * crosses this interface.  Kernel faults surface as BH_EDEVICE on a later
 * call or at stream synchronisation.
 */
#ifndef BH_H
#define BH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BH_OK = 0,
  BH_EINVAL = -1,        /* NULL pointer, size out of range, L > L_max   */
  BH_ENOMEM = -2,        /* device or host allocation failed             */
  BH_EDEVICE = -3,       /* HIP runtime error                            */
  BH_EUNSUPPORTED = -4   /* shape outside the supported range            */
};

#define BH_MAX_L 64      /* largest bandlimit of any plan                 */
#define BH_MAX_N 256     /* largest box edge of any plan                  */

typedef struct bh_plan bh_plan;

/* Last error message of the calling thread ("" if none). */
const char* bh_last_error(void);

/* ---------------------------------------------------------------------
 * Host-only tables (no GPU needed).  Sec. II-A: index set and zeros.
 * ------------------------------------------------------------------- */

/* C(L): number of complex coefficients of band L (all m); <0 on error. */
int64_t bh_index_size(int L);

/* Per-coefficient table of band L, host arrays of length C(L), any may be
 * NULL: degree l, radial index k (1-based), order m, and lambda_lk. */
int bh_index_table(int L, int32_t* l, int32_t* k, int32_t* m, double* lambda);

/* Number of radial entries (l,k) of band L; <0 on error. */
int bh_radial_count(int L);

/* Per-radial-entry table of band L in coefficient order, host arrays of
 * length bh_radial_count(L), any may be NULL: l, k, lambda_lk, c_lk. */
int bh_radial_table(int L, int32_t* l, int32_t* k, double* lambda, double* c);

/* Number of cell-centred voxels strictly inside the unit ball, N^3 grid. */
int64_t bh_ball_voxels(int N);

/* ---------------------------------------------------------------------
 * Plans
 * ------------------------------------------------------------------- */

/* Build the plan for box edge N (2..BH_MAX_N) and bandlimit L_max
 * (0..BH_MAX_L) on HIP device `device`: host tables, then the basis matrix
 * (h^3 conj(psi) at ball voxels, FP32, about 4*V_ball*C(L_max) bytes) on the
 * device.  Synchronous.  *out is NULL on error. */
int bh_plan_create(int N, int L_max, int device, bh_plan** out);

/* Release a plan and its device memory (NULL is accepted).  Synchronises
 * the device first. */
void bh_plan_destroy(bh_plan* p);

/* Complex coefficient count of the plan's band L (0 <= L <= L_max). */
int64_t bh_plan_num_coeffs(const bh_plan* p, int L);

/* Synchronise `stream`, then report errors that the plan's kernels found in
 * device-side arguments since the last report: BH_EINVAL if a particle's
 * template index (bh_align_t, bh_align_uneven) was outside the template
 * table or a volume row (bh_expand_rows) outside the volume stack, else
 * BH_OK.  Reporting clears the flag.  The flag lives in pinned
 * host memory that the kernels write, so bh_align_t and bh_align_uneven
 * also return it at entry (enqueuing nothing) once the offending call's
 * kernels have run. */
int bh_plan_check(bh_plan* p, void* stream);

/* ---------------------------------------------------------------------
 * Expansion (Sec. II-A): volumes -> coefficients of band L_max.
 * vols:   dev float[B][N][N][N]
 * coeffs: dev float[B][C(L_max)][2]
 * B >= 0 (B == 0 is a no-op).
 * ------------------------------------------------------------------- */
int bh_expand(bh_plan* p, const float* vols, int64_t B, float* coeffs, void* stream);

/* Expansion with a choice of arithmetic (same layouts as bh_expand):
 *  BH_EXPAND_FP32:   as bh_expand (FP32 MFMA, FP32 accumulation).
 *  BH_EXPAND_BF16:   basis and samples rounded to BF16, BF16 MFMA with FP32
 *                    accumulation; relative error ~2^-8 per term.
 *  BH_EXPAND_BF16X3: each FP32 value split as hi + lo (both BF16); the sum
 *                    of hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32
 *                    accumulation, close to FP32 accuracy.  If `coarse` is
 *                    not NULL (dev float[B][C(L_max)][2]) the hi*hi part
 *                    alone (the BF16 result) is written there as well.
 * The BF16 basis (2 bytes x V x C for hi and again for lo) is built on the
 * first BF16 call and kept by the plan.
 * Adding BH_EXPAND_BATCH_INVARIANT to the mode fixes the summation order of
 * each particle's coefficients independently of B (a particle expanded
 * alone or in any batch gives the same bits); otherwise the voxel sum is cut
 * into 1..16 slices (split-K) by a rule of the batch size, more for small
 * batches, so that the GEMM's workgroups fill the GPU. */
enum { BH_EXPAND_FP32 = 0, BH_EXPAND_BF16 = 1, BH_EXPAND_BF16X3 = 2,
       BH_EXPAND_BATCH_INVARIANT = 16 };
int bh_expand_ex(bh_plan* p, const float* vols, int64_t B, int mode, float* coeffs, float* coarse,
                 void* stream);

/* As bh_expand_ex, writing particle b's coefficients at coeffs + 2*b*ldc
 * (ldc >= C(L_max) complex entries; the rest of each row is left as is), so
 * particles of several plans can share one coefficient array. */
int bh_expand_into(bh_plan* p, const float* vols, int64_t B, int mode, float* coeffs, int64_t ldc,
                   float* coarse, void* stream);

/* Expansion (Sec. II-A) of volumes picked by row from a resident stack,
 * read in place: particle b is volume rows[b] of vols.
 * vols:   dev float[n_vols][N][N][N]
 * rows:   dev int64[B], 8-byte aligned, each in 0..n_vols-1 (repeats allowed)
 * coeffs, ldc, coarse, mode: as bh_expand_into (ldc == 0: C(L_max)).
 * The result for particle b is bit-identical to bh_expand_into on a copy
 * of vols[rows[b]] at position b (same mode, same B).  A row outside
 * 0..n_vols-1 is not read: that particle's coefficients have NaN real
 * parts (the imaginary parts of m = 0 coefficients stay 0) and the
 * plan's error word is raised, which bh_plan_check (and the next
 * bh_align_t or bh_align_uneven on the plan) reports as BH_EINVAL. */
int bh_expand_rows(bh_plan* p, const float* vols, int64_t n_vols, const int64_t* rows, int64_t B,
                   int mode, float* coeffs, int64_t ldc, float* coarse, void* stream);

/* ---------------------------------------------------------------------
 * Allocation-free expansion, for callers that cannot allocate device memory
 * during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same layouts as bh_expand; the result
 * is bit-identical to bh_expand_ex with BH_EXPAND_FP32 |
 * BH_EXPAND_BATCH_INVARIANT.
 *
 * Instead of the plan's growable scratch, the folded volumes and split-K
 * partial sums live in one static device array of BH_NOALLOC_SCRATCH_BYTES
 * per GPU, held by the library from its load until the process ends.  The
 * batch is processed in passes of bh_expand_noalloc_batch(p) particles (a
 * multiple of 128); a plan whose 128-particle pass does not fit (0 from
 * bh_expand_noalloc_batch, e.g. box edges far above 96 at L = 40) gets
 * BH_EUNSUPPORTED.  The call makes no hipMalloc, hipFree or other
 * allocating call; the caller passes the volumes and the coefficient
 * output.  All calls on one GPU share its scratch, so two calls that
 * overlap on the device (different streams, or different host threads)
 * race and give wrong results: serialise them.
 * ------------------------------------------------------------------- */
#define BH_NOALLOC_SCRATCH_BYTES (256ull << 20)
int bh_expand_noalloc(bh_plan* p, const float* vols, int64_t B, float* coeffs, void* stream);
/* Particles per pass of bh_expand_noalloc for this plan; <0 on error. */
int64_t bh_expand_noalloc_batch(const bh_plan* p);

/* ---------------------------------------------------------------------
 * Cross-power of Eq. (2) for band L (0 <= L <= L_max).
 * a:  dev float[B][C(L_max)][2]  particle coefficients
 * b:  dev float[C(L_max)][2]     template coefficients
 * xi: dev double[B][E(L)][2], E(L) = sum_{l<=L} (2l+1)^2; block l is
 *     row-major [m][n], m, n = -l..l, blocks in increasing l.
 * ------------------------------------------------------------------- */
int bh_cross_power(bh_plan* p, const float* a, const float* b, int64_t B, int L,
                   double* xi, void* stream);

/* ---------------------------------------------------------------------
 * Score and Euler gradient of Eq. (2) for band L at R rotations per
 * particle (Sec. II-B, II-C).
 * euler: dev double[B][R][3]
 * score: dev double[B][R]
 * grad:  dev double[B][R][3] (d/dalpha, d/dbeta, d/dgamma) or NULL
 * 1 <= R <= 1<<20.
 * ------------------------------------------------------------------- */
int bh_correlate(bh_plan* p, const float* a, const float* b, int64_t B, int L,
                 const double* euler, int R, double* score, double* grad, void* stream);

/* As bh_correlate, with the Hessian of the score in (alpha, beta, gamma)
 * (the closed-form derivatives of Sec. II-C taken twice: alpha brings
 * -i m, gamma -i n, beta d^l'' for d^l):
 * hess: dev double[B][R][6] = (aa, ab, ag, bb, bg, gg); grad may be NULL. */
int bh_correlate_hess(bh_plan* p, const float* a, const float* b, int64_t B, int L,
                      const double* euler, int R, double* score, double* grad, double* hess,
                      void* stream);

/* Candidate selection on its own (the rule of n_keep above), e.g. between
 * single-band calls: from every particle's P restarts (P <= 1024) keep K
 * (1 <= K <= min(64, P)) in the order taken.
 * euler: dev double[B][P][3], score: dev double[B][P];
 * euler_out: dev double[B][K][3], score_out: dev double[B][K]. */
int bh_prune_candidates(bh_plan* p, const double* euler, const double* score, int64_t B, int P,
                        int K, double min_sep, double* euler_out, double* score_out,
                        void* stream);

/* ---------------------------------------------------------------------
 * Degree energies of the band-L cross-power (Sec. II-C, energy ratio):
 * energy[b][l] = ||xi^l||_F^2 = sum_{m,n} |xi^l_{mn}|^2, l = 0..L.
 * The energy ratio Ratio(L') = sum_{l > L'} E_l / sum_l E_l is their tail
 * sum; bands for the march are chosen where it falls below thresholds.
 * energy: dev double[B][L+1].
 * ------------------------------------------------------------------- */
int bh_degree_energy(bh_plan* p, const float* a, const float* b, int64_t B, int L,
                     double* energy, void* stream);

/* ---------------------------------------------------------------------
 * Band selection by the energy ratio (Fig. 1 caption, Sec. III: the
 * bandlimits of the march are where the cross-power energy left out by a
 * truncation falls below thresholds).  For each particle b, against its
 * template (tmpl_idx as in bh_align_t), with E_l = ||xi^l||_F^2 of the
 * band-L_top cross-power:
 *   Ratio_b(L') = sum_{L' < l <= L_top} E_l / sum_{l <= L_top} E_l
 *   (0 where every E_l is 0; non-increasing in L', Ratio_b(L_top) = 0),
 *   bands[b][j] = the smallest L' with Ratio_b(L') <= thresholds[j].
 * For the batch, common[j] = the smallest L' with Ratio_b(L') <= tau_j for
 * at least ceil(B/2) particles, i.e. the lower median of bands[.][j].  A
 * march schedule is the distinct common[j] (above 0) in increasing order
 * followed by L_top.
 * thresholds: host double[n_tau], 1 <= n_tau <= 16, each in [0, 1]
 * bands:      dev int32[B][n_tau]
 * common:     dev int32[n_tau], or NULL
 * ratio:      dev double[B][L_top + 1], or NULL
 * A particle whose template index is outside the table gets NaN ratios and
 * L_top for every threshold; the error is reported as for bh_align_t.
 * ------------------------------------------------------------------- */
int bh_select_bands(bh_plan* p, const float* a, const float* templates, int n_templates,
                    const int32_t* tmpl_idx, int64_t B, int L_top, const double* thresholds,
                    int n_tau, int32_t* bands, int32_t* common, double* ratio, void* stream);

/* ---------------------------------------------------------------------
 * Alignment (Sec. II-C): frequency marching over `bands` with multi-start
 * gradient ascent.  For each band L_b (each <= L_max, any order): evaluate
 * (S, grad S) at the carried point x; step eta = step_init / W_b with
 * W_b = sum_{l<=L_b} l(l+1) ||a_l|| ||b_l|| over the band (0 if W_b = 0);
 * then `steps_per_band` times: x' = wrap(x + eta * G^{-1}(x) grad S(x)),
 * G the SO(3) metric in ZYZ coordinates with sin^2(beta) floored at 1e-6;
 * accept x' if S(x') >= S(x) (eta *= step_grow) else eta *= step_shrink.
 * wrap: beta into [0, pi] via R(a, b, g) = R(a + pi, 2pi - b, g + pi),
 * alpha and gamma into [-pi, pi).  The best restart (highest final score,
 * lowest index on ties) is returned.
 * starts:    dev double[B][n_restarts][3]   starting Euler triples
 * euler_out: dev double[B][3]
 * score_out: dev double[B]
 * all_euler: dev double[B][n_restarts][3] final point of every restart, or NULL
 * all_score: dev double[B][n_restarts] its score, or NULL
 * ------------------------------------------------------------------- */
typedef struct {
  const int32_t* bands;     /* host array of n_bands bandlimits           */
  int32_t n_bands;          /* 1..16                                      */
  int32_t steps_per_band;   /* 0..10000                                   */
  int32_t n_restarts;       /* 1..65536                                   */
  double step_init;         /* > 0                                        */
  double step_grow;         /* > 0                                        */
  double step_shrink;       /* > 0                                        */
  int32_t batch_invariant;  /* nonzero: a particle's results do not depend
                               on the other particles of the call (fixed
                               work split); 0: the split may widen for
                               small batches (lower latency, summation
                               order then depends on the batch size)      */
  int32_t newton_bands;     /* 0..n_bands: the last newton_bands bands take
                               Newton steps (below) instead               */
  int32_t newton_steps;     /* steps of a Newton band (0: steps_per_band)  */
  int32_t n_keep;           /* 0: every restart runs every band; 1..64
                               (< n_restarts <= 1024): after the first band
                               only n_keep candidates continue (below)    */
  double keep_min_sep;      /* radians in [0, pi]: candidates closer than
                               this count as the same local maximum       */
} bh_align_opts;

/* Newton bands (Sec. II-C, III): evaluate S, grad S and the Hessian H at the
 * carried point; mu = 1; then per step: d = (-H)^{-1} grad S if -H is
 * positive definite (all leading principal minors > 0), else
 * eta0 g^{-1} grad S with eta0 = step_init / W_b; d scaled to a largest
 * component of at most 0.5 rad; x' = wrap(x + mu d); accept if
 * S(x') >= S(x) (mu = min(1, mu * step_grow)) else mu *= step_shrink.
 *
 * Candidates (Sec. III: local maxima of the lowest band): after the first
 * band the restarts are visited by decreasing score (lowest index first on
 * ties) and one is kept if its rotation is farther than keep_min_sep from
 * every one kept so far, until n_keep are kept; if fewer are that far
 * apart, the rest are filled with the skipped restarts in the same order.
 * The later bands run the n_keep candidates only; all_euler / all_score
 * then hold n_keep entries per particle: [B][n_keep][3], [B][n_keep]. */

int bh_align(bh_plan* p, const float* a, const float* b, int64_t B,
             const bh_align_opts* opts, const double* starts,
             double* euler_out, double* score_out,
             double* all_euler, double* all_score, void* stream);

/* As bh_align, against one of several templates per particle:
 * templates: dev float[n_templates][C(L_max)][2]
 * tmpl_idx:  dev int32[B], template of each particle, in 0..n_templates-1;
 *            may be NULL if n_templates == 1.  The indices are device data,
 *            so they are checked by the kernels: a particle with an index
 *            outside the table gets a NaN score (its rotation is not
 *            meaningful), no memory outside the table is read, and the
 *            error is reported as BH_EINVAL by bh_plan_check or by a later
 *            bh_align_t / bh_align_uneven call on the plan.
 * A call with one band and all_euler set advances every restart by one band
 * of the march; its all_euler output is the next call's starts. */
int bh_align_t(bh_plan* p, const float* a, const float* templates, int n_templates,
               const int32_t* tmpl_idx, int64_t B, const bh_align_opts* opts,
               const double* starts, double* euler_out, double* score_out,
               double* all_euler, double* all_score, void* stream);

/* ---------------------------------------------------------------------
 * Uneven batches: particles of different bandlimits (box sizes) marched
 * together, one launch per band for every particle that takes it.
 * Band indices are a frequency-ordered prefix, so coefficients of any plan
 * share the layout of band L; the particle rows (and template rows) are
 * laid out with a common complex stride lda (ldt) >= C(largest band used).
 * Lp:       host int32[B], each particle's bandlimit, non-increasing along
 *           the batch (sort by bandlimit first); particle b takes every band
 *           of opts->bands (strictly increasing) that is <= Lp[b], and all
 *           take the first one.
 * Otherwise as bh_align_t; the band tables come from plan p (L_max >= the
 * largest band taken).  Newton bands count from the end of opts->bands.
 * ------------------------------------------------------------------- */
int bh_align_uneven(bh_plan* p, const float* a, int64_t lda, const int32_t* Lp,
                    const float* templates, int64_t ldt, int n_templates, const int32_t* tmpl_idx,
                    int64_t B, const bh_align_opts* opts, const double* starts,
                    double* euler_out, double* score_out, double* all_euler, double* all_score,
                    void* stream);

/* ---------------------------------------------------------------------
 * Shift search (Sec. II-C: Eq. (2) maximised for each shift of a grid,
 * then the best shift kept).  For each particle b and each integer voxel
 * shift s = (dx, dy, dz) of the table, the shifted volume
 *   f_s[i][j][k] = f_b[i + dx][j + dy][k + dz]   (0 outside the box),
 * i.e. f_s(x) = f(x + s h), is expanded (FP32, as bh_expand) and aligned
 * with `opts` from the particle's starts; the shift with the highest final
 * score wins (lowest table index on ties).
 * vols:      dev float[B][N][N][N]
 * shifts:    host int32[S][3], 1 <= S <= 125, |d| <= N (read during the call)
 * b:         dev float[C(L_max)][2] template coefficients
 * starts:    dev double[B][n_restarts][3] (used for every shift)
 * euler_out: dev double[B][3], score_out: dev double[B],
 * shift_out: dev int32[B] index into `shifts`.
 * Device scratch grows to about B*S*(8 C + 24 n_restarts) bytes plus the
 * expansion and march buffers of B*S particles.
 * ------------------------------------------------------------------- */
int bh_align_shifts(bh_plan* p, const float* vols, int64_t B, const int32_t* shifts, int S,
                    const float* b, const bh_align_opts* opts, const double* starts,
                    double* euler_out, double* score_out, int32_t* shift_out, void* stream);

/* ---------------------------------------------------------------------
 * Autotuning: launch shapes chosen by timing on this GPU.
 * bh_plan_autotune times, on random data of B particles (synchronously, on
 * `stream`), the candidate shapes and keeps the fastest in the plan:
 *  BH_TUNE_MARCH:       waves per workgroup of the ascent kernel
 *                       (4, 5, 6, 8, 10, 12, 16) for each band of `bands`,
 *                       n_restarts restarts, 2 ascent steps per trial, then
 *                       whether persistent workgroups (only as many as are
 *                       resident, looping over the particles) are faster;
 *  BH_TUNE_EXPAND:      split-K factor (1..16) of the FP32 expansion GEMM for
 *                       B particles' tile count;
 *  BH_TUNE_EXPAND_BF16: the same for the split-BF16 GEMM.
 * Later calls use the tuned choices (the tuned wave count depends on the
 * band only, so batch-invariant calls use it too; batch-invariant expansions
 * keep their fixed split).  bh_plan_tuning reports, for band L and batch
 * size B, the tuned wave count (0: built-in rule), whether its launches are
 * persistent, and the split-K factors the expansions would use.
 * ------------------------------------------------------------------- */
enum { BH_TUNE_MARCH = 1, BH_TUNE_EXPAND = 2, BH_TUNE_EXPAND_BF16 = 4 };
int bh_plan_autotune(bh_plan* p, int64_t B, int n_restarts, const int32_t* bands, int n_bands,
                     int what, void* stream);
int bh_plan_tuning(const bh_plan* p, int L, int64_t B, int* waves, int* persistent,
                   int* split_f32, int* split_bf16);
/* Pin the ascent kernel's shape for band L (e.g. from a saved tuning run):
 * waves 0 (built-in rule) or one of 4, 5, 6, 8, 10, 12, 16 (at most 2L+1
 * unless 4); persistent 0/1. */
int bh_plan_set_tuning(bh_plan* p, int L, int waves, int persistent);

/* ---------------------------------------------------------------------
 * Per-kernel timing (for measurement; off by default).
 * bh_profile_enable(p, 1) synchronises the device, clears earlier records
 * and starts recording a pair of HIP events on the call's stream around
 * every kernel launch of this plan; bh_profile_enable(p, 0) stops.
 * bh_profile_read waits for the recorded events whose kernel name equals
 * `name` (or starts with it when `name` ends in '*') and returns their
 * number, summed duration in milliseconds and summed work units (kernel
 * specific: particles x evaluations x class entries for the score kernels,
 * particles for the expansion).  Kernel names: "gather", "gemm", "reduce",
 * "xi_classes", "band_weight", "march_L<L>", "select", "correlate_L<L>",
 * "xi_dense".  Outputs may be NULL.
 * ------------------------------------------------------------------- */
int bh_profile_enable(bh_plan* p, int enable);
int bh_profile_read(bh_plan* p, const char* name, int64_t* launches, double* total_ms,
                    int64_t* work);
/* Wall time in milliseconds during which at least one recorded launch whose
 * kernel name matches `name` (as bh_profile_read) was running: the union of
 * their [start, stop] intervals, on whichever streams they ran (a march
 * split over two streams overlaps its launches). */
int bh_profile_busy(bh_plan* p, const char* name, double* busy_ms);

/* Split eligible marches (bh_align, bh_align_t with the plain gradient
 * march, at least 512 particles of 64 restarts, no graph capture) into two
 * halves marched on two streams: streams 2 (the default) or 1 (never).
 * Results are the same bits either way. */
int bh_plan_set_march_streams(bh_plan* p, int streams);

/* ---------------------------------------------------------------------
 * Reference kernels for hardware traffic counters (measurement only): a
 * counter's reading for a kernel that moves a known number of bytes in the
 * same way scales the counter's readings for the library's kernels.
 *  BH_CALIB_COPY_VECTOR: copy `bytes` (a multiple of 16) from src to dst,
 *      16 bytes per lane per load and store (dev buffers of `bytes`);
 *  BH_CALIB_READ_SCALAR: read `bytes` (a multiple of 64) of src in
 *      wave-uniform 64-byte loads through the scalar cache, as the ascent
 *      kernel reads its class weights; dst (dev double[BH_CALIB_READ_GROUPS])
 *      receives one sum per workgroup.
 * Asynchronous on `stream`.
 * ------------------------------------------------------------------- */
enum { BH_CALIB_COPY_VECTOR = 0, BH_CALIB_READ_SCALAR = 1 };
#define BH_CALIB_READ_GROUPS 2048
int bh_calib_copy(void* dst, const void* src, int64_t bytes, int mode, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BH_H */
