/*
 * pam.h - C-ABI of the MI355X (gfx950) AS-TAX passive-acoustic-mapping library.
 *
 * The library reconstructs passive acoustic maps from channel RF with the
 * cross-correlated angular-spectrum method with triple apodization (AS-TAX):
 *   1. Fourier transform of every channel over time, keeping the bins of the
 *      selected frequency set Omega (Eq. 1, F_t; Omega of Eq. 3);
 *   2. per bin, the lateral Fourier transform of each apodized sub-aperture
 *      (Eq. 1, F_x; Pattern-m apodization of Sections II-A and II-C);
 *   3. the angular-spectrum propagator exp(i z sqrt(w^2/c^2 - kx^2)) at every
 *      depth of the image grid (Eq. 2);
 *   4. the inverse lateral transform giving the monochromatic fields p_i(r, w);
 *   5. the sums over w of the sub-aperture cross-spectra, giving the NCCs
 *      rho_12, rho_23, rho_31 (Eq. 4, negative frequencies as conjugates per
 *      Appendix A) and the energy sum_w |p_1 + p_2 + p_3|^2;
 *   6. the TAX weight (rho_12 rho_23 rho_31)^(1/3) (Eq. 10) with every pair
 *      floored at eps (text after Eq. 4), normalised to maximum 1 (NNCC), and
 *      the image I = rho_n^2 * sum_w |p_1 + p_2 + p_3|^2 (Eq. 11).
 * With n_sub = 2 the same path computes AS-DAX (Eq. 5) and with n_sub = 1
 * plain AS (Eq. 3, weight 1).
 *
 * Conventions
 *   Units are SI.  Geometry: a linear array on the plane z = 0 whose centre is
 *   the lateral origin (Fig. 1).  The forward time transform uses exp(-i w t),
 *   the lateral transforms exp(-i kx x) forward and exp(+i kx x)/N_x inverse,
 *   and the propagator exp(+i z kz) with the principal square root (evanescent
 *   components decay as exp(-z sqrt(kx^2 - k^2)) unless PAM_EVAN_ZERO).
 *   Bins: 0 < k < n_t/2 with lo <= k fs / n_t <= hi for some closed band.
 *   Energies use the positive bins only, with no 1/n_t factor.
 *
 * Ownership and errors
 *   The caller owns every buffer passed in; a plan owns only its resident
 *   device tables.  pam_as_tax never allocates device memory: all scratch
 *   space is the caller's workspace.  Every argument is validated before any
 *   work is enqueued; on error nothing is enqueued and no output is written.
 *   Device faults surface at the caller's next synchronisation of the stream.  A
 *   PAM_ERR_DEVICE from a launch after validation (a HIP runtime failure) can leave the
 *   earlier stages of that call enqueued; their results are then incomplete and the
 *   outputs must not be used.
 *   A plan is immutable after creation: concurrent pam_as_tax calls on one
 *   plan are safe when they use different streams and different workspaces.
 */
#ifndef PAM_H
#define PAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pam_plan_s* pam_plan_t;

typedef enum {
  PAM_OK = 0,
  PAM_ERR_INVALID_ARG = -1, /* a parameter is out of range, null or not finite */
  PAM_ERR_OOM = -2,         /* device or host allocation failed (pam_plan only) */
  PAM_ERR_DEVICE = -3,      /* a HIP runtime call or kernel launch failed */
  PAM_ERR_UNSUPPORTED = -4, /* valid but outside what the kernels handle (sizes) */
  PAM_ERR_WORKSPACE = -5    /* workspace null or smaller than pam_workspace_size */
} pam_status_t;

/* How the L physical channels are laid on the N_x-column lateral grid. */
typedef enum {
  PAM_LATERAL_PAD = 0,  /* column o + l, o = floor((N_x - L)/2), spacing = pitch          */
  PAM_LATERAL_STUFF = 1 /* column s*l, s = N_x / L integer, spacing = pitch / s;
                           the zero channels in between are the paper's 2x zero-stuffing
                           (Section II-E), apodization indexed on physical elements     */
} pam_lateral_t;

/* Arithmetic of the inverse lateral transform (the dominant contraction).  The
 * propagator phase z*kz and its reduction modulo 2 pi are FP64 in every mode,
 * the sine/cosine FP32; all accumulations are FP32; NCC denominators FP64. */
typedef enum {
  PAM_PREC_FP32 = 0,       /* FP32 operands, FP32 matrix-core products                */
  PAM_PREC_SPLIT_BF16 = 1, /* operands split hi+lo in BF16, three BF16 products       */
  PAM_PREC_SPLIT_FP16 = 2, /* operands split hi+lo in FP16 (power-of-two pre-scaled)  */
  PAM_PREC_BF16 = 3,       /* single BF16 product                                     */
  PAM_PREC_FP16 = 4        /* single FP16 product (pre-scaled)                        */
} pam_precision_t;

typedef enum {
  PAM_EVAN_DECAY = 0, /* literal Eq. 2 with the principal root: evanescent terms decay */
  PAM_EVAN_ZERO = 1   /* evanescent lateral wavenumbers dropped                        */
} pam_evanescent_t;

/* Imaging set-up (the paper's problem statement: RF on the array plane, element
 * pitch and sampling rate of Section II-D, sound speed of Eq. 2, frequency set
 * of Section II-E, image grid, apodization set of Sections II-A/II-C, eps of
 * the text after Eq. 4).  Arrays are host memory, read during pam_plan only. */
typedef struct {
  int32_t n_elements;        /* L >= 1 physical channels                                  */
  double pitch_m;            /* element pitch > 0                                         */
  double fs_hz;              /* sampling rate > 0                                         */
  double c_mps;              /* sound speed > 0                                           */
  int32_t n_samples;         /* largest record length n_t served: power of two, 32..16384 */
  int32_t n_bands;           /* >= 1 closed bands making up Omega                         */
  const double* band_lo_hz;  /* [n_bands]                                                 */
  const double* band_hi_hz;  /* [n_bands], lo <= hi                                       */
  int32_t n_depths;          /* n_z >= 1                                                  */
  const double* depths_m;    /* [n_z], finite, >= 0, measured from the array plane        */
  int32_t n_x;               /* N_x lateral columns: multiple of 32, >= L, <= 512         */
  pam_lateral_t lateral;
  int32_t n_sub;             /* 1 (AS), 2 (AS-DAX) or 3 (AS-TAX)                          */
  const uint8_t* apod;       /* [n_sub][L] masks in {0,1}, or NULL for Pattern-m          */
  int32_t pattern_m;         /* m of Pattern-m when apod is NULL (0 means 16)             */
  double eps;                /* NCC floor, 0 < eps < 1 (0 means 1e-3)                     */
  pam_precision_t precision;
  pam_evanescent_t evanescent;
  int32_t coherence;         /* 1: also accumulate adjacent-pixel cross-spectra (see below);
                                needs n_sub = 1, n_x = 256 and an even n_depths; else 0       */
} pam_geometry_t;

/* Sizes a plan settles on, for callers that size their own buffers. */
typedef struct {
  int32_t n_bins;      /* bins of Omega on the plan's n_samples grid                        */
  int32_t n_z, n_x, n_sub, n_elements, n_samples, n_pairs;
  int32_t device;
} pam_plan_info_t;

/* Where each stage's result lies inside a workspace (byte offsets), for callers
 * that check intermediate results.  Layouts (all row-major, last index fastest):
 *   spectra  complex64 [F][n_sel][L]          time-transform bins, Omega order
 *   coeffs   complex64 [F][n_sel][n_sub][N_x] lateral coefficients: at N_x = 256 and 512
 *            (and 128 with FP32 operands) the spectrum P_i(q)/N_x stored at r*16 + q1 for
 *            q = (N_x/16) q1 + r (factored transform), otherwise folded into cos/sin slot
 *            order; scaled by a power of two for FP16 operands (scale 1 otherwise)
 *   scales   float32   [F][n_sel]             1 / (power-of-two scale of coeffs)
 *   accum    float32   [n_split][F][n_acc][n_z][N_x] partial sums over disjoint bin
 *            ranges (the region reserves room beyond n_split F planes); channels S_1..S_nsub then C_12, C_23, C_31 (n_sub = 3) or C_12;
 *            with coherence (n_sub = 1): S, then Re and Im of the lateral pair sum
 *            G_x(z, x) = sum_w p(z, x) conj(p(z, x ^ 1)) and of the axial pair sum
 *            G_z(z, x) = sum_w p(z, x) conj(p(z ^ 1, x)) (pairs of adjacent columns 2j, 2j+1
 *            and of adjacent depths 2i, 2i+1), n_acc = 5
 *   energy   float32   [F][n_z][N_x]          sum_w |sum_i p_i|^2
 *   weight   float32   [F][n_z][N_x]          weight before normalisation
 * n_sel is the number of plan bins on the call's record-length grid. */
typedef struct {
  size_t spectra, coeffs, scales, accum, energy, weight, blockmax, total;
  int32_t n_sel, n_split, n_acc;
} pam_workspace_layout_t;

/* Build a plan on HIP device `device`: validates g, builds the FP64 frequency,
 * wavenumber and depth tables, masks, lateral placement and transform tables,
 * and copies them to the device (the paper's pre-run, Section II-E).
 * On error *out is set to NULL and nothing is leaked. */
pam_status_t pam_plan(const pam_geometry_t* g, int device, pam_plan_t* out);

pam_status_t pam_plan_get_info(pam_plan_t p, pam_plan_info_t* info);

/* Copy the plan's bin indices k (on its n_samples grid) into host array bins[n_bins]. */
pam_status_t pam_plan_get_bins(pam_plan_t p, int32_t* bins, int32_t capacity);

/* Workspace bytes and stage layout for n_frames frames of n_t samples each.
 * n_t must be n_samples / 2^j (j >= 0) and >= 32; such a record uses the plan
 * bins whose frequency lies on its own grid (every 2^j-th bin k).  The size never
 * shrinks as n_frames or n_t grows, so a workspace sized for n frames of n_t samples
 * serves every call of at most n frames of at most n_t samples.  The fields stage
 * splits each frame's bins into n_split ranges (chosen per call from the frames, the
 * bins and how many fields workgroups the device holds at once); the accum region
 * reserves n_frames plus a fixed number of spare planes, enough for any split the
 * library picks. */
pam_status_t pam_workspace_size(pam_plan_t p, int64_t n_frames, int32_t n_t, size_t* bytes);
pam_status_t pam_workspace_layout(pam_plan_t p, int64_t n_frames, int32_t n_t,
                                  pam_workspace_layout_t* layout);

/* Reconstruct n_frames frames (asynchronous on hip_stream; NULL = default stream).
 *   rf        device float32 [n_frames][L][n_t], time fastest               (in)
 *   image     device float32 [n_frames][n_z][N_x], I of Eq. 11              (out, required)
 *   nncc      device float32 [n_frames][n_z][N_x], rho_n, or NULL           (out)
 *   rho_pairs device float32 [n_frames][n_pairs][n_z][N_x], NCC of each pair
 *             (12, 23, 31) before the eps floor, or NULL                    (out)
 *   workspace device scratch of at least pam_workspace_size bytes, 256-byte aligned
 * n_frames may be 0 (nothing is enqueued). */
pam_status_t pam_as_tax(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t,
                        float* image, float* nncc, float* rho_pairs,
                        void* workspace, size_t ws_bytes, void* hip_stream);

/* Number of HIP events pam_as_tax_events records: before K1 (time FFT), after K1,
 * after K2 (lateral transform), after K3 (fields and cross-spectra), after K4
 * (weight, NNCC and image). */
#define PAM_N_STAGE_EVENTS 5

/* pam_as_tax that also records the caller's HIP events (hipEvent_t handles created
 * by the caller with timing enabled, array of PAM_N_STAGE_EVENTS) on hip_stream at
 * the stage boundaries, so a caller can time each kernel on the stream it runs on.
 * Same arguments, validation and results as pam_as_tax; events may not be NULL. */
pam_status_t pam_as_tax_events(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t,
                               float* image, float* nncc, float* rho_pairs,
                               void* workspace, size_t ws_bytes, void* hip_stream,
                               void* const* events);

/* The comparison beamformer of the paper's appendix on the same plan, inputs and
 * outputs: frequency-domain delay-and-sum (FD-TEA) fields
 *   p_i(r, w) = sum_l a_i[l] F_t{s_l}(w) exp(+i w tau_l(r)),  tau_l(r) = |r - r_l| / c
 * (Appendix "PAM with DAX and TAX", the frequency-domain form of Eq. 6 with unit
 * distance weights; r_l the element positions on z = 0, r the plan's image grid),
 * followed by the same cross-spectra sums, NCC, TAX weight (n_sub = 3; DAX for 2,
 * plain FD-TEA for 1), NNCC and image as pam_as_tax (Eq. 4, Eq. 10, Eq. 11).
 * Same arguments, layouts, workspace size, validation and errors as pam_as_tax; the
 * plan's lateral transform tables and precision are not used (FP32 arithmetic, FP64
 * travel-time phases). */
pam_status_t pam_fd_tea_tax(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t,
                            float* image, float* nncc, float* rho_pairs,
                            void* workspace, size_t ws_bytes, void* hip_stream);

/* Bytes of the library's built-in device scratch used by pam_as_tax_noalloc (128 MiB:
 * one frame of 128 elements x 4096 samples x 768 bins on a 512 x 256 grid needs about
 * 110 MB, most of it the partial-sum planes of the bin split). */
#define PAM_NOALLOC_SCRATCH_BYTES (128u << 20)

/* pam_as_tax without a caller workspace and without any allocation, for callers that
 * cannot allocate device memory (work captured into a HIP graph, tight serving loops,
 * harnesses that forbid allocation).  Same arguments (minus the workspace), validation
 * and results as pam_as_tax; the intermediate results live in a device array of
 * PAM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends.
 *   Errors: PAM_ERR_WORKSPACE when the call needs more scratch than
 *   PAM_NOALLOC_SCRATCH_BYTES (pam_workspace_size gives the need; split the frames
 *   into smaller calls); otherwise as pam_as_tax.
 *   Concurrency: every call on one GPU shares that GPU's scratch, which keeps the last
 *   call's contents; calls that overlap on one GPU (other streams, other threads) race
 *   and must be serialised by the caller.  No stage needs the scratch cleared: every
 *   value a kernel reads was written earlier in the same call. */
pam_status_t pam_as_tax_noalloc(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t,
                                float* image, float* nncc, float* rho_pairs, void* hip_stream);

/* Frames of different record lengths in one call (the ragged batches of Section II-E's
 * record lengths: every record on its own time-frequency grid, all on one plan).
 * groups[g] = {n_t, n_frames}: group g holds n_frames records of n_t samples (each n_t one
 * of the plan's record lengths, as for pam_as_tax; 1 <= n_groups <= 8, at most 65535 frames
 * in all).  rf (device) holds the groups back to back, group g as
 * [n_frames][L][n_t] after the groups before it; image, nncc (and rho_pairs) hold the
 * frames in the same order.  Stages K1, K2 and K4 run per group.  On the factored fields
 * kernels (N_x = 256 or 512, and 128 with FP32 operands) the fields stage runs as one launch
 * over all groups (a grouped work list, one bin split for the call) when the library's cost
 * estimate of that launch is below the sum of the groups' own launches; otherwise, and on
 * the other kernels, it runs per group with each group's own split.  The workspace
 * (pam_workspace_size_grouped bytes, 256-byte aligned) holds the groups' workspaces back to
 * back, each laid out as pam_workspace_layout would for that group and split; it serves any
 * group list whose groups, position by position, have no more frames and no longer
 * records.  Results equal pam_as_tax on each group up to FP32 summation order (the bin split
 * depends on the frames of the call).  Errors as pam_as_tax; PAM_ERR_INVALID_ARG for a bad
 * group list. */
typedef struct {
  int32_t n_t;       /* record length of the group's frames */
  int64_t n_frames;  /* frames in the group (may be 0) */
} pam_group_t;
pam_status_t pam_workspace_size_grouped(pam_plan_t p, const pam_group_t* groups, int32_t n_groups, size_t* bytes);
pam_status_t pam_as_tax_grouped(pam_plan_t p, const float* rf, const pam_group_t* groups, int32_t n_groups,
                                float* image, float* nncc, float* rho_pairs, void* workspace, size_t ws_bytes,
                                void* hip_stream);

/* Release the plan's device tables.  NULL-safe; no work may be in flight. */
void pam_destroy(pam_plan_t p);

const char* pam_status_string(pam_status_t s);

/* Test hooks for the error paths (callers: test suites).
 * pam_debug_fail_allocation(n): the n-th next device allocation made while building a
 *   plan (n = 0: the next one) fails as if the device were out of memory, so pam_plan
 *   returns PAM_ERR_OOM after releasing what it had allocated; n < 0 disarms.  One
 *   injected failure per call; not meant for use beside concurrent pam_plan calls.
 * pam_debug_live_allocations(): the number of device allocations held by all live plans
 *   of the process (a leak check: unchanged across a failed pam_plan).
 * pam_debug_grouped_one_launch(p, groups, n_groups): 1 if pam_as_tax_grouped with this
 *   group list runs the fields stage as one grouped launch, 0 if per group, or a negative
 *   pam_status_t for a bad plan or group list (so tests can cover both schedules). */
void pam_debug_fail_allocation(int32_t n);
int64_t pam_debug_live_allocations(void);
int32_t pam_debug_grouped_one_launch(pam_plan_t p, const pam_group_t* groups, int32_t n_groups);

#ifdef __cplusplus
}
#endif
#endif /* PAM_H */
