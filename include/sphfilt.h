/*
 * sphfilt.h -- C-ABI of the double FFT filter for spherical grids on MI355X.
 *
 * The operation (arXiv:2305.01537, Sec. II.A "Filtering algorithms"):
 *
 *   Every evolved field X(x1, theta, phi) is filtered first along theta, then
 *   along phi.
 *   Theta-pass: theta is extended across the poles to a 2pi-periodic line by
 *     pairing meridian phi with meridian phi + pi under the field's axis
 *     parity sign (-1)^a (the extension equation), the line is transformed,
 *     mode l is multiplied by f(|l|, l_max) and the result transformed back
 *     and written to both meridians.
 *   Phi-pass: every ring (x1, theta_j) is transformed along phi, mode m is
 *     multiplied by f(|m|, m_max) and transformed back.
 *   Cutoffs (the l_max / m_max equations):
 *     l_max = max(floor, 2 (r/dr_min) L),
 *     m_max = max(floor, 2 (r/dr_min) sin(theta_j) L), floor = 2 in the paper.
 *   Filter kinds: exponential (eq. exp_filter), Gaussian (eq. gaussian_filter)
 *     and the spectrally sharp low-pass mentioned beside them.
 *
 * Grid and layout, fixed by this library:
 *   fields are FP64, contiguous, C order [n_fields][n_r][n_theta][n_phi]
 *   (phi fastest); theta_j = (j + 1/2) pi / n_theta (cell centred, no point on
 *   a pole), phi_k = 2 pi k / n_phi; n_phi must be even.  The extended half of
 *   a theta line maps row n (n >= n_theta) to row 2 n_theta - 1 - n of
 *   meridian k + n_phi/2.  sin(theta_j) is evaluated at the mirror-symmetric
 *   colatitude (min(j, n_theta-1-j) + 1/2) pi / n_theta.
 *
 * The forward filter is F = Phi o Theta.  Each pass is a real symmetric
 * linear operator, so the adjoint (transpose) is F^T = Theta o Phi.
 *
 * Errors: every entry point returns an int status (SPHFILT_OK or a negative
 * SPHFILT_E* code); nothing is thrown across the ABI.  Arguments are
 * validated on the host before any device call.  Device entry points only
 * enqueue work on the given HIP stream and return; the caller synchronises.
 *
 * Supported sizes: 2*n_theta and n_phi each in
 * {32, 48, 64, 80, 96, 128, 160, 192, 256} (48, 96 and 192 are transformed
 * with a radix-3 stage, 80 and 160 with a radix-5 stage).  Other sizes
 * return SPHFILT_EUNSUPPORTED.
 */
#ifndef SPHFILT_H
#define SPHFILT_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SPHFILT_OK            0
#define SPHFILT_EINVAL       (-1)  /* bad argument (shape, pointer, parity, cutoff) */
#define SPHFILT_ENOMEM       (-2)  /* host or device allocation failed            */
#define SPHFILT_EDEVICE      (-3)  /* HIP runtime or kernel launch error          */
#define SPHFILT_EUNSUPPORTED (-4)  /* valid for the method, not built here (size) */

/* ---- filter kinds (Sec. II.A) ----------------------------------------- */
#define SPHFILT_EXP   0   /* f = 1 for |l| <= c, exp(-(|l| - c)) above        (eq. exp_filter)      */
#define SPHFILT_GAUSS 1   /* f = exp(log(0.9) (|l| / (c + 1))^2)               (eq. gaussian_filter) */
#define SPHFILT_SHARP 2   /* f = 1 for |l| <= c, 0 above (sharp low-pass named beside eq. exp_filter) */
#define SPHFILT_HYBRID 3  /* per line: GAUSS if Jameson's detector fires, else EXP (the automatic
                             switch at the end of Sec. II.A); see sphfilt_cutoff and sphfilt_apply_ex */

typedef struct sphfilt_plan_s  *sphfilt_plan;   /* opaque; immutable after create */
typedef struct sphfilt_batch_s *sphfilt_batch;  /* opaque; see sphfilt_batch_create */

/*
 * Cutoff parameters (Sec. II.A, l_max / m_max equations).
 *   rho          [n_r] r_i / dr_min, each finite and > 0 (r is the physical
 *                radius, e.g. after a fisheye map).  NULL => uniform
 *                cell-centred grid rho_i = i + 1/2.
 *   L            [n_fields] the cutoff scale cal-L, each finite and > 0
 *                (the paper uses 3 for metric fields and 12 for matter).
 *   kind         [n_fields] SPHFILT_EXP / GAUSS / SHARP / HYBRID, or NULL =>
 *                all EXP.
 *   floor_modes  finite, >= 0: the lowest cutoff; 2 in the paper.
 *   detector_eps, detector_threshold
 *                Jameson's detector of the hybrid kind: a line (an extended
 *                theta line or a phi ring, periodic) takes the Gaussian
 *                filter if some cell has
 *                |u_{i-1} - 2u_i + u_{i+1}| / (|u_{i-1}| + 2|u_i| + |u_{i+1}| + eps)
 *                >= threshold.  0 selects the defaults eps = 1e-12 and
 *                threshold = 0.95 (the paper's); otherwise finite, eps >= 0,
 *                threshold > 0.  Unused unless some field is HYBRID.
 * The arrays are read during the call only; the plan keeps its own copy.
 */
typedef struct {
    const double *rho;
    const double *L;
    const int    *kind;
    double        floor_modes;
    double        detector_eps;
    double        detector_threshold;
} sphfilt_cutoff;

/*
 * Work and traffic figures of one plan, computed on the host.
 *   theta_shells_active  shells (field, r) whose theta mask is not all ones
 *   theta_lines_*        extended theta lines (one per meridian pair)
 *   phi_rings_*          phi rings
 *   bytes_*              algorithmic HBM bytes of one call: 8 B read + 8 B
 *                        written per point of every line a pass must touch.
 *                        In place, identity lines are skipped; out of place,
 *                        the first pass also copies its identity lines.
 *   shells_fused         shells a plan sends through the fused shell kernel
 *                        (see sphfilt_plan_set_fused); 0 if the grid does not
 *                        allow it
 *   bytes_fused_inplace  algorithmic bytes of one in-place call (forward or
 *                        adjoint) with those shells fused: 16 B per point of a
 *                        fused shell, plus the two-pass figure of the rest
 */
typedef struct {
    long long n_points;
    long long theta_shells_total, theta_shells_active;
    long long theta_lines_total, theta_lines_active;
    long long phi_rings_total, phi_rings_active;
    long long bytes_forward_inplace, bytes_forward_outofplace;
    long long bytes_adjoint_inplace, bytes_adjoint_outofplace;
    long long shells_fused, bytes_fused_inplace;
} sphfilt_stats;

/*
 * Create a plan for n_fields fields on an n_r x n_theta x n_phi grid.
 *   out     receives the plan handle (set to NULL on error).
 *   parity  [n_fields] axis parity sign (-1)^a of each field, +1 or -1
 *           (Sec. II.A, the extension equation).
 *   cut     cutoff parameters, see sphfilt_cutoff.
 * Builds the cutoff tables, the lists of non-identity lines and the twiddle
 * tables on the host, then allocates and uploads them to the current HIP
 * device (and, where overlap can apply, creates the plan's second stream; see
 * sphfilt_plan_set_overlap).  The plan owns that device memory until
 * sphfilt_plan_destroy and keeps no scratch, so one plan may be applied
 * concurrently on several streams.
 * Returns SPHFILT_EINVAL for n_* <= 0, odd n_phi, NULL pointers, parity not
 * +-1, non-finite or non-positive rho / L, unknown kind, bad floor;
 * SPHFILT_EUNSUPPORTED for unsupported sizes; SPHFILT_ENOMEM /
 * SPHFILT_EDEVICE when allocation or upload fails.
 */
int sphfilt_plan_create(sphfilt_plan *out, int n_r, int n_theta, int n_phi, int n_fields,
                        const int *parity, const sphfilt_cutoff *cut);

/* Release the plan's device tables.  NULL is accepted.  Not stream-ordered:
 * the caller makes sure no enqueued call still uses the plan. */
int sphfilt_plan_destroy(sphfilt_plan plan);

/*
 * out = Phi(Theta(in)): the double FFT filter, theta first (Sec. II.A).
 *   in, out  device pointers to n_fields*n_r*n_theta*n_phi doubles, layout
 *            [f][r][theta][phi], each 16-byte aligned (hipMalloc and the
 *            PyTorch allocator give 256-byte alignment; the theta pass moves
 *            two adjacent doubles per access), else SPHFILT_EINVAL.  in == out
 *            (in place) is allowed and is the fast path: lines whose mask is
 *            all ones are not touched.  Any other overlap of the two ranges is
 *            SPHFILT_EINVAL.
 *   stream   a hipStream_t (NULL = the null stream).
 * Enqueues two kernels and returns; SPHFILT_EDEVICE if a launch fails.
 */
int sphfilt_apply(sphfilt_plan plan, const double *in, double *out, void *stream);

/* out = Theta(Phi(in)) = F^T in: the transpose of sphfilt_apply (each pass is
 * real symmetric).  Arguments and errors as for sphfilt_apply. */
int sphfilt_apply_adjoint(sphfilt_plan plan, const double *in, double *out, void *stream);

/*
 * The filter with control over the hybrid kind's decisions.
 *   adjoint     0: Phi(Theta(in)); 1: Theta(Phi(in)).
 *   theta_dec   device bytes [n_fields][n_r][n_phi/2], one per extended theta
 *               line (meridian pair k); phi_dec: [n_fields][n_r][n_theta], one
 *               per ring.  1 = Gaussian, 0 = exponential; entries of
 *               non-hybrid fields are not touched.
 *   replay      0: hybrid lines decide from the data each pass sees; if the
 *               buffers are not NULL the decisions are written there.
 *               1: hybrid lines use the decisions in the buffers (both
 *               required): the filter is then linear, and the adjoint call
 *               with the decisions of a forward call is its exact transpose.
 * Other arguments and errors as for sphfilt_apply.
 */
int sphfilt_apply_ex(sphfilt_plan plan, const double *in, double *out, int adjoint,
                     unsigned char *theta_dec, unsigned char *phi_dec, int replay, void *stream);

/* The theta-pass alone (Sec. II.A, theta FFT filter on extended lines).
 * Arguments and errors as for sphfilt_apply. */
int sphfilt_apply_theta(sphfilt_plan plan, const double *in, double *out, void *stream);

/* The phi-pass alone (Sec. II.A, phi FFT filter on rings). */
int sphfilt_apply_phi(sphfilt_plan plan, const double *in, double *out, void *stream);

/* Work and traffic figures of a plan (host only, no device call). */
int sphfilt_plan_stats(sphfilt_plan plan, sphfilt_stats *out);

/* The same figures for a would-be plan, without creating one or touching a
 * device; validates exactly like sphfilt_plan_create. */
int sphfilt_workload_stats(int n_r, int n_theta, int n_phi, int n_fields, const int *parity,
                           const sphfilt_cutoff *cut, sphfilt_stats *out);

/*
 * Launch shape of a plan's kernels (tuning only: results are bitwise
 * independent of phi_lines, and of theta_cols except where 2*n_theta = 256,
 * where it moves round-off only; see below).
 *   theta_cols  complex lines per shell in one theta workgroup: 4, 8, 16,
 *               32 or 64, at most n_phi/4, at most the lines of one theta
 *               workgroup (16 for 2*n_theta = 160, 192 or 256, 32 for 64,
 *               80, 96 or 128, 64 for 32 or 48), and 2*theta_cols must
 *               divide n_phi/2.  A workgroup covers 2*theta_cols meridian
 *               pairs of each of its 256/lanes/theta_cols shells; each line
 *               packs two adjacent ones, or, where 2*n_theta = 256, two
 *               theta_cols apart.  The default is the widest such tile.
 *               0 keeps the value.  For fields that are not hybrid the
 *               plan's theta kernel runs workgroups of 128 lanes where that
 *               measured faster (2*n_theta = 32, 48, 64, 96, 160, 192), and
 *               there takes the smaller of theta_cols and the lines of 128
 *               lanes (the result does not depend on the width at these
 *               lengths).
 *   phi_lines   ring pairs per workgroup of the phi kernel: 4, 8, 16, 32 or
 *               64 (at most 256 lanes per workgroup).  The default is 4 at
 *               n_phi = 256, 8 at 64, 80, 96, 128, 160 and 192, and a full
 *               256-lane workgroup otherwise.  0 keeps the value.
 * Returns SPHFILT_EINVAL for other values.  Not thread-safe against
 * concurrent apply calls on the same plan.
 */
int sphfilt_plan_set_schedule(sphfilt_plan plan, int theta_cols, int phi_lines);
int sphfilt_plan_get_schedule(sphfilt_plan plan, int *theta_cols, int *phi_lines);

/*
 * Fused shells.  On grids with n_phi = 2 * n_theta in {32, 64, 128} a whole
 * shell (field, radius) fits in one workgroup's LDS.  A shell whose every
 * theta line and every ring is filtered (no identity line) then goes through
 * one kernel that loads it once, runs both passes in LDS and registers, and
 * stores it once: one HBM round trip instead of two (the passes are applied
 * in the order of the call, so the operator is unchanged).  The other shells
 * take the two-pass path (on these grids only ring pairs are left: a shell
 * the theta pass filters has all its rings filtered, since m_max <= l_max),
 * in the same launch.  Results equal those of the two-pass path up to
 * rounding (the same line transforms, with multiply-adds contracted
 * differently by the compiler).
 *   enable  1 (the default): fuse where possible; 0: always two passes.
 * set_fused returns SPHFILT_EINVAL for other values; it is not thread-safe
 * against concurrent apply calls on the same plan.  get_fused reports the
 * setting and the number of shells fused when it is on (NULL outputs are
 * skipped).
 */
int sphfilt_plan_set_fused(sphfilt_plan plan, int enable);
int sphfilt_plan_get_fused(sphfilt_plan plan, int *enable, int *shells_fused);

/*
 * Autotune a plan: the theta tile width and phi ring pairs per workgroup
 * (sphfilt_plan_set_schedule), fused shells, the theta variant and the
 * overlap mode, by coordinate descent from the plan's current settings, each
 * candidate timed as forward filters in place, back to back (as a
 * time-stepping loop calls them), on scratch fields of the plan's size that
 * the call allocates and frees.  The untuned settings are a
 * candidate, so the pick is never slower than them by the tuner's own
 * measurement.
 *   tune_cache_path  a JSON file shared with the batch tuner: if it holds
 *                    settings for this plan (grid, fields, cutoffs) on this
 *                    GPU architecture they are applied without timing, else
 *                    the tuner runs and records its pick there (SPHFILT_EINVAL
 *                    if the file cannot be written).  NULL: the file named
 *                    by SPHFILT_TUNE_CACHE if set and not empty, else tune
 *                    without recording.
 * Synchronous; not thread-safe against concurrent calls on the same plan.
 * sphfilt_plan_tuned_times reports the tuner's time per forward call with
 * the pick and with the settings it started from (negative when not tuned;
 * NULL outputs are skipped).
 */
int sphfilt_plan_tune(sphfilt_plan plan, const char *tune_cache_path);
int sphfilt_plan_tuned_times(sphfilt_plan plan, double *tuned_us, double *default_us);

/*
 * Theta-pass variant (grids with n_phi = 2 * n_theta in {32, 64} only).
 * On one extended theta line the theta filter is the circular convolution
 * with c[d] = (1/N) sum_q f(|q|; l_max) cos(2 pi q d / N), the inverse
 * transform of the mask (Sec. II.A, theta filter); all lines of a shell share
 * l_max, so a shell's theta pass is one product of that N x N circulant with
 * the N x N/2 matrix of its extended lines.  SPHFILT_THETA_MFMA computes it
 * that way on the FP64 matrix cores (2N flops per point instead of the
 * FFT's ~5 log2 N, no transposes), in the two-pass path and inside the fused
 * shell kernel; hybrid fields keep the FFT.  Results equal the FFT path's to
 * rounding (a different summation order), not bit for bit.
 *   variant  SPHFILT_THETA_FFT (the default) or SPHFILT_THETA_MFMA.
 * set returns SPHFILT_EINVAL for other values and SPHFILT_EUNSUPPORTED for
 * MFMA on other grids; not thread-safe against concurrent apply calls on
 * the same plan.
 */
#define SPHFILT_THETA_FFT  0
#define SPHFILT_THETA_MFMA 1
int sphfilt_plan_set_theta_variant(sphfilt_plan plan, int variant);
int sphfilt_plan_get_theta_variant(sphfilt_plan plan, int *variant);

/*
 * Overlapped passes (in place, shells not fused).  The rings of shells whose
 * theta mask is all ones do not depend on the theta pass.  An overlapped
 * in-place call runs them on a second stream owned by the plan, alongside the
 * theta pass and the rings of the theta-filtered shells on the caller's
 * stream; the caller's stream then waits for that stream (event fork and
 * join, so the call stays stream-ordered and can be captured in a HIP graph).
 * Each ring's arithmetic is unchanged: results are bitwise those of the
 * two-pass path.  The stream and two events are created with the plan (on
 * its device) when the plan has theta-filtered shells that are not fused and
 * rings independent of them, and released by sphfilt_plan_destroy; no call
 * creates them, so a call can be captured in a HIP graph.  Enqueueing takes a
 * lock of the plan.
 *   mode  0 (the default): both passes on the caller's stream;
 *         1: overlap when those rings move at least 128 MiB (below that the
 *           fork and join cost more than they hide);
 *         2: overlap whenever there is theta work and such a ring.
 * With the default phi launch shape the overlapped passes measured slower
 * than the two passes in a row (the second stream's small workgroups crowd
 * the theta pass); sphfilt_plan_tune tries every mode.
 * set_overlap returns SPHFILT_EINVAL for other values; get_overlap needs a
 * non-NULL output.
 */
int sphfilt_plan_set_overlap(sphfilt_plan plan, int mode);
int sphfilt_plan_get_overlap(sphfilt_plan plan, int *mode);

/* ======================================================================
 * Batched filter: many uneven spherical patches in one launch.
 *
 * Each patch is filtered exactly as by its own plan (same operator, same
 * per-line arithmetic: bit-identical results to a two-pass plan without
 * hybrid fields, equal to rounding otherwise); the batch schedules every
 * patch's theta groups and ring-pair groups as items of one persistent
 * kernel, replayed from a captured HIP graph.  This is the GPU counterpart of
 * the paper's OpenMP loop over many line transforms on one rank (Sec. II.B).
 * ====================================================================== */

/* One patch: grid, fields, parities and cutoffs, as for sphfilt_plan_create. */
typedef struct {
    int n_r, n_theta, n_phi, n_fields;
    const int *parity;          /* [n_fields], +1 or -1 */
    sphfilt_cutoff cut;
} sphfilt_patch_desc;

/*
 * Create a batch of n_patches patches on the current HIP device.
 *   desc             [n_patches] patch descriptions; validated like
 *                    sphfilt_plan_create (same error codes).  A batch with
 *                    a line that is not a power of two (48, 80, 96, 160 or
 *                    192 points) runs a kernel instance that carries those
 *                    lengths too (one wave per SIMD).  Read during the call
 *                    only.
 *   tune_cache_path  a JSON file: if it holds a schedule for this set of
 *                    patches on this GPU architecture, that schedule is used;
 *                    if not, the autotuner times the candidate schedules (see
 *                    sphfilt_batch_schedule) on scratch fields it allocates
 *                    and frees, and records the winner there (SPHFILT_EINVAL
 *                    if the file cannot be written).  NULL: the file named by
 *                    the environment variable SPHFILT_TUNE_CACHE if it is set
 *                    and not empty, else the untuned default schedule.
 * The batch owns its device tables and a small set of work counters; calls on
 * one batch must be stream-ordered (two overlapping calls on one batch race
 * on the counters).
 */
int sphfilt_batch_create(sphfilt_batch *out, int n_patches, const sphfilt_patch_desc *desc,
                         const char *tune_cache_path);

/* Release the batch (synchronises the device first).  NULL is accepted. */
int sphfilt_batch_destroy(sphfilt_batch batch);

/*
 * Filter every patch: outs[p] = Phi(Theta(ins[p])) (adjoint = 0) or
 * Theta(Phi(ins[p])) (adjoint != 0).
 *   ins, outs  host arrays of n_patches device pointers, each patch's fields
 *              in the layout of sphfilt_apply and 16-byte aligned as there
 *              (else SPHFILT_EINVAL).  ins[p] == outs[p] for every
 *              patch is the in-place fast path; an output that partially
 *              overlaps its own input, or overlaps any other patch's input
 *              or output, is SPHFILT_EINVAL.
 *   stream     a hipStream_t (NULL = the null stream).
 * The first call with a given set of pointers (and direction) captures a HIP
 * graph (a counter-reset kernel and the persistent kernel) and caches it;
 * later calls replay it with one graph launch.  Enqueues and returns.
 */
int sphfilt_batch_apply(sphfilt_batch batch, const double *const *ins, double *const *outs,
                        int adjoint, void *stream);

/*
 * For callers that cannot allocate device memory during a call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same filter as sphfilt_batch_apply, with the same arguments, checks and
 * results (the same kernels on the same work lists), that allocates nothing.
 * The batch's tables and work lists are built by sphfilt_batch_create (and
 * rebuilt by sphfilt_batch_tune / sphfilt_batch_set_fused); the per-call
 * counters, tickets, error word and the patch pointer tables live in a
 * statically allocated device array of the library, about 1.02 MiB
 * (256 B + 16 KiB of pointer tables + 1 MiB of counters), one copy per device,
 * held until the process ends.  The kernels are enqueued directly on `stream`
 * (no graph is captured; split = 2 schedules still fork onto the batch's own
 * stream and join back).
 * Limits: at most 1024 patches and 262144 shells (n_fields * n_r summed over
 * the patches), else SPHFILT_EUNSUPPORTED.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (on different streams, from any batch) race and give wrong
 * results; calls must be ordered on one stream, or synchronised.  The array
 * keeps the last call's contents; each call clears what must start at zero
 * (counters, tickets, error word) with a kernel before its filter kernels.
 * sphfilt_batch_status reports this array's error word when the batch's last
 * call was this one (valid until the next allocation-free call on the device).
 */
int sphfilt_batch_apply_noalloc(sphfilt_batch batch, const double *const *ins,
                                double *const *outs, int adjoint, void *stream);

/* Run the autotuner now (see sphfilt_batch_create); tune_cache_path may be
 * NULL to tune without recording.  Synchronous. */
int sphfilt_batch_tune(sphfilt_batch batch, const char *tune_cache_path);

/*
 * Schedule of the batch kernel.
 *   split              0: one persistent kernel; second-pass items wait on
 *                      per-shell counters of the first pass.  1: two
 *                      persistent kernels, first pass then second pass.
 *                      2: as 1, and the second-pass items whose shells no
 *                      first-pass item writes (in place: the rings of
 *                      theta-idle shells) run on a parallel branch of the
 *                      graph, on a stream of the batch, alongside the first
 *                      pass.
 *   workgroups_per_cu  -1: one workgroup per work item (each takes one item
 *                      and exits).  k > 0: a persistent grid of k workgroups
 *                      per compute unit looping over items; 0 = the most
 *                      that fit.  k above the most that fit (the occupancy
 *                      of the persistent kernel: 1 on batches with hybrid
 *                      fields) is SPHFILT_EINVAL.
 * get_schedule also returns the tuned time of one call in microseconds
 * (negative when not tuned).  Results do not depend on the schedule.
 */
int sphfilt_batch_set_schedule(sphfilt_batch batch, int split, int workgroups_per_cu);
int sphfilt_batch_get_schedule(sphfilt_batch batch, int *split, int *workgroups_per_cu,
                               double *tuned_us);

/*
 * The whole schedule of a batch, as the autotuner searches it (coordinate
 * descent from the untuned schedule, every candidate timed on scratch fields
 * with the batch's own kernels, calls back to back; the pick and both times
 * are recorded in the JSON cache):
 *   split, workgroups_per_cu  as for sphfilt_batch_set_schedule (get: the
 *                      effective workgroups per CU).
 *   fused              fused items (see sphfilt_batch_set_fused), 0 or 1.
 *   theta_tiles        meridian tiles per theta work item: 1, 2, 4 or 8 (an
 *                      item runs them one after another).
 *   phi_groups         workgroup rounds of ring pairs per phi work item: 1,
 *                      2, 4 or 8.
 *   theta_cols[i]      theta sub-tile width (as theta_cols of
 *                      sphfilt_plan_set_schedule) for patches whose theta
 *                      line has {32, 48, 64, 80, 96, 128, 160, 192, 256}[i]
 *                      points; 0 = the default width.  A width a patch's grid
 *                      does not take falls back to its default.
 *   tuned_us, default_us  (get only) the tuner's time per call with the
 *                      picked and with the untuned schedule; negative when
 *                      not tuned.
 * set_schedule_ex returns SPHFILT_EINVAL for values outside these sets;
 * changing the item shapes (everything but split and workgroups_per_cu)
 * synchronises the device and rebuilds the work lists and graphs.  Results
 * do not depend on the schedule except through theta_cols where a theta line
 * has 256 points (round-off only; see sphfilt_plan_set_schedule).
 */
typedef struct {
    int split, workgroups_per_cu, fused, theta_tiles, phi_groups;
    int theta_cols[9];
    double tuned_us, default_us;
} sphfilt_batch_schedule;
int sphfilt_batch_set_schedule_ex(sphfilt_batch batch, const sphfilt_batch_schedule *sched);
int sphfilt_batch_get_schedule_ex(sphfilt_batch batch, sphfilt_batch_schedule *sched);

/* Device error word of the batch's last call (synchronises the device): 0,
 * or 1 if a second-pass item gave up waiting for its shells (a library bug;
 * such an item stores nothing, so its lines hold the first pass's result and
 * the call's output is invalid).  Callers that need the guarantee poll this
 * after their calls. */
int sphfilt_batch_status(sphfilt_batch batch, int *device_error);

/* Work and traffic figures summed over the batch's patches (host only);
 * shells_fused and bytes_fused_inplace follow sphfilt_batch_set_fused. */
int sphfilt_batch_stats(sphfilt_batch batch, sphfilt_stats *out);

/*
 * Fused shells in a batch (as sphfilt_plan_set_fused): a patch with
 * n_phi = 2 * n_theta <= 128 runs its theta-filtered shells as fused items
 * (one HBM round trip for both passes) and the rings of its other shells in
 * the first pass, so it has no second-pass work.
 *   enable  1 or 0 (every patch in two passes).  The autotuner times both
 *           (when some patch allows fused items) with every schedule and keeps
 *           the fastest; untuned batches start with 1.
 * Changing it drops the batch's captured graphs and work lists (they are
 * rebuilt on the next call) after synchronising the device.  get_fused
 * reports the setting and the number of shells fused (NULL outputs are
 * skipped).
 */
int sphfilt_batch_set_fused(sphfilt_batch batch, int enable);
int sphfilt_batch_get_fused(sphfilt_batch batch, int *enable, int *shells_fused);

/* Human-readable text of a status code (static storage). */
const char *sphfilt_status_string(int status);

/* Library version, "major.minor.patch" (static storage). */
const char *sphfilt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPHFILT_H */
