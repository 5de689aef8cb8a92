/*
 * cpra.h - C ABI of the carousel phase retrieval (CPRA) hot path on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: F. Ai, V. Lomakin, O. Shpyrko, "Real time 3D coherent X-ray
 * diffraction imaging" (arXiv 2402.05283).  A scan is N_p intensity maps
 * I(q_t,n, q_i,n) of N x N pixels, one per rotation angle theta_n about z
 * (problem statement, Eq. 1-3).  Each map is phased by 2D iterative phase
 * retrieval of its projected object (PO); the POs of neighbouring angles
 * are re-combined at the start of every episode (Eq. 4, the "carousel");
 * the retrieved 2D spectra are finally inserted along their Fourier slices
 * into a 3D spectrum and transformed back (step D).
 *
 * Conventions shared by every entry point:
 *   - Real-space arrays (supports, POs) are [n][z][t] with z the rotation
 *     axis, t the transverse axis, origin at index N/2 (centred).
 *   - Intensities are [n][w][u] with zero frequency at index N/2 (centred),
 *     w the frequency along z and u along t.  I < 0 marks an unmeasured
 *     pixel (beamstop); NaN or Inf is rejected.
 *   - The output volume is [z][y][x], origin at index N/2.
 *   - All calls return a cpra_status and never throw or abort.  An argument
 *     error leaves the plan unchanged.  A device error poisons the plan:
 *     every later call on it returns CPRA_ERR_STATE (cpra_destroy excepted).
 *   - One host thread per plan at a time; distinct plans are independent.
 */
#ifndef CPRA_H
#define CPRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpra_plan_s* cpra_plan_t;

typedef enum {
  CPRA_OK = 0,
  CPRA_ERR_ARG = -1,          /* invalid argument; nothing changed            */
  CPRA_ERR_OOM = -2,          /* workspace too small                          */
  CPRA_ERR_DEVICE = -3,       /* HIP runtime error; the plan is now poisoned  */
  CPRA_ERR_STATE = -4,        /* call not valid in the plan's current state   */
  CPRA_ERR_UNSUPPORTED = -5,  /* size or option not built                     */
  CPRA_ERR_DATA = -6          /* NaN or Inf in the intensities                */
} cpra_status;

enum { CPRA_HIO = 0, CPRA_ER = 1, CPRA_RAAR = 2 };   /* real-space update     */
enum { CPRA_INSERT_NEAREST = 0, CPRA_INSERT_BILINEAR = 1 };   /* step D insertion */
enum { CPRA_WRAP_MIRROR = 0, CPRA_WRAP_PLAIN = 1 };  /* carousel seam rule    */
enum { CPRA_REAL_F32 = 0, CPRA_REAL_F64 = 1 };       /* arithmetic precision  */
enum { CPRA_AMP_F32 = 0, CPRA_AMP_F16 = 1 };         /* amplitude storage     */
enum { CPRA_PTR_HOST = 0, CPRA_PTR_DEVICE = 1, CPRA_PTR_DEVICE_ASYNC = 2 };

typedef struct {
  uint32_t struct_size;  /* = sizeof(cpra_params)                                     */
  int32_t N;             /* map side; 64, 128, 192, 256, 384, 512 or 1024 (else        
                            UNSUPPORTED)                                               */
  int32_t Np;            /* number of angles, >= 1                                      */
  const double* theta;   /* Np angles in radians (host, copied), or NULL: pi*n/Np       */
  double alpha[3];       /* Eq. 4 weights a_-1, a_0, a_+1; each >= 0, |sum - 1| <= 1e-12 */
  int32_t n_ei;          /* iterations per episode (coupling period), >= 1              */
  int32_t wrap;          /* CPRA_WRAP_MIRROR: the neighbour reached across the 180-deg
                            seam is t-mirrored (PO at theta+pi); CPRA_WRAP_PLAIN: not   */
  int32_t positivity;    /* 1: the object constraint is support AND (g' >= 0)           */
  int32_t real_type;     /* CPRA_REAL_F32 (product path) or CPRA_REAL_F64               */
  int32_t amp_type;      /* CPRA_AMP_F32, or CPRA_AMP_F16 (F32 plans only): sqrt(I) kept
                            as binary16 times a per-angle power-of-two scale            */
  uint64_t seed;         /* key of the counter-based SplitMix64 initial phases          */
  int32_t n_guess;       /* N_r independent reconstructions of the scan held at once
                            (step C's random guesses; 0 means 1).  Guess r of angle n is
                            slot r * Np + n: its own iterate and random start (phase
                            stream index r * Np + n), the angle's data shared.        */
  int32_t insertion;     /* step D's interpolation: CPRA_INSERT_NEAREST (nearest voxel,
                            plain average) or CPRA_INSERT_BILINEAR (four cells around the
                            slice point, weighted average sum(w E) / sum(w))          */
  const double* taps;    /* NULL, or n_taps = 2K+1 weights alpha_{-K..K} of Eq. 4 (copied
                            at plan creation; >= 0, sum 1, centre > 0, 2K+1 <= Np), in
                            place of alpha: O_n <- sum_k alpha_k X_{n+k}, periodic, the
                            wrapped neighbours t-mirrored under CPRA_WRAP_MIRROR        */
  int32_t n_taps;        /* 0 (use alpha) or odd >= 3                                   */
} cpra_params;

/*
 * Device workspace bytes a plan with these parameters needs (host only; no
 * GPU call).  ERR_ARG / ERR_UNSUPPORTED for invalid or unbuilt parameters.
 */
cpra_status cpra_workspace_size(const cpra_params* params, size_t* bytes);

/*
 * Create a plan on the current HIP device.  `workspace` is caller-owned
 * device memory of at least cpra_workspace_size() bytes, 256-byte aligned,
 * that must outlive the plan; `hip_stream` (hipStream_t, NULL = default
 * stream) orders all of the plan's device work.  The plan owns only host
 * memory.  Twiddle tables are generated on the device in FP64.
 */
cpra_status cpra_plan(const cpra_params* params, void* workspace, size_t workspace_bytes, void* hip_stream,
                      cpra_plan_t* out);

/* The same call under its earlier name (identical arguments and behaviour). */
cpra_status cpra_plan_create(const cpra_params* params, void* workspace, size_t workspace_bytes,
                             void* hip_stream, cpra_plan_t* out);

/*
 * Input preparation (problem statement; step A initialisation): hand over
 * the maps of angles [first, first+count).  intensity: count x N x N float,
 * centred [n][w][u]; support: count x N x N uint8 (nonzero = inside),
 * centred [n][z][t].  Both on the host (CPRA_PTR_HOST: copied before the
 * call returns) or on the device (CPRA_PTR_DEVICE, CPRA_PTR_DEVICE_ASYNC:
 * read in stream order).
 * Computes A = sqrt(I), packs the support, and draws each angle's random
 * initial PO (W_0): Re F2^-1(A exp(i phi)), phi from SplitMix64(seed) at
 * counter (n*N + w)*N + u.  An angle may be submitted once.  An angle that
 * arrives mid-episode waits and joins at the next episode boundary.
 * CPRA_PTR_HOST and CPRA_PTR_DEVICE synchronise the stream and return
 * ERR_DATA (nothing submitted) if the intensities hold a NaN or Inf.
 * CPRA_PTR_DEVICE_ASYNC (for a serving loop that must not wait on the GPU)
 * does not synchronise with plans of one guess: the angles count as
 * submitted at once, and the NaN/Inf check completes in stream order; the
 * first call on the plan after it completes (submit, iterate, iterate_batch,
 * read_objects, assemble_volume) returns ERR_DATA if it failed, and the plan
 * is then poisoned.  The device inputs must stay valid until the stream has
 * consumed them.
 */
cpra_status cpra_submit_angles(cpra_plan_t plan, int32_t first, int32_t count,
                               const float* intensity, const uint8_t* support, int32_t ptr_kind);

/*
 * Run n_iter iterations over the angles present (steps B, Eq. 4).  At each
 * episode boundary (global iteration count k with k mod n_ei == 0) every
 * present PO is replaced by a_-1 X_{n-1} + a_0 X_n + a_+1 X_{n+1}, X the
 * previous episode's objects, over the periodic ring of present angles
 * (absent neighbours drop out, weights renormalised).  Each iteration:
 * G = F2(g); E_F = sqrt(sum (|G|-A)^2 / sum A^2) over measured pixels;
 * G' = A G/|G|; g' = Re F2^-1(G'); gamma = support AND (g' >= 0);
 * HIO (algo CPRA_HIO): g <- g' on gamma, g - beta g' elsewhere;
 * ER (CPRA_ER): g <- g' on gamma, 0 elsewhere;
 * RAAR (CPRA_RAAR, Luke's relaxed averaged alternating reflections, the
 * paper's choice for the measured cell): g <- beta/2 (R_S R_M + 1) g +
 * (1 - beta) P_M g with P_M g = g', R = 2P - 1 and P_S the support (and
 * positivity) projection; per pixel g' where 2g' - g meets the constraints,
 * beta g + (1 - 2 beta) g' elsewhere.  The last iteration of an
 * episode writes the estimate g' on gamma, 0 elsewhere.
 * Every guess runs the same schedule on its own ring of slots.
 * err_out: NULL, or host n_iter x (n_guess * Np) doubles receiving E_F per
 * slot (NaN for absent angles); non-NULL synchronises the stream.  Otherwise
 * asynchronous.  ERR_STATE if no angle is present.
 */
cpra_status cpra_iterate(cpra_plan_t plan, int32_t n_iter, int32_t algo, double beta, double* err_out);

/*
 * Step A, pre-reconstruction: PO 1 (angle 0) of every guess runs n_iter
 * iterations of plain 2D phase retrieval from its current object, with no
 * coupling; the last iteration writes the estimate.  The other angles keep
 * their random starts, which together make the first episode W_0.  Does
 * not change k.  err_out: NULL, or host n_guess x n_iter doubles (E_F).
 * ERR_STATE unless angle 0 has been submitted.  Synchronises only when
 * err_out is non-NULL.
 */
cpra_status cpra_prereconstruct(cpra_plan_t plan, int32_t n_iter, int32_t algo, double beta, double* err_out);

/*
 * Step B in its consecutive form: n_episodes episodes, each taking the POs
 * in order n = 0 .. Np-1.  PO n (of every guess at once) is re-initialised
 * from Eq. 4 over its neighbours' most recent objects (n-1 from this
 * episode, n+1 from the previous one, the ring wrapping with the t-mirror
 * across the 180-degree seam under CPRA_WRAP_MIRROR), then runs n_ei
 * iterations, the last writing its estimate.  Work is sequential over
 * angles and parallel over guesses.  k advances by n_episodes * n_ei.
 * err_out: NULL, or host n_episodes x n_guess x Np x n_ei doubles (E_F);
 * non-NULL synchronises after every angle.  ERR_STATE unless every angle
 * has been submitted and k mod n_ei == 0.
 */
cpra_status cpra_sweep(cpra_plan_t plan, int32_t n_episodes, int32_t algo, double beta, double* err_out);

/*
 * Step C, merge of the guesses.  Error of a guess: E = sqrt(sum_n sum_q
 * (|F2 X_n| - A_n)^2 / sum_n sum_q A_n^2) over measured q, on its current
 * objects X_n.  Keeps the n_best guesses of lowest E (ties in guess order);
 * moves every kept PO's mass centre c = sum X r / sum X (r from the centre
 * index N/2) to the origin by the cyclic integer shift floor(-c + 1/2) per
 * axis; for every kept guess but the best, compares its shifted PO 1 with
 * the best guess's shifted PO 1 and with its central inversion X(-r), and
 * inverts all its POs if the inversion is nearer (squared distance, FP64);
 * averages the kept guesses.  The result replaces guess 0's objects (slots
 * 0 .. Np-1) and its row spectra, so cpra_read_objects (first Np planes)
 * and cpra_assemble_volume (step D) use it; other guesses are unchanged.
 * kept, inverted: NULL or host arrays of n_best entries receiving the kept
 * guesses in rank order and whether each was inverted.  ERR_ARG unless
 * 1 <= n_best <= n_guess; ERR_STATE unless every angle has been submitted
 * and k mod n_ei == 0.  Synchronises the stream.
 */
cpra_status cpra_merge(cpra_plan_t plan, int32_t n_best, int32_t* kept, int32_t* inverted);

/*
 * HIP graphs for the iteration (off by default): with enable != 0, whole
 * episodes that start at a boundary (k mod n_ei == 0) in cpra_iterate
 * without err_out and in cpra_iterate_batch are replayed from a captured
 * graph of the episode's 2 n_ei launches (one graph per ping-pong parity,
 * recaptured when the angle set, algo or beta changes).  Results are
 * bit-identical to the launch-by-launch path; per-pass event timing is not
 * recorded for graph episodes.  Saves launch overhead for small N.
 */
cpra_status cpra_set_graphs(cpra_plan_t plan, int32_t enable);

/*
 * Launch order inside an episode.  Between two coupling boundaries every
 * slot iterates on its own, so the n_ei - 1 iterations after a boundary may
 * run chunk by chunk: the listed slots are cut into chunks of `slots`, and
 * each chunk runs all of those iterations (column and row pass per
 * iteration) before the next chunk starts.  A chunk's planes then stay in
 * the last-level cache between passes.  The boundary iteration always runs
 * over all slots (Eq. 4 reads the neighbours' previous episode).  Results
 * are bit-identical for any chunk size.  slots = 0 (the default) or
 * slots >= listed slots: every launch covers all slots.  ERR_ARG if
 * slots < 0.
 */
cpra_status cpra_set_chunk(cpra_plan_t plan, int32_t slots);

/*
 * Several independent scans at once (the data-parallel dimension of steps B
 * and C over scans rather than angles): `count` distinct plans, possibly of
 * different N and Np, each advance n_iter iterations with the same algo and
 * beta.  Each plan's episode phase follows its own k, exactly as
 * cpra_iterate would.  Plans of one size class (same N, real type and
 * amplitude type) with three-tap coupling and launch-by-launch episodes
 * share launches: per iteration, one column-pass and one row-pass launch
 * over the listed slots of up to 16 such plans (more launches only when the
 * plans stand at different points of their episodes), issued on the first
 * plan's stream, which is ordered after every plan's stream before and
 * before every plan's stream after.  Other plans advance interleaved,
 * iteration by iteration, each on its own stream.  Results are those of
 * calling cpra_iterate on each plan alone, bit for bit.  No error history is
 * returned (use cpra_iterate for that).  Checks every plan first: NULL
 * array, NULL or repeated plans, a poisoned plan, or a plan with no angle
 * return ERR_ARG / ERR_STATE and no plan advances.  A device error poisons
 * the plan it occurred in and returns ERR_DEVICE; the others stay usable.
 * Asynchronous, except where a plan's angle set changes at a boundary (its
 * coupling tables are uploaded and the stream synchronised).
 */
cpra_status cpra_iterate_batch(cpra_plan_t* plans, int32_t count, int32_t n_iter, int32_t algo, double beta);

/*
 * Process-wide choice of the size classes whose plans share launches in
 * cpra_iterate_batch: those with N <= max_n (0: none; the library's default
 * is given in its documentation of measurements).  Plans outside advance
 * on their own streams with their own launches; results are identical
 * either way.  ERR_ARG if max_n < 0.
 */
cpra_status cpra_set_batch_fusion(int32_t max_n);

/* The current setting of cpra_set_batch_fusion (host only). */
cpra_status cpra_get_batch_fusion(int32_t* max_n);

/*
 * Launch choices of a plan that do not change its results, only its speed:
 * row_tile 0 runs the row pass with its compiled rows per workgroup, 1 with
 * twice as many; chunk as cpra_set_chunk; graphs as cpra_set_graphs.
 * ms_per_iteration: the time one iteration took with them (filled by
 * cpra_autotune; ignored by cpra_set_tuning).
 */
typedef struct {
  int32_t row_tile;
  int32_t chunk;
  int32_t graphs;
  double ms_per_iteration;
} cpra_tuning;

/* Apply launch choices to a plan (host only).  ERR_ARG for a bad value. */
cpra_status cpra_set_tuning(cpra_plan_t plan, const cpra_tuning* t);

/*
 * Autotuner: build a temporary plan with these parameters on `workspace`
 * (cpra_workspace_size bytes, the caller's; its contents are overwritten),
 * fill it with a synthetic scan generated on the device, and time n_iter
 * HIO iterations (rounded up to whole episodes) for every combination of
 * row_tile {0, 1}, chunk {0, slots/2, slots/4 where >= 16 slots} and graphs
 * {0, 1}, each after one warm episode, with HIP events on `hip_stream`.
 * Returns the fastest in *best, or the default choices (all 0) unless the
 * fastest beats them by more than 2% (closer than that is timing noise), and
 * records it for the shape (N, Np, real type, amplitude type, guesses): plans
 * of that shape created afterwards in this process start with these choices.
 * Synchronises the stream.
 */
cpra_status cpra_autotune(const cpra_params* params, void* workspace, size_t workspace_bytes, void* hip_stream,
                          int32_t n_iter, cpra_tuning* best);

/*
 * Shrinkwrap support update (the conventional 2D shrinkwrap step, run by
 * the paper at the end of each episode to tighten the space constraints):
 * for every present angle, blur the current object with the periodic 2D
 * Gaussian k(dz) k(dt), k(d) = exp(-d^2 / 2 sigma^2) for |d| <= ceil(4
 * sigma) normalised to sum 1, and make the support the pixels where the
 * blurred object is >= threshold * its maximum.  Replaces the submitted
 * supports.  ERR_ARG unless sigma > 0 with ceil(4 sigma) < N/2 and
 * 0 < threshold <= 1; ERR_UNSUPPORTED for plans with several guesses (the
 * support is per angle); ERR_STATE unless k mod n_ei == 0.  Synchronises.
 */
cpra_status cpra_shrinkwrap(cpra_plan_t plan, double sigma, double threshold);

/*
 * The supports in use, Np x N x N [n][z][t] centred, 0/1 bytes, into host
 * memory (as submitted, or as replaced by cpra_shrinkwrap).  Synchronises.
 */
cpra_status cpra_read_support(cpra_plan_t plan, uint8_t* out);

/*
 * Current real-space iterate of every slot, n_guess x Np x N x N [r][n][z][t]
 * centred, float (F32 plans) or double (F64 plans), host or device.  At an
 * episode end this is the episode's estimate; angles not submitted yet read
 * as zero.  Host copies synchronise the stream.
 */
cpra_status cpra_read_objects(cpra_plan_t plan, void* out, int32_t ptr_kind);

/*
 * Warm start: replace the current iterate of every submitted angle by
 * `objects` (n_guess x Np x N x N [r][n][z][t] centred, float for F32 plans
 * or double for F64 plans; host or device; rows of angles not yet submitted
 * are ignored)
 * and recompute the plan's internal row spectra from it.  The iteration
 * count k is unchanged, so the next episode boundary couples these objects.
 * Lets a caller seed a scan from an earlier result or from a separate
 * pre-reconstruction.  Synchronises the stream.
 */
cpra_status cpra_load_objects(cpra_plan_t plan, const void* objects, int32_t ptr_kind);

/*
 * Step D: insert the spectra F2(O'_n) of the current estimates along their
 * Fourier slices (nearest voxel of (-u sin t, u cos t, w), floor(x+0.5) in
 * FP64, averaged per voxel; or, with CPRA_INSERT_BILINEAR, the four voxels
 * around that point with bilinear weights built in FP64, weighted average;
 * empty voxels zero) and return the real part of
 * the 3D inverse transform: N x N x N [z][y][x] centred, float (F32 plans)
 * or double (F64 plans), device memory.  Computed z-plane by z-plane (the
 * 3D transform factorises into the row spectra already held per angle), so
 * no N^3 complex grid is formed.  The first step-D call of a plan (this or
 * cpra_refine_volume) builds the insertion tables on the host and uploads
 * them on the stream (the host copy may wait for the stream's earlier
 * work); the kernels are queued asynchronously.  ERR_STATE unless
 * k mod n_ei == 0 and k > 0.
 */
cpra_status cpra_assemble_volume(cpra_plan_t plan, void* d_volume);

/*
 * Bytes of device workspace cpra_refine_volume needs for these parameters
 * (about N^3 x (4 x the real size + 1)).  Host-only.
 */
cpra_status cpra_refine_workspace_size(const cpra_params* params, size_t* bytes);

/*
 * 3D refinement after step D (the tomographic iterations that follow the
 * Fourier-slice insertion): starts from the step-D volume of the current
 * estimates and runs n_iter error-reduction iterations in 3D.
 *  - Fourier constraint: the Hermitian part (E(k) + conj E(-k))/2 of the
 *    inserted spectrum on every measured (k_y, k_x) cell and its mirror, for
 *    all k_z; other cells free.  As the insertion fills whole k_z lines, this
 *    is applied per z-plane in the (z, k_y, k_x) domain (2D transforms only).
 *  - Real-space constraint: the intersection over the present angles of the
 *    back-projected 2D supports (voxel (z, y, x), centred, is kept when
 *    t = floor(y cos t_n - x sin t_n + 1/2), FP64, lies in angle n's support
 *    at row z), and positivity if the plan has it.
 *  - Every shrink_every iterations (0: never) the 3D support is replaced by
 *    the 3D shrinkwrap of the volume: separable periodic Gaussian, window
 *    +-ceil(4 sigma) normalised, kept where >= threshold * its maximum.
 * Writes the refined N^3 volume ([z][y][x] centred, the plan's real type)
 * to d_volume.  work: device, 256-byte aligned, cpra_refine_workspace_size
 * bytes, the caller's.  ERR_STATE unless k mod n_ei == 0 and k > 0.
 * Synchronises the stream.
 */
cpra_status cpra_refine_volume(cpra_plan_t plan, int32_t n_iter, int32_t shrink_every, double sigma,
                               double threshold, void* work, size_t work_bytes, void* d_volume);

/*
 * cpra_refine_volume without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, computation,
 * results and errors as cpra_refine_volume; its scratch is a fixed 40 MiB
 * device array inside the library (one copy per GPU, held until the process
 * ends), enough for N <= 128 with F32 plans and N <= 64 with F64 plans;
 * larger plans return CPRA_ERR_UNSUPPORTED.  The scratch starts with no
 * required contents (every kernel writes what it reads).  Calls on one GPU
 * share that array: two calls whose device work overlaps (different
 * streams, or different host threads) race and give undefined results.
 * Calls no hipMalloc, hipFree or other allocating device routine.
 */
cpra_status cpra_refine_volume_noalloc(cpra_plan_t plan, int32_t n_iter, int32_t shrink_every, double sigma,
                                       double threshold, void* d_volume);

/* Free the plan's host memory.  The workspace stays the caller's.  In a process forked
   after the plan was created, only the host bookkeeping is dropped (no HIP call). */
cpra_status cpra_destroy(cpra_plan_t plan);

/* Last error message of the plan (or of the last failed create if plan is NULL). */
const char* cpra_last_error(cpra_plan_t plan);

/* Global iteration count k of the plan (host only). */
cpra_status cpra_iteration_count(cpra_plan_t plan, int64_t* k);

/*
 * Measurement: enable (1) or disable (0) HIP-event timing of every column
 * and row pass the plan launches (one event before, between and after the
 * two passes of each iteration, on the plan's stream).  Enabling resets the
 * accumulated times.
 */
cpra_status cpra_set_kernel_timing(cpra_plan_t plan, int32_t enable);

/*
 * Summed device time (ms) and launch counts of the column and row passes
 * recorded since timing was enabled or last read; synchronises the stream
 * and resets the accumulators.
 */
cpra_status cpra_kernel_timing(cpra_plan_t plan, double* col_ms, int64_t* col_launches, double* row_ms,
                               int64_t* row_launches);

/*
 * Host-only geometry of step D (no GPU call), for checking: for every angle
 * n and centred frequency index iu (u = iu - N/2) the native voxel indices
 * kx = floor(-u sin(theta_n) + 0.5) mod N and ky = floor(u cos(theta_n) + 0.5)
 * mod N.  kx_out, ky_out: host Np x N int32.  theta NULL: pi*n/Np.
 */
cpra_status cpra_slice_cells(int32_t N, int32_t Np, const double* theta, int32_t* kx_out, int32_t* ky_out);

/*
 * Host-only coupling table (no GPU call): for each angle, the neighbour
 * indices, rescaled weights and seam-mirror flags used at an episode
 * boundary, given which angles are present (uint8 Np, NULL = all).
 * left/right: int32 Np; w: double Np x 3 (a_-1, a_0, a_+1 after
 * renormalisation); mirror: uint8 Np x 2 (left, right).
 */
cpra_status cpra_coupling_table(const cpra_params* params, const uint8_t* present, int32_t* left,
                                int32_t* right, double* w, uint8_t* mirror);

#ifdef __cplusplus
}
#endif
#endif /* CPRA_H */
