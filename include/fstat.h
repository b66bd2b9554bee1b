/*
 * fstat.h - C ABI of the MI355X (gfx950) F-statistic search library.
 *
 * The library evaluates the F-statistic of an all-sky search for periodic
 * gravitational waves over a grid of (sky position, spindown) templates and
 * registers every frequency bin above a threshold as a candidate.  The
 * operation is the core loop of the paper's search code (Sect. 2, Fig. 3):
 * per sky position, amplitude and phase demodulation and resampling; per
 * spindown, spindown demodulation, two FFTs with 2x Fourier interpolation,
 * the F-statistic on every bin, and threshold crossings as candidates of
 * five numbers (sky position, frequency, spindown, F).
 *
 * Conventions shared by every call:
 *  - Every call returns an fstat_status; nothing aborts or throws across the
 *    ABI.  fstat_last_error() gives a text for the last failure on a plan.
 *  - "device" pointers are HIP device memory (for example from PyTorch);
 *    "host" pointers are ordinary process memory.
 *  - The caller owns every input buffer and keeps it alive and unchanged
 *    until the stream work that reads it has completed.  The library never
 *    frees caller memory.  The plan owns its kernels' tables, its candidate
 *    buffer and (unless the caller supplies one) its workspace.
 *  - Calls on one plan are not thread-safe; distinct plans are independent.
 *  - Stream arguments are hipStream_t passed as void*; NULL is the null stream.
 *    Work "asynchronous on `stream`" starts after the work already enqueued on
 *    that stream and finishes before the work enqueued on it afterwards.  Parts
 *    of it may run on streams the plan or the network owns (default priority),
 *    joined to `stream` with events: the per-sky stage of the next sky batch
 *    beside the current batch's templates, the next batch's convolutions beside
 *    the current batch's dense layers.
 */
#ifndef FSTAT_H
#define FSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fstat_plan_s* fstat_plan_t;

typedef enum {
  FSTAT_OK = 0,
  FSTAT_E_INVAL = 1,            /* an argument is out of range or inconsistent */
  FSTAT_E_NOMEM = 2,            /* a device or host allocation failed */
  FSTAT_E_ADMISSION = 3,        /* a segment's minimum workspace exceeds the budget */
  FSTAT_E_OVERFLOW = 4,         /* more candidates than the buffer holds (true count reported) */
  FSTAT_E_DEVICE = 5,           /* a HIP runtime call failed (no usable GPU, launch error) */
  FSTAT_E_STATE = 6,            /* call not valid in the plan's current state */
  FSTAT_E_NOT_IMPLEMENTED = 7
} fstat_status;

/* Arithmetic of the path.  FP64: every step in double precision.  MIXED:
 * time of arrival, phases, spline positions and reductions in FP64; the
 * demodulated series, resampling values, FFTs and F in FP32. */
typedef enum { FSTAT_PREC_FP64 = 0, FSTAT_PREC_MIXED = 1 } fstat_precision;

/* F-statistic form.  SIMPLIFIED: 2F = 2/(N sigma^2) (|Fa|^2/A + |Fb|^2/B),
 * A = <a^2>, B = <b^2>.  FULL adds the cross term C = <ab>:
 * 2F = 2/(N sigma^2) (B|Fa|^2 + A|Fb|^2 - 2C Re(Fa Fb*)) / (AB - C^2). */
typedef enum { FSTAT_FORM_SIMPLIFIED = 0, FSTAT_FORM_FULL = 1 } fstat_form;

/* One data segment: one (frame, band) pair of the paper (Sect. 2, Eq. 1). */
typedef struct {
  int64_t n;            /* samples, 2048 <= n <= 2^19 */
  double dt;            /* sampling interval, s, > 0 */
  double f_off;         /* lower band edge, Hz (Eq. 1); the series is heterodyned by it */
  double sigma2;        /* noise variance of x, > 0 */
  const double* x;      /* device, n doubles: the narrowband series */
  const double* r_ssb;  /* device, 3*n doubles: detector-to-SSB vector in light-seconds,
                           component-major (x[0..n), y[0..n), z[0..n)), equatorial frame;
                           the content of the paper's ephemeris file (Sect. 2) */
  double lat;           /* detector latitude, rad */
  double gamma;         /* arm-bisector orientation, rad counter-clockwise from local East */
  double phi_r;         /* local sidereal angle of the detector at the first sample, rad */
} fstat_segment;

typedef struct {
  int32_t nfft;                   /* FFT length, power of two >= 2n; 0 = nextpow2(2n) per segment */
  int32_t k_min, k_max;           /* searched bins [k_min, k_max); 0,0 = [0, nfft/2) */
  double threshold_2F;            /* a bin is a candidate when 2F > threshold (strict) */
  int32_t precision;              /* fstat_precision */
  int32_t form;                   /* fstat_form */
  int64_t candidate_capacity;     /* entries of the device candidate buffer, >= 1 */
  size_t workspace_budget_bytes;  /* admission limit for the workspace; 0 = no limit */
  int32_t templates_per_launch;   /* spindown templates per FFT launch; 1 = one template per
                                     launch; 0 = the library's choice (sized for the plan's
                                     longest transform: a segment with a shorter one takes
                                     proportionally more per launch, at most 4096) */
  int32_t skies_per_batch;        /* sky positions prepared together; 0 = the library's choice */
  int32_t use_graph;              /* 1: capture each search call as a HIP graph and replay it while
                                     the call's arguments are unchanged */
  const char* tuning_cache_path;  /* autotuner results file (read by fstat_plan when both batch
                                     sizes are 0, written by fstat_autotune); NULL = none */
  int32_t interbinning;           /* 0: the template transforms are nfft points long (the 2x
                                     interpolation by zero-padding, Sect. 2).  1: they are nfft/2
                                     points long; bin 2k of the nfft grid is bin k of that transform
                                     (the same value), bin 2k+1 is estimated from its neighbours as
                                     c (X_k - X_{k+1 mod nfft/2}) for both series, with c chosen so
                                     that a sinusoid midway between two bins over the n samples comes
                                     out exactly (c = n sin h / (2 sin(n h) sin((n-1) h)),
                                     h = pi/nfft; about pi/4 when n = nfft/2).  Halves the template
                                     stage's memory traffic; the odd bins are an approximation
                                     (exact for a sinusoid midway between bins; odd bins of pure
                                     noise have a larger mean than even ones).  Both precisions
                                     (FP64, and mixed precision at nfft = 2^20, store the
                                     transforms, then form 2F in a pass of their own); needs
                                     nfft >= 2^13. */
} fstat_options;

/* The paper's five numbers of a candidate (Sect. 2). */
typedef struct { double f_hz, fdot, alpha, delta, twoF; } fstat_candidate;

/* Integer key of a candidate: which search call, segment, sky index, spindown
 * index and frequency bin produced it; bins are f_hz = f_off + bin/(nfft dt).
 * vet_score is the vetting network's score in (0, 1) after
 * fstat_plan_vet_candidates, NaN otherwise. */
typedef struct { int32_t search, segment, sky, fdot_idx, bin; float vet_score; } fstat_candidate_key;

/* Fill *opt with defaults: nfft 0, all bins, threshold 20, MIXED, SIMPLIFIED,
 * capacity 1<<24, no budget, library-chosen batching, graphs on. */
void fstat_options_default(fstat_options* opt);

/* Create a plan for nseg segments (host array, copied): the problem statement of
 * Sect. 2 (data segments of Eq. 1's bands, their ephemeris, the F threshold).
 * Validates every
 * argument, chooses FFT factorizations and batch sizes, and performs the
 * admission check: FSTAT_E_ADMISSION when even one sky and one template of
 * the largest segment need more workspace than workspace_budget_bytes.
 * Allocates the plan's tables and candidate buffer on the current device.
 * On failure *out_plan is NULL. */
fstat_status fstat_plan(const fstat_segment* segs, int32_t nseg, const fstat_options* opt,
                        fstat_plan_t* out_plan);

/* Workspace bytes the plan needs (its chosen batch sizes; memory of the search
 * loop of Sect. 2 held between calls). */
fstat_status fstat_plan_workspace_size(fstat_plan_t plan, size_t* bytes);

/* Hand the plan a caller-owned device workspace of at least
 * fstat_plan_workspace_size bytes, 256-byte aligned.  Without this call the
 * plan allocates its own on first use. */
fstat_status fstat_plan_set_workspace(fstat_plan_t plan, void* dev_ptr, size_t bytes);

/* The search loop of Sect. 2 (Fig. 3): for every sky position, demodulation and
 * resampling; for every spindown, spindown demodulation, the two FFTs twice as long
 * as the data, F on every bin and each bin above the threshold as a candidate.
 * Enqueue the search of every (sky, spindown) template on one segment
 * (segment >= 0) or on every segment of the plan (segment = -1) with the
 * same template lists.  alpha, delta (nsky) and fdot (nfdot) are device
 * arrays of doubles.  Asynchronous on `stream`; candidates are appended to
 * the plan's device buffer and tagged with this call's search index.  The
 * lists may be released once the stream has passed this work. */
fstat_status fstat_search_batch(fstat_plan_t plan, int32_t segment,
                                const double* alpha, const double* delta, int32_t nsky,
                                const double* fdot, int32_t nfdot, void* stream);

/* The candidates of Sect. 2: every crossing as the five numbers frequency,
 * spindown, sky position (alpha, delta) and 2F, plus its integer key.
 * Wait for the plan's work, then copy out and drain the candidates found
 * since the previous call, sorted by key (search, segment, sky, fdot_idx,
 * bin).  out / keys are host arrays of `capacity` entries (either may be
 * NULL).  *n_found receives the true number of crossings, also when it
 * exceeds the device buffer or `capacity`; then FSTAT_E_OVERFLOW is
 * returned and the first min(capacity, stored) entries in key order are
 * written.  With out and keys both NULL the call only reports the count and
 * drains the buffer (FSTAT_E_OVERFLOW only if the device buffer overflowed).
 * When the device buffer overflowed, which crossings were kept is
 * unspecified.  The ordering and the records are formed on the device in memory the
 * plan allocates at its first full drain and keeps until fstat_destroy (about 36 bytes
 * per stored crossing and 12 per template of the drained searches, plus 64 per
 * crossing copied out); FSTAT_E_NOMEM if it cannot, with the candidates kept for a
 * later call (a count-only drain needs none).  Copies into page-locked host arrays are
 * the fastest. */
fstat_status fstat_candidates(fstat_plan_t plan, fstat_candidate* out, fstat_candidate_key* keys,
                              int64_t capacity, int64_t* n_found);

/* F on every bin (Sect. 2), stored instead of thresholded.
 * Enqueue 2F over bins [k_min, k_max) of every template of one segment into
 * the device array out, laid out [sky][fdot][bin - k_min], float for MIXED
 * and double for FP64.  Same kernels as the search, with the threshold
 * stage replaced by a store.  Asynchronous on `stream`. */
fstat_status fstat_twoF_spectrum(fstat_plan_t plan, int32_t segment,
                                 const double* alpha, const double* delta, int32_t nsky,
                                 const double* fdot, int32_t nfdot, void* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): fstat_twoF_spectrum with
 * the same arguments, layout and results, run on a static device scratch of
 * FSTAT_STATIC_SCRATCH_BYTES instead of the plan's workspace.  Each GPU the library
 * runs on holds its own such scratch, from when the library's device code is loaded
 * on it until the process ends.  The call allocates nothing and creates nothing: every launch goes
 * to `stream` in order (no graph, no second stream, no timing events), with the
 * plan's batch sizes shrunk until the workspace of the plan's largest segment fits
 * the scratch.  FSTAT_E_INVAL when even one sky position and one template do not fit
 * (mixed precision fits nfft <= 2^19, FP64 nfft <= 2^18), or for the arguments
 * fstat_twoF_spectrum rejects; FSTAT_E_STATE when the plan's device is not current.
 * Every call on one GPU uses that GPU's one scratch, whatever the plan: calls that
 * overlap on one GPU (on different streams, threads or plans) race on it and give
 * wrong spectra, so order them on one stream.  Nothing in the scratch needs to start
 * at zero: every kernel writes what it reads.  Asynchronous on `stream`. */
#define FSTAT_STATIC_SCRATCH_BYTES (64ull << 20)
fstat_status fstat_twoF_spectrum_static(fstat_plan_t plan, int32_t segment, const double* alpha,
                                        const double* delta, int32_t nsky, const double* fdot, int32_t nfdot,
                                        void* out, void* stream);

/* The per-sky steps of Sect. 2 (direction, Roemer delay, a(t), b(t), phase
 * demodulation, resampling with the FFT and splines), exposed one by one.
 * Per-sky intermediates of one sky position, for stage-by-stage checks.
 * Device outputs (complex values interleaved re, im; float for MIXED,
 * double for FP64), any may be NULL:
 *   abc    3 doubles: A = <a^2>, B = <b^2>, C = <ab>
 *   za, zb n complex: amplitude- and phase-demodulated series
 *   ua, ub nfft complex: 2x upsampled series
 *   zta, ztb n complex: resampled series on the barycentric grid
 * Synchronous: waits for `stream`, runs the sky stage on it and returns once the
 * outputs are written.  Uses the plan's workspace (allocating it on first use). */
fstat_status fstat_sky_stages(fstat_plan_t plan, int32_t segment, double alpha, double delta,
                              double* abc, void* za, void* zb, void* ua, void* ub,
                              void* zta, void* ztb, void* stream);

/* ---- Lattice grid (Sect. 2: grid generating matrix, sky loop over the
 * integers n, m, spindown loop over s; Sect. 1.1: grid points reconciled
 * with the Fourier frequencies, resampling once per sky position) ----
 *
 * Grid points are the integer combinations k M0 + s M1 + n M2 + m M3 of the
 * rows of M over the phase parameters (w0, w1, w2, w3):
 *   w0 = 2 pi f dt        frequency above f_off, radians per sample;
 *   w1 = pi fdot dt^2     spindown: phase w1 j^2 at sample j;
 *   (w2, w3) = W (x_e, y_e), W = 2 pi f_ref (1 AU / c): the source
 *                         direction's components in the ecliptic plane,
 *                         x_e toward the vernal equinox.
 * dt is the sampling interval of the segment searched.  Row 0 is the
 * frequency vector: (w_F, 0, 0, 0) with w_F a whole number of bins
 * 2 pi / nfft of every segment searched.  Row 1 is the spindown vector, with
 * no sky components.  Rows 2 and 3 are the sky vectors.  A sky point is on
 * the sky when x_e^2 + y_e^2 <= 1; its third ecliptic component is
 * hemisphere * sqrt(1 - x_e^2 - y_e^2), and the obliquity epsilon turns
 * ecliptic axes into equatorial ones. */
typedef struct {
  double M[16];      /* row-major 4 x 4: M[4 r + c] is component c of row r */
  double epsilon;    /* obliquity of the ecliptic, rad */
  double f_ref;      /* Hz, > 0: scale W of the sky coordinates (the band's upper edge) */
} fstat_lattice;

/* Host only.  The smallest box n in [box[0], box[1]], m in [box[2], box[3]]
 * that holds every (n, m) on the sky.  FSTAT_E_INVAL for a NULL argument,
 * non-finite values or parallel sky rows. */
fstat_status fstat_lattice_sky_range(const fstat_lattice* lat, int32_t box[4]);

/* Sky loop of the grid (Sect. 2, "sky position recovered"): every (n, m) of
 * the box (host array, as above) whose point is on the sky, in order of n,
 * then m, on the hemisphere given (+1 north, -1 south of the ecliptic).
 * Point i (i < capacity) is written to the device arrays alpha[i], delta[i]
 * (rad, alpha in [0, 2 pi]), w_freq[i], w_spin[i] (the w0 and w1 components
 * of n M2 + m M3) and nm[2 i], nm[2 i + 1] (nm may be NULL).  The device
 * int64 *count receives the number of points on the sky, also when it
 * exceeds capacity.  At most 2^26 box points.  Asynchronous on `stream`;
 * the caller owns every array.  FSTAT_E_INVAL for bad arguments. */
fstat_status fstat_lattice_sky(const fstat_lattice* lat, int32_t hemisphere, const int32_t box[4],
                               int64_t capacity, double* alpha, double* delta, double* w_freq,
                               double* w_spin, int32_t* nm, int64_t* count, void* stream);

/* Search of the lattice templates: the nsky sky points of device arrays
 * alpha, delta, w_freq, w_spin (as written by fstat_lattice_sky) times the
 * spindown integers s = s_lo .. s_hi, on one segment or on every segment
 * (segment = -1).  Template (i, s) has spindown phase coefficient
 * w1 = s M1[1] + w_spin[i] and frequency component w0 = s M1[0] + w_freq[i];
 * the FFT evaluates the frequencies f_off + (k + u) / (nfft dt), where u is
 * the fraction of w0 nfft / (2 pi) above the integer below it (a value within
 * 1e-6 below an integer counts as that integer).  Candidates carry
 * fdot_idx = s - s_lo, f_hz = f_off + (bin + u) / (nfft dt) and
 * fdot = w1 / (pi dt^2).  With spectrum NULL, candidates are registered as by
 * fstat_search_batch; otherwise 2F of one segment is stored to spectrum as by
 * fstat_twoF_spectrum.  FSTAT_E_INVAL when row 0 or row 1 breaks the
 * constraints above.  Asynchronous on `stream`. */
fstat_status fstat_search_lattice(fstat_plan_t plan, int32_t segment, const fstat_lattice* lat,
                                  const double* alpha, const double* delta, const double* w_freq,
                                  const double* w_spin, int32_t nsky, int32_t s_lo, int32_t s_hi,
                                  void* spectrum, void* stream);

/* Per-kernel timing.  When enabled, the plan brackets each launch of the
 * kernel classes below with HIP events on the launch stream;
 * fstat_profile_read waits for them and reports the number of launches and
 * their summed duration since the last reset.  While enabled, searches run
 * eagerly (no graphs) and entirely on the caller's stream, so that each timed
 * launch runs alone. */
typedef enum {
  FSTAT_KERNEL_SKY_PREP = 0,      /* demodulation + antenna sums */
  FSTAT_KERNEL_RESAMPLE = 1,      /* upsampling FFTs + spline */
  FSTAT_KERNEL_TEMPLATE_A = 2,    /* spindown chirp + first FFT pass */
  FSTAT_KERNEL_TEMPLATE_B = 3,    /* second FFT pass + F + threshold + compaction */
  FSTAT_KERNEL_COUNT = 4
} fstat_kernel_class;
fstat_status fstat_profile_enable(fstat_plan_t plan, int32_t on);
fstat_status fstat_profile_read(fstat_plan_t plan, int32_t kernel_class, int64_t* launches,
                                double* total_ms, int32_t reset);

/* Plan facts: FFT length nfft of the bin grid and factors P x Q of the
 * template transforms of a segment (P Q = nfft, or nfft/2 with
 * interbinning), the batch
 * sizes in force, the first-pass kernel variant (0: series one after the
 * other through one LDS tile, 1: both series in LDS at once) and the
 * second-pass variant (0: one launch-wide grid of row tiles; 1: about one
 * resident round of wavefronts that walk the launch's rows, prefetching the
 * next row and staging candidates in LDS; variant 1 applies to the mixed
 * precision path with P <= 512, other segments use row tiles; with
 * interbinning the mixed-precision second pass with P <= 512 is always a walk
 * of wavefronts over chunks of consecutive rows; FP64 and P = 1024 use row
 * tiles that store the transforms for a separate 2F pass).  Any output pointer
 * may be NULL. */
fstat_status fstat_plan_info(fstat_plan_t plan, int32_t segment, int32_t* nfft, int32_t* p,
                             int32_t* q, int32_t* templates_per_launch, int32_t* skies_per_batch,
                             int32_t* pass_a_variant, int32_t* pass_b_variant);

/* Autotuner: time the search of `segment` (its own data, a synthetic grid of
 * 128 sky positions and 256 spindowns) for candidate templates-per-launch, skies-per-batch and
 * first-pass kernel variants that fit the workspace budget, keep the fastest,
 * and append it to options.tuning_cache_path if set (one line per device,
 * FFT length and precision: "<device> <nfft> <precision + 2 interbinning>
 * <templates per launch> <skies per batch> <pass_a_variant + 2
 * pass_b_variant>"; the last
 * matching line wins).  Runs synchronously on `stream` for roughly
 * budget_ms, and at least one warm-up and one timed search per candidate
 * (about 1.5 s at nfft = 2^18).  Must be called before fstat_plan_set_workspace: the workspace
 * size changes with the batch sizes (query it again afterwards), and before
 * fstat_plan_attach_vetter.  Candidates found by the trial searches are
 * discarded. */
fstat_status fstat_autotune(fstat_plan_t plan, int32_t segment, double budget_ms, void* stream);

/* Release the plan and everything it owns (waits for its work first).
 * NULL is accepted; a second destroy of the same handle is undefined, as
 * for free(). */
fstat_status fstat_destroy(fstat_plan_t plan);

/* ---- Candidate vetting (a learned score for threshold crossings; not part of
 * the paper's method, whose threshold stays the fallback) -------------------
 * The network scores the 256-bin 2F window centred on a crossing:
 *   u = log(1 + 2F) - log 5; three "same" convolutions of width 7 with 32
 *   channels and ReLU (1 -> 32 -> 32 -> 32); flattened position-major
 *   (x[p*32 + c]); dense 8192 -> 128 -> 128 -> 1 with ReLU; logit.
 * Parameters are one FP32 vector (the master copy), in the order w1[32][1][7],
 * b1[32], w2[32][32][7], b2, w3[32][32][7], b3, w4[128][8192], b4[128],
 * w5[128][128], b5, w6[1][128], b6[1]; the matrix products use BF16 copies of
 * weights and activations with FP32 accumulation. */
typedef struct fstat_vet_s* fstat_vet_t;

/* Number of parameters (1 080 001). */
int64_t fstat_vet_param_count(void);

/* A network for batches of up to max_batch patches, parameters zero until set. */
fstat_status fstat_vet_create(int32_t max_batch, fstat_vet_t* out);

/* Host FP32 parameter vector in and out (n = fstat_vet_param_count()); setting
 * resets the optimiser state. */
fstat_status fstat_vet_set_params(fstat_vet_t vet, const float* params, int64_t n);
fstat_status fstat_vet_get_params(fstat_vet_t vet, float* params, int64_t n);

/* Logits of n patches (device [n][256] 2F values) into device logits[n]; any n
 * (processed in batches of max_batch).  Asynchronous on `stream`.  The first
 * convolution runs on the matrix cores with input and weights split into BF16
 * pairs (hi + lo, about FP32 before its output's BF16 rounding), so its outputs can
 * differ in the last BF16 place from the FP32 first layer of fstat_vet_gradient. */
fstat_status fstat_vet_forward(fstat_vet_t vet, const float* patches, int64_t n, float* logits, void* stream);

/* Mean binary cross-entropy of n <= max_batch patches with device labels[n]
 * (0 or 1) and its gradient.  loss (device, 1 float) and grad (device, param
 * count floats) may be NULL; the gradient is kept for fstat_vet_adam_step. */
fstat_status fstat_vet_gradient(fstat_vet_t vet, const float* patches, const float* labels, int64_t n,
                                float* loss, float* grad, void* stream);

/* One Adam step with the last gradient (bias-corrected). */
fstat_status fstat_vet_adam_step(fstat_vet_t vet, float lr, float beta1, float beta2, float eps, void* stream);

fstat_status fstat_vet_destroy(fstat_vet_t vet);

/* Attach a network to a plan: from now on every search also stores, right after
 * each F kernel launch, the 256-bin 2F window of each new crossing (up to
 * patch_capacity <= candidate_capacity crossings per drain).  NULL detaches.
 * The plan keeps using the network until it is detached or the plan destroyed. */
fstat_status fstat_plan_attach_vetter(fstat_plan_t plan, fstat_vet_t vet, int64_t patch_capacity);

/* Score the stored windows of the crossings found since the last drain with the
 * attached network, in batches of the network's max_batch on `stream`.  Waits for
 * the plan's searches before it starts and for the scoring before it returns;
 * fstat_candidates then reports the scores in the keys (NaN for crossings beyond
 * patch_capacity). */
fstat_status fstat_plan_vet_candidates(fstat_plan_t plan, void* stream);

/* Static text for a status code. */
const char* fstat_strerror(fstat_status status);

/* Text of the last failure on this plan ("" if none); with plan NULL, the
 * global text of the last failed call that has no plan (fstat_plan,
 * fstat_lattice_sky_range, fstat_lattice_sky).  Valid until the next call. */
const char* fstat_last_error(fstat_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* FSTAT_H */
