/*
 * hp2sph.h -- C ABI of libhp2sph: HP2SPH spherical-harmonic analysis of
 * HEALPix maps on AMD Instinct MI355X (gfx950).
 *
 * The method is Algorithm 1 (HP2SPH) of Drake & Wright, "A Fast and Accurate
 * Algorithm for Spherical Harmonic Analysis on HEALPix Grids with
 * Applications to the Cosmic Microwave Background Radiation"
 * (arXiv:1904.10514):
 *   Step 1 (Sec. 3.1, eqs. upsamp, trig_expansion, interp_cond): per-ring
 *          trigonometric interpolation by FFT;
 *   Step 2 (Sec. 3.2, eqs. DFS, nufft2, normal_eq): double Fourier sphere and
 *          the least-squares fit in colatitude truncated to 4 Nside + 1 modes,
 *          with pole values from a quadratic least-squares fit to the three
 *          rings nearest each pole;
 *   Step 3 (Sec. 3.3): Slevinsky's conversion of the bivariate Fourier
 *          coefficients to spherical-harmonic coefficients, order by order,
 *          as products of Givens rotations;
 * followed by the angular power spectrum, eq. (APS) (Sec. 1).  Conventions
 * are those of Appendix A (eqs. ssph, sphip) with the Condon-Shortley phase
 * and Y_l^{-m} = (-1)^m conj(Y_l^m).
 *
 * Band: HP2SPH yields degrees l <= p = 2 Nside (the 4 Nside + 1 colatitude
 * modes of Sec. 3.2.2).  A plan asks for lmax <= 2 Nside per map; a smaller
 * lmax truncates the p-band result (values for l <= lmax are unchanged).
 *
 * Precision modes:
 *   HP2SPH_F64         every stage in FP64.
 *   HP2SPH_F32_REFINE  the colatitude fit and Legendre conversion run in FP32
 *                      (FP32 arithmetic and accumulation, FP64-built tables
 *                      rounded once); then one step of eq. (uzawa) (Sec. 2.2)
 *                      with A := HP2SPH: a0 = A32 f, r = f - S64 a0,
 *                      a1 = a0 + A32 r (FP64 add).  The ring transforms of f
 *                      and the residual are FP64: the residual is formed in
 *                      ring-Fourier space, Ring(f) - Ring(S64 a0), where
 *                      Ring(S64 a0) is evaluated exactly from the synthesis
 *                      coefficients by folding aliased modes, and rounded to
 *                      FP32 for the second FP32 pass.
 *   HP2SPH_F32         one FP32 analysis, no refinement (diagnostic).
 *   HP2SPH_EQUAL_WEIGHT
 *                      not HP2SPH: the equal-weight quadrature analysis of
 *                      eq. (healsph) (Sec. 2.2), a = (4 pi / N) S^* f, and its
 *                      Jacobi iteration, eq. (uzawa) with that A, in FP64 --
 *                      the method the paper compares HP2SPH with.  See
 *                      hp2sph_analyze_iterative.
 *
 * Conventions of every call:
 *   - All functions return an int status: HP2SPH_OK (0) or a negative code;
 *     none throws or aborts.  hp2sph_last_error() returns a thread-local
 *     message for the last failing call on that thread.
 *   - Device pointers are HIP device memory on the device that was current
 *     when the plan was created; the caller owns them.  `stream` is a
 *     hipStream_t (NULL = the default stream); work is enqueued
 *     asynchronously on it.
 *   - Maps: FP64, RING order (rings north to south, points of a ring with
 *     longitude ascending from the ring's first point, eq. healpts), the maps
 *     of a batch back to back: map b starts at sum_{b'<b} 12 nside[b']^2.
 *     16-byte aligned (rings are read and written as pairs of doubles).
 *   - a_lm: complex128 as interleaved (re, im) doubles, per map packed
 *     m-major for m >= 0: index(l, m) = m (2 lmax + 1 - m) / 2 + l,
 *     0 <= m <= l <= lmax; a_l^{-m} = (-1)^m conj(a_l^m) is implied.  The
 *     maps of a batch back to back: map b starts at
 *     sum_{b'<b} (lmax[b']+1)(lmax[b']+2)/2 complex entries.  16-byte aligned.
 *   - C_l: FP64, lmax[b]+1 values per map, back to back.
 *   - A plan is not re-entrant: two calls that share one workspace must not
 *     overlap in time (serialise them on one stream).
 */
#ifndef HP2SPH_H
#define HP2SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hp2sph_plan_s* hp2sph_plan_t;

enum {
    HP2SPH_F64 = 0,
    HP2SPH_F32_REFINE = 1,
    HP2SPH_F32 = 2,
    HP2SPH_EQUAL_WEIGHT = 3
};

enum {
    HP2SPH_OK = 0,
    HP2SPH_EINVAL = -1,      /* bad argument (size, mode, null/misaligned pointer) */
    HP2SPH_ENOMEM = -2,      /* host or device allocation of plan tables failed  */
    HP2SPH_EDEVICE = -3,     /* a HIP call failed; see hp2sph_last_error()       */
    HP2SPH_EWORKSPACE = -4,  /* workspace null, misaligned or too small          */
    HP2SPH_ESTATE = -5       /* plan handle null, never created or destroyed     */
};

/* Largest nside a plan accepts (FFT lengths and LDS budgets are sized for it). */
#define HP2SPH_MAX_NSIDE 2048

/*
 * Create a plan for `batch` maps.  nside[b] is a power of two in
 * [2, HP2SPH_MAX_NSIDE]; 0 <= lmax[b] <= 2 nside[b].  Maps with equal nside
 * form one group; each stage of an analysis is one launch over a work list
 * that holds every group (the ring transforms of nside 2048 in a launch of
 * their own, with twice the threads per workgroup), except the Givens sweeps
 * of staged groups and the equal-weight analysis, which run per group.  The
 * workspace holds every group's buffers side by side.  The set-up
 * (geometry, the colatitude least-squares solve fused with the Legendre
 * connection, Givens angles, FFT twiddles) is built here on the host in FP64
 * and copied to the device once; nothing of it is rebuilt per call.
 * If the environment variable HP2SPH_TABLE_CACHE names a directory, the host
 * tables of each nside are read from a file there when one written by the
 * same build of the library exists, and written there otherwise (one file
 * per nside, written under a temporary name and renamed; about 200 MB at
 * nside 1024, 1 GB at 2048).  A missing, unreadable or foreign file only
 * costs the rebuild; an unwritable directory is not an error.
 * On success *out receives the plan (owned by the caller; free it with
 * hp2sph_plan_destroy).  Errors: EINVAL, ENOMEM, EDEVICE.
 */
int hp2sph_plan_create(const int32_t* nside, const int32_t* lmax, int32_t batch,
                       int32_t mode, hp2sph_plan_t* out);

/*
 * Execution strategies for the colatitude fit and the conversion to
 * spherical harmonics (Steps 2-3); both compute the same a_lm up to rounding.
 *   HP2SPH_STRATEGY_STAGED  a dense GEMM per parity block (the fused
 *       colatitude least squares + order-0/1 Legendre connection, shared by
 *       all modes and maps) followed by the Givens sweeps of Slevinsky's
 *       conversion for every order m in the hot path.
 *   HP2SPH_STRATEGY_TABLES  the sweeps are applied once, at plan creation, to
 *       the columns of that matrix, giving one dense matrix per (parity
 *       block, order m) -- the "per-m precomputed tables"; the hot path is
 *       then one grouped MFMA GEMM over all orders, which also skips the polar
 *       rings that cannot carry mode m.  Costs O(nside^3) device memory
 *       (~29 GB FP64 at nside 1024).
 *   HP2SPH_STRATEGY_AUTO    tables when the group has >= 8 maps and its tables
 *       take at most a quarter of device memory and fit in the free memory;
 *       staged otherwise.
 */
enum {
    HP2SPH_STRATEGY_AUTO = 0,
    HP2SPH_STRATEGY_STAGED = 1,
    HP2SPH_STRATEGY_TABLES = 2
};

/* hp2sph_plan_create with an explicit strategy (see above).  Table
 * construction runs on the GPU (Givens sweeps on the set-up matrices) and
 * synchronises the device.  Errors: as hp2sph_plan_create, EINVAL for an
 * unknown strategy, ENOMEM if the tables do not fit in the free device memory
 * (checked before anything is built or allocated for them). */
int hp2sph_plan_create_ex(const int32_t* nside, const int32_t* lmax, int32_t batch,
                          int32_t mode, int32_t strategy, hp2sph_plan_t* out);

/* Strategy in use: STAGED or TABLES if all nside groups use it, AUTO if mixed. */
int hp2sph_plan_strategy(hp2sph_plan_t plan, int32_t* strategy);

/* Device workspace (bytes) hp2sph_analyze / hp2sph_synthesize need. */
int hp2sph_workspace_size(hp2sph_plan_t plan, size_t* bytes);

/*
 * Analysis, Algorithm 1: maps (device, FP64, read only) -> alm (device,
 * complex128, written).  workspace: device, 256-byte aligned, contents need
 * not be initialised and are clobbered; workspace_bytes: its size, at least
 * hp2sph_workspace_size (EWORKSPACE otherwise, before anything is launched).
 * For an HP2SPH_EQUAL_WEIGHT plan this is hp2sph_analyze_iterative with
 * niter = 3, the iteration count the paper gives as HEALPix's default.
 * Errors: EINVAL (null/misaligned maps or alm), EWORKSPACE, ESTATE, EDEVICE.
 */
int hp2sph_analyze(hp2sph_plan_t plan, const double* maps, double* alm,
                   void* workspace, size_t workspace_bytes, void* stream);

/*
 * hp2sph_analyze with no workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the workspace is a static device array of
 * HP2SPH_NOALLOC_WORKSPACE bytes inside the library, one per device, held
 * until the process ends (its device address is looked up when the first
 * plan is created on that device).  The call allocates nothing and records
 * no profiling events; it computes exactly what hp2sph_analyze computes.
 * Every call on a device shares that device's array and leaves its contents
 * behind: calls that overlap in time on one device (two streams, two
 * threads) race on it and must be serialised by the caller.  maps, alm,
 * stream as for hp2sph_analyze.
 * Errors: EINVAL (the plan needs more than HP2SPH_NOALLOC_WORKSPACE bytes of
 * workspace -- see hp2sph_workspace_size -- or null/misaligned maps or alm),
 * ESTATE, EDEVICE.
 */
#define HP2SPH_NOALLOC_WORKSPACE (256u << 20)
int hp2sph_analyze_noalloc(hp2sph_plan_t plan, const double* maps, double* alm, void* stream);

/*
 * Equal-weight analysis with Jacobi iterations (Sec. 2.2, eqs. healsph,
 * uzawa, richardson), for plans created with HP2SPH_EQUAL_WEIGHT:
 *   a(0) = A f,  a(k+1) = a(k) + A (f - S a(k)),  k < niter,
 * A = (4 pi / N) S^* (eq. healsph: a_l^m = (4 pi / N) sum_i conj(Y_l^m) f_i
 * over the N pixels), S the exact synthesis (hp2sph_synthesize), everything in
 * FP64.  A is the synthesis transposed: per ring the longitude sums
 * sum_q f_q e^{-i m lambda_q} for every m <= lmax (modes beyond the ring's
 * Nyquist mode alias), then the transposed evaluation of the orthonormal
 * Legendre functions at the ring colatitudes.  The iteration converges to the
 * least-squares a_lm (eq. richardson) at the rate of the spectral radius of
 * I - (4 pi / N) S^* S.  Degrees l <= lmax <= 2 nside (the plan's band).
 * maps, alm, workspace, workspace_bytes as for hp2sph_analyze;
 * 0 <= niter <= HP2SPH_MAX_JACOBI.
 * Errors: EINVAL (plan of another mode, niter out of range, null/misaligned
 * pointers), EWORKSPACE, ESTATE, EDEVICE.
 */
#define HP2SPH_MAX_JACOBI 1000
int hp2sph_analyze_iterative(hp2sph_plan_t plan, const double* maps, double* alm,
                             int32_t niter, void* workspace, size_t workspace_bytes,
                             void* stream);

/*
 * Exact synthesis, eq. (synthesis) (Sec. 2.2): alm (device, complex128,
 * layout as above, read only) -> maps (device, FP64, written), always in
 * FP64, through the same stages transposed (reverse Givens sweeps,
 * evaluation of the order-0/1 Legendre series at the ring colatitudes,
 * inverse per-ring FFT with aliasing of |m| >= n/2 onto the ring's modes).
 * This is the S of the refinement round; it is exposed as the next step the
 * paper names in Sec. 5.  Errors as for hp2sph_analyze.
 */
int hp2sph_synthesize(hp2sph_plan_t plan, const double* alm, double* maps,
                      void* workspace, size_t workspace_bytes, void* stream);

/*
 * Angular power spectrum, eq. (APS): C_l = (|a_l^0|^2 + 2 sum_{m=1}^{l}
 * |a_l^m|^2) / (2l+1) per map, FP64 accumulation in a fixed order (results
 * are bitwise reproducible).  alm device (read), cl device (written).
 * Errors: EINVAL, ESTATE, EDEVICE.
 */
int hp2sph_power_spectrum(hp2sph_plan_t plan, const double* alm, double* cl,
                          void* stream);

/* Free the plan's device tables and host state.  ESTATE for a null handle or
 * one that is not a live plan (never created, or destroyed already): handles
 * are looked up among the live plans, never dereferenced, so a second destroy
 * is reported, not undefined.  Destroying a plan while a call on it runs on
 * another thread is the caller's error. */
int hp2sph_plan_destroy(hp2sph_plan_t plan);

/* Thread-local text of the last error on the calling thread ("" if none). */
const char* hp2sph_last_error(void);

/*
 * Per-stage timing with HIP events recorded on the caller's stream around
 * every kernel launch of the plan (for benchmarks; adds two event records per
 * launch).  hp2sph_profile(plan, 1) clears the accumulators and starts
 * recording; hp2sph_profile(plan, 0) stops.  hp2sph_profile_read waits for the
 * recorded events and returns, per stage, the summed milliseconds and the
 * number of launches (arrays of length nstages, at most HP2SPH_NSTAGES).
 * Stages: 0 ring transform (S1), 1 pole values (S2), 2 analysis GEMM (S3),
 * 3 analysis Givens sweeps (S4), 4 pack a_lm, 5 unpack a_lm (in the
 * refinement: FP32 a0 widened to FP64 in place of an unpack; in the Jacobi
 * iteration on per-order tables: the update a + A r in that layout), 6 synthesis
 * sweeps, 7 synthesis GEMM, 8 inverse ring transform, 9 C_l (S5),
 * 10 residual in ring-Fourier space (the refinement's, and the Jacobi
 * iteration's longitude sums of f - S a), 11 longitude sums of the
 * equal-weight analysis, 12 its transposed-evaluation GEMM.
 * Errors: ESTATE, EINVAL, EDEVICE.
 */
#define HP2SPH_NSTAGES 13
int hp2sph_profile(hp2sph_plan_t plan, int32_t enable);
int hp2sph_profile_read(hp2sph_plan_t plan, double* ms, int32_t* launches, int32_t nstages);

/*
 * Workgroup schedules of the grouped GEMMs (the analysis GEMM of S3/S4 with
 * per-order tables or staged blocks, the synthesis GEMM of the refinement and
 * of the Jacobi iteration, the transposed-evaluation GEMM of the equal-weight
 * analysis).  A schedule only decides which workgroup runs which 128 x 128
 * output tile; every tile sums its k steps in the same order whatever runs
 * it, so results are bitwise the same under every schedule.  Not part of the
 * paper's method: a placement choice for MI355X, whose 8 XCDs (each with its
 * own L2) receive workgroups in turn by workgroup id.
 *   HP2SPH_SCHED_XCD_ROUND_ROBIN  problems (orders / parity blocks, longest
 *       first) dealt to the XCDs in turn, all tiles of a problem on one XCD
 *       (the default of a new plan for a GEMM of at least 16 problems, such as
 *       the per-order GEMMs of the tables strategy);
 *   HP2SPH_SCHED_XCD_BALANCED     each problem, longest first, to the XCD with
 *       the least work so far (tiles times k extent), tiles kept together;
 *   HP2SPH_SCHED_LINEAR           workgroup w runs tile w of the problem list
 *       (no XCD placement);
 *   HP2SPH_SCHED_LINEAR_ROWS      as LINEAR, but within a problem the row tiles
 *       of one column panel run back to back (row tile fastest), so a column
 *       panel of B is fetched once while the row tiles that need it are in
 *       flight, instead of once per row tile (the default for a GEMM of fewer
 *       than 16 problems, such as the four parity blocks of the staged
 *       strategy, where placing whole problems on XCDs would leave XCDs idle).
 */
enum {
    HP2SPH_SCHED_XCD_ROUND_ROBIN = 0,
    HP2SPH_SCHED_XCD_BALANCED = 1,
    HP2SPH_SCHED_LINEAR = 2,
    HP2SPH_SCHED_LINEAR_ROWS = 3,
    HP2SPH_NSCHED = 4
};

/* Use schedule `sched` for every GEMM of the plan (host state only: takes
 * effect for launches enqueued afterwards; a graph captured before keeps the
 * schedule it was captured with).  Errors: ESTATE, EINVAL (unknown sched). */
int hp2sph_set_schedule(hp2sph_plan_t plan, int32_t sched);

/*
 * Autotuner: for each GEMM that hp2sph_analyze launches (GEMMs in launch
 * order; the analysis modes merge every nside group into one GEMM per role),
 * times hp2sph_analyze of the caller's maps under each candidate schedule of
 * that GEMM, the others held at their current choice, and keeps the fastest;
 * then the same for the launch options of the fold and the pack
 * (hp2sph_set_option).  A candidate replaces the current choice only
 * when it is more than 0.5 % faster (the run-to-run spread of a timed
 * analysis).  Each timing is the fastest of `reps` analyses (HIP events on
 * `stream`, after one untimed analysis).  Synchronous: returns after the last
 * timed run, with alm holding hp2sph_analyze(maps) and *best_ms (if not null)
 * the time of one analysis under the chosen schedules.  Stage profiling
 * (hp2sph_profile) is paused meanwhile.  The choices are remembered for the
 * plan's shape (device, mode, and each group's nside, map count and
 * strategy): a plan of that shape created later in the process starts with
 * them, and so does one in a later process when the environment variable
 * HP2SPH_TUNE_CACHE names a file (read at the first plan creation, appended
 * to by each autotune; an unreadable file is ignored).  maps, alm,
 * workspace, workspace_bytes, stream as for hp2sph_analyze; 1 <= reps <=
 * HP2SPH_MAX_TUNE_REPS.
 * Errors: as hp2sph_analyze, EINVAL for reps out of range, EDEVICE.
 */
#define HP2SPH_MAX_TUNE_REPS 100
int hp2sph_autotune(hp2sph_plan_t plan, const double* maps, double* alm, void* workspace,
                    size_t workspace_bytes, void* stream, int32_t reps, double* best_ms);

/* Schedules in use by the GEMMs hp2sph_analyze launches, in the order the
 * autotuner visits them: writes min(cap, count) ids to out (may be null when
 * cap is 0) and the count to *count.  Errors: ESTATE, EINVAL. */
int hp2sph_schedules(hp2sph_plan_t plan, int32_t* out, int32_t cap, int32_t* count);

/*
 * Launch options of the work-list stages.  The stages of an analysis run as
 * one launch over a work list that holds every nside group of the plan
 * (items grouped by nside, largest first).  Results are bitwise the same
 * under every value of the first three; HP2SPH_OPT_RING_THREADS changes the
 * FFT's pass structure, so its results agree to rounding (a few ulp of the
 * ring coefficients), not bit for bit.  hp2sph_autotune chooses them after
 * the GEMM schedules and remembers its choices per plan shape.  Host state
 * only, like hp2sph_set_schedule.
 *   HP2SPH_OPT_FOLD_GRID  work grid of the refinement's residual fold (an
 *       item is one ring pair of 16 maps, or of one map in the staged
 *       layout): 0 for one workgroup per item (the default), or g >= 8 for a
 *       persistent launch of g workgroups (rounded down to a multiple of 8,
 *       so that each item keeps its XCD) that walk the list; the autotuner
 *       tries 0, 2 and 4 workgroups per compute unit.
 *   HP2SPH_OPT_PACK_MAPS  maps per pack tile (tile shape of the a_lm pack in
 *       the mode-major layout of the per-order tables: 64 degrees x 16, 32 or
 *       64 maps; 32 by default); the autotuner tries all three.
 *   HP2SPH_OPT_RING_ORDER  order in which the ring transform's items (one
 *       ring pair of one map each) meet the workgroups: 0 (default) deals ring
 *       pairs to the 8 XCDs in turn and runs the maps of a pair back to back
 *       on its XCD; 1 runs pairs in order, maps of a pair back to back; 2
 *       runs maps in order, all pairs of a map back to back.  The autotuner
 *       tries all three (not for HP2SPH_EQUAL_WEIGHT plans).
 *   HP2SPH_OPT_RING_THREADS  workgroup size of the ring transform for the
 *       groups up to nside 1024: 256 (default: up to 16 complex values per
 *       thread, radix-16 passes) or 512 (up to 8 values per thread, radix-8
 *       passes: one pass more, twice the waves per compute unit).  Groups
 *       at nside 2048 always run 512 threads with 16 values each.  The
 *       autotuner tries both (not for HP2SPH_EQUAL_WEIGHT plans).
 * Errors: ESTATE, EINVAL (unknown option, value out of range, null output).
 */
enum {
    HP2SPH_OPT_FOLD_GRID = 0,
    HP2SPH_OPT_PACK_MAPS = 1,
    HP2SPH_OPT_RING_ORDER = 2,
    HP2SPH_OPT_RING_THREADS = 3
};
int hp2sph_set_option(hp2sph_plan_t plan, int32_t option, int32_t value);
int hp2sph_get_option(hp2sph_plan_t plan, int32_t option, int32_t* value);

/*
 * Host-only inspection of a schedule (no GPU needed): the workgroup -> (problem,
 * tile) map that schedule `sched` gives a list of n GEMM problems of M[i] x N[i]
 * outputs and extent K[i] in launch order, as the GEMM kernel reads it: entry w
 * is the pair (problem, tile within the problem) at out[2w], out[2w + 1], or
 * (-1, -1) for a workgroup that has no tile.  Tiles are 128 x 128 and numbered
 * row-major within a problem.  Writes min(capacity, 2 * workgroups) entries
 * and sets *count to 2 * workgroups.  Errors: EINVAL (unknown sched, n < 0,
 * null arrays, a non-positive size).
 */
int hp2sph_schedule_map(int32_t sched, const int32_t* M, const int32_t* N, const int32_t* K, int32_t n,
                        int32_t* out, int64_t capacity, int64_t* count);

/*
 * Host-only check of the grouped GEMMs' memory accesses (no GPU needed; used
 * by tests).  Builds the GEMM problem lists a plan of `nmaps` maps of one
 * `nside` with `mode` and `strategy` (STAGED or TABLES) would launch, over
 * stand-in table addresses of the sizes the plan allocates, and checks them:
 * every problem's A rows inside its table, B and C inside their workspace
 * regions, and a replay of the kernel's staging addresses (the same offset
 * functions the kernel runs) for every tile of every problem -- each element
 * inside the problem must be read through an offset below its k step's
 * descriptor size and inside the allocation, each element outside it must get
 * an offset the descriptor range check turns into zero.  Writes the number
 * of checks to *checked, of failures to *violations (the first one described
 * in hp2sph_last_error()) and of vector reads of the zero row padding of the
 * per-order tables to *padding.  Errors: EINVAL, ENOMEM.
 */
int hp2sph_gemm_check(int32_t nside, int32_t nmaps, int32_t mode, int32_t strategy,
                      int64_t* checked, int64_t* violations, int64_t* padding);

/*
 * Host-only inspection of the set-up tables (no GPU needed; used by tests).
 * Writes up to `capacity` doubles of table `table` for `nside` into `out`
 * and the full element count into *count (out may be NULL to query the
 * count).  Tables:
 *   HP2SPH_TABLE_RINGS    per ring r = 1..4nside-1: z, n, phi0, start (4 doubles each)
 *   HP2SPH_TABLE_POLE     the three pole weights (quadratic extrapolation in z
 *                         of the three nearest ring means to the pole)
 *   HP2SPH_TABLE_ANALYSIS block `block` (0..3 = (k even, +), (k even, -),
 *                         (k odd, +), (k odd, -)): the matrix mapping the
 *                         half-ring data h = 0..2nside to the order-0/1
 *                         Legendre coefficients, stored [h][l'] (row-major,
 *                         2nside+1 rows, (number of l of the block) columns)
 *   HP2SPH_TABLE_SYNTHESIS block `block`: the evaluation matrix, stored
 *                         [l'][h]
 *   HP2SPH_TABLE_GIVENS   block `block`: (c, s) for sweep t = 1.. and chain
 *                         position l' >= t, stored as rows t = 1..T of
 *                         (ntop+1) pairs (entries l' < t are zero)
 * Errors: EINVAL (bad nside/table/block), ENOMEM.
 */
enum {
    HP2SPH_TABLE_RINGS = 0,
    HP2SPH_TABLE_POLE = 1,
    HP2SPH_TABLE_ANALYSIS = 2,
    HP2SPH_TABLE_SYNTHESIS = 3,
    HP2SPH_TABLE_GIVENS = 4
};
int hp2sph_host_table(int32_t nside, int32_t table, int32_t block, double* out,
                      int64_t capacity, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* HP2SPH_H */
