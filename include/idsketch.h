/*
 * idsketch: CountSketch / TensorSketch interpolative decomposition on AMD
 * Instinct MI355X (gfx950).
 *
 * The method (Malik & Becker, "Fast randomized matrix and tensor
 * interpolative decomposition using CountSketch"):
 *   matrix ID  A ~= A[:, J] P      (problem statement, Section 1.2.1)
 *     Algorithm 2: draw a CountSketch S, form Y = S A implicitly, then run
 *     Algorithm 1 (rank-K column-pivoted QR of Y, J from the pivots,
 *     P = [I, R11^{-1} R12] Pi^T) on Y.  This library optionally inserts a
 *     Gaussian projection Y = G (S A) between the two stages.
 *   tensor ID  X_hat = sum_k lambda_hat_k X^(j_k)   (Section 1.2.2, eq. X*)
 *     Algorithm 3: TensorSketch Y = T M of the implicit matrix
 *     M = (Khatri-Rao of the factors) diag(lambda) via per-mode CountSketch,
 *     FFT, Hadamard product and inverse FFT; Algorithm 1 on Y; then
 *     lambda_hat_k = lambda_{j_k} sum_r p_kr.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer on the current HIP device,
 *     owned by the caller, unless stated otherwise.  The library never
 *     allocates or frees user-visible memory; scratch space comes from the
 *     caller's workspace (size from the matching *_workspace_size call,
 *     256-byte aligned).
 *   - All calls are asynchronous on `stream` (a hipStream_t passed as void*;
 *     NULL = the default stream).  Argument errors are detected on the host
 *     and returned before anything is launched.  Results (including k_eff)
 *     are valid once the stream has been synchronised.
 *   - Indices are 0-based (the paper's [m] = {1..m}).  Dense matrices are
 *     row-major unless stated otherwise.
 *   - Random maps: the CountSketch bucket h(i) and sign D_ii of row i come
 *     from a counter-based SplitMix64 stream (Steele, Lea & Flood 2014):
 *       key   = mix64(seed XOR mix64(tag))
 *       z_i   = mix64(key + (i+1) * 0x9e3779b97f4a7c15)
 *       h(i)  = (hi32(z_i) * L) >> 32,   D_ii = bit0(z_i) ? -1 : +1
 *     TensorSketch mode n uses tag (tag_base + n + 1).
 *   - Errors: a nonzero ids_status; ids_last_error() gives a message for the
 *     calling thread.
 */
#ifndef IDSKETCH_H
#define IDSKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ids_status;
enum {
    IDS_OK = 0,
    IDS_EINVAL = 1,      /* bad sizes, null pointers, unsupported shapes */
    IDS_EDTYPE = 2,      /* unsupported dtype combination */
    IDS_EWORKSPACE = 3,  /* workspace missing, too small or misaligned */
    IDS_EHIP = 4,        /* a HIP runtime call failed (message has details) */
    /* codes written to a device status word (never returned by a call): */
    IDS_ETIMEOUT = 5,    /* a device-wide wait of the pivoted QR gave up; k_eff = -1,
                            J, P and lambda_hat are undefined (never expected unless
                            forced with ids_set_wait_limit(0)) */
    IDS_ERANKDEF = 6,    /* the pivoted QR met a zero trailing norm before step k
                            (rank deficiency, Fact 1 needs K < rank): k_eff < k, the
                            rank-k_eff ID is returned */
    IDS_ENONFINITE = 7   /* a non-finite value (NaN, infinity, or a column norm that
                            overflows) in the sketch; results are undefined */
};

/* element types */
enum { IDS_F64 = 0, IDS_F32 = 1, IDS_BF16 = 2 };
/* matrix formats */
enum { IDS_DENSE = 0, IDS_CSR = 1 };
/* ids_sketch_cfg.flags */
#define IDS_HASH_FULLRANK 1u /* modified map h~ = f o pi (Remark 2, Prop. 4) */
#define IDS_CHECK_FINITE 2u  /* scan the finished sketch Y and write IDS_OK or
                                IDS_ENONFINITE to cfg->status (a NaN or infinity
                                anywhere in A reaches Y through its bucket) */
#define IDS_DETERMINISTIC 4u /* CSR A: add the entries of a bucket in increasing
                                row order (a row's entries in storage order), the
                                order of the definition of S A, so repeated runs
                                give bitwise-identical Y (and J, P); slower than
                                the default atomic accumulation.  Dense A is
                                always summed in this order; no effect there */

typedef struct {
    int32_t fmt;            /* IDS_DENSE: row-major m x n, leading dim ld (elements)
                               IDS_CSR:   rowptr[m+1] (int64), colind[nnz] (int32,
                                          in [0,n); duplicates are summed), val[nnz] */
    int32_t dtype;          /* dense: IDS_F64, IDS_F32 or IDS_BF16; CSR: IDS_F64 */
    int64_t m, n, ld, nnz;
    const void* val;
    const int64_t* rowptr;
    const int32_t* colind;
} ids_matrix;

typedef struct {
    int64_t l1;             /* CountSketch height L1 (1 <= l1 <= 32768)           */
    int64_t l;              /* final sketch height; l == l1: no projection (the   */
                            /* paper's Algorithm 2 exactly); l < l1: Y = G (S A)  */
    uint64_t seed, tag;     /* random-map stream                                   */
    uint32_t flags;         /* IDS_HASH_FULLRANK | IDS_CHECK_FINITE |
                               IDS_DETERMINISTIC                                   */
    int32_t acc;            /* CountSketch accumulation: IDS_F64 or IDS_F32        */
                            /* (F64 input requires IDS_F64)                        */
    int32_t proj;           /* projection arithmetic: IDS_F64 (FP64 MFMA) or       */
                            /* IDS_F32 (FP32 MFMA); must equal acc                 */
    const void* G;          /* l x l1 row-major Gaussian, element type = proj;     */
                            /* ignored when l == l1; NULL: drawn on the device     */
                            /* from the stream (seed, tag | 2^63): entry e uses    */
                            /* outputs 2e, 2e+1 as uniforms u1 = ((z >> 11) + 1)   */
                            /* 2^-53, u2 = (z >> 11) 2^-53 and the Box-Muller      */
                            /* value sqrt(-2 ln u1) cos(2 pi u2), in FP64, rounded  */
                            /* to proj (the workspace grows by l x l1 elements)    */
    const int64_t* fr_pi;   /* IDS_HASH_FULLRANK: permutation pi of [0, m)        */
    const int32_t* fr_x;    /* IDS_HASH_FULLRANK: x[q] in [0, l1) for q >= l1     */
    int32_t* status;        /* IDS_CHECK_FINITE: device int32 status word          */
} ids_sketch_cfg;

/*
 * id_sketch -- Algorithm 2, "draw S" and "compute Y = S A implicitly"
 * (CountSketch, Section 1.3), optionally followed by the Gaussian projection
 * of the sketch (Section 1.2.1).
 *   A      matrix descriptor (device data).
 *   cfg    sketch configuration.
 *   Y      output, l x n, COLUMN-major with leading dimension ldy >= l
 *          (entry (i, j) at Y[j*ldy + i]); element type ydt = cfg->acc.
 * Workspace: ids_sketch_workspace_size().  Dense A is deterministic: the same
 * inputs give bitwise-identical Y (rows of a bucket are added in increasing
 * row order, the order of the textbook definition).  CSR A is summed with
 * atomic adds whose order is not fixed: Y can differ between runs by
 * rounding (FP64, a few ulps of the bucket sums), and is exact whenever the
 * sums are (e.g. integer-valued entries); with IDS_DETERMINISTIC it is summed
 * in the definition's order and is bitwise reproducible.
 */
ids_status ids_sketch_workspace_size(const ids_matrix* A, const ids_sketch_cfg* cfg,
                                     size_t* bytes);
ids_status id_sketch(const ids_matrix* A, const ids_sketch_cfg* cfg, void* Y, int32_t ydt,
                     int64_t ldy, void* ws, size_t ws_bytes, void* stream);

/*
 * id_project -- the projection step alone: Y = G Y1 with G l x q row-major,
 * Y1 q x n row-major (leading dim ld1), Y l x n column-major (leading dim
 * ldy).  dtype IDS_F64 (FP64 MFMA) or IDS_F32 (FP32 MFMA); G, Y1, Y share it.
 */
ids_status id_project(int32_t dtype, int64_t l, int64_t q, int64_t n, const void* G,
                      const void* Y1, int64_t ld1, void* Y, int64_t ldy, void* stream);

/*
 * id_gaussian_sketch -- the Gaussian sketch Y = Omega A of a dense matrix:
 * the sketch of the Gaussian ID the paper compares its method with (Section
 * 1.2.1; Table 1), here as a same-GPU baseline.  Computed on the matrix cores
 * (FP64 or FP32 MFMA) with the m dimension split over workgroups and the
 * partial products summed in a fixed order (deterministic).
 *   A      dense row-major m x n, IDS_F64 or IDS_F32 (A->fmt IDS_DENSE).
 *   l      sketch rows, 1 <= l <= 4096.
 *   Omega  l x m row-major, the dtype of A (caller-owned, e.g. N(0,1)).
 *   Y      output, l x n column-major, leading dimension ldy >= l, the dtype
 *          of A; feed it to id_select.
 * Workspace: ids_gaussian_workspace_size() (may be 0).
 */
ids_status ids_gaussian_workspace_size(const ids_matrix* A, int64_t l, size_t* bytes);
ids_status id_gaussian_sketch(const ids_matrix* A, int64_t l, const void* Omega, void* Y,
                              int64_t ldy, void* ws, size_t ws_bytes, void* stream);

/*
 * id_select -- Algorithm 1 on a sketch Y (l x n): rank-k column-pivoted QR
 * (greedy largest trailing column norm, ties to the smallest column index,
 * norms recomputed in FP64 every step), J from the pivots, and
 * P = [I, R11^{-1} R12] Pi^T in the original column order (P[:, J[t]] = e_t).
 *   Y      entry (i, j) at Y[i*rs + j*cs]; ydt IDS_F64 or IDS_F32 (FP32 is
 *          widened to FP64 on load; all arithmetic is FP64).
 *   k      1 <= k < n and k <= l; l <= 4096.  Shapes the register-resident
 *          factorisation cannot hold (about 2000-8000 columns for long
 *          sketches, 30000-60000 for short ones) run as column steps
 *          (columns in HBM, one kernel per pivot step; same results).
 *   J      int64[k]   chosen columns (entries >= k_eff are set to -1).
 *   P      double[k*n] row-major (rows >= k_eff are zero).
 *   k_eff  int64[1]   number of pivots taken: k unless a zero trailing norm
 *          (rank deficiency) stopped the factorisation early; -1 if a
 *          device-wide wait gave up.
 *   status int32[1] device status word or NULL: IDS_OK, IDS_ERANKDEF
 *          (k_eff < k), IDS_ENONFINITE or IDS_ETIMEOUT (then k_eff = -1 and
 *          J, P are undefined).  Valid once the stream has been synchronised.
 */
ids_status ids_select_workspace_size(int64_t l, int64_t n, int64_t k, size_t* bytes);
ids_status id_select(const void* Y, int32_t ydt, int64_t l, int64_t n, int64_t rs, int64_t cs,
                     int64_t k, int64_t* J, double* P, int64_t* k_eff, int32_t* status, void* ws,
                     size_t ws_bytes, void* stream);

/*
 * ids_select_plan_info -- how id_select runs a shape (host only, nothing is
 * launched): info[0] kernel family (0: grouped lanes, l <= 256; 1: row
 * bands; 2: column steps -- the columns in HBM and two ordinary kernels per
 * pivot step, for shapes wider than the register-resident kernels hold),
 * info[1] candidate exchange (0: speculative column slots; 1: the owner
 * publishes the winner's column after the vote; 2: none), info[2]
 * workgroups, info[3] candidate publishers per pivot step.  int32 info[4],
 * host memory.
 */
ids_status ids_select_plan_info(int64_t l, int64_t n, int64_t k, int32_t* info);

/*
 * id_select_noalloc -- id_select with no workspace argument and no device
 * allocation, for callers that cannot allocate (code under HIP graph capture,
 * serving loops with a fixed memory budget, harnesses that forbid hipMalloc).
 * The caller still owns Y, J, P, k_eff and status.  Scratch is a static
 * device buffer of IDS_SELECT_NOALLOC_MAX_BYTES on each GPU, held from the
 * library's first use there until the process ends; a shape whose
 * ids_select_workspace_size exceeds it is rejected with IDS_EWORKSPACE
 * before anything is launched.  Every call on one GPU shares that buffer
 * (each call re-initialises what it reads): calls that may overlap on one GPU
 * (several streams or threads) race and must be serialised by the caller.
 * Same kernels and results as id_select (bitwise identical); no stage timing.
 */
#define IDS_SELECT_NOALLOC_MAX_BYTES (32u << 20)
ids_status id_select_noalloc(const void* Y, int32_t ydt, int64_t l, int64_t n, int64_t rs, int64_t cs,
                             int64_t k, int64_t* J, double* P, int64_t* k_eff, int32_t* status,
                             void* stream);

/*
 * ids_set_wait_limit -- polls after which a device-wide wait of the pivoted
 * QR gives up (default 2^20, far beyond any normal wait; polls < 0 restores
 * it).  0 treats the exchange as expired from the start: every wait gives up
 * as soon as it finds data missing and the factorisation reports
 * IDS_ETIMEOUT, k_eff = -1 -- a host-forced test of the give-up path (the
 * kernels still finish their bounded loops).  Applies to calls made after it,
 * process-wide.
 */
void ids_set_wait_limit(int64_t polls);

/*
 * tensor_id -- Algorithm 3 for an N-way CP tensor (eq. def-X-tensor) with R
 * terms, in FP64.
 *   factors  host array of N device pointers; factor n is I_n x R COLUMN-major
 *            (entry (i, r) at factors[n][r*ld[n] + i], ld[n] >= dims[n]).
 *   lambda   double[R] s-values.
 *   Jlen     TensorSketch length L (power of two, 16 <= Jlen <= 4096).
 *   k        target rank, k < R, k <= Jlen.
 *   l, G     optional Gaussian second stage (the Gaussian sketch of Section
 *            1.2.1 applied to the TensorSketch): l = 0 factors T M itself
 *            (Algorithm 3 as printed); k <= l <= Jlen factors G (T M), G an
 *            l x Jlen row-major FP64 device buffer (caller-owned, e.g. N(0,1)
 *            entries) or NULL: drawn on the device from the stream
 *            (seed, 0 | 2^63) as ids_sketch_cfg.G describes.
 *   Y        optional output (may be NULL): the sketch T M, Jlen x R
 *            column-major (leading dimension Jlen), before any projection.
 *   J, P, k_eff, status  as in id_select; lambda_hat double[k] (entries >=
 *            k_eff are zero).
 * Random maps h_n, s_n: stream (seed, tag n + 1) over [0, I_n) into Jlen.
 */
ids_status ids_tensor_workspace_size(int32_t N, const int64_t* dims, int64_t R, int64_t k,
                                     int64_t Jlen, int64_t l, size_t* bytes);
ids_status tensor_id(int32_t N, const int64_t* dims, int64_t R, const double* const* factors,
                     const int64_t* ld, const double* lambda, int64_t k, int64_t Jlen,
                     int64_t l, const double* G, uint64_t seed, double* Y, int64_t* J,
                     double* P, double* lambda_hat, int64_t* k_eff, int32_t* status, void* ws,
                     size_t ws_bytes, void* stream);

/*
 * tensor_id_csc -- tensor_id for factors with sparse columns (the paper's
 * sparse CP tensors, whose TensorSketch costs O(N nnz) plus the FFTs).
 * Factor n is I_n x R in compressed sparse column form (host arrays of N
 * device pointers): column r's nonzeros are rowind[n][q], val[n][q] for
 * q in [colptr[n][r], colptr[n][r + 1]), rows strictly ascending within a
 * column and in [0, dims[n]); colptr int64[R + 1], rowind int32, val FP64.
 * Each bucket of a mode's CountSketch takes its entries in ascending row
 * order, as the dense path does, so the results equal tensor_id's on the
 * same tensor stored densely.  Everything else as tensor_id; workspace:
 * ids_tensor_csc_workspace_size (no bucket plans).
 */
ids_status ids_tensor_csc_workspace_size(int32_t N, const int64_t* dims, int64_t R, int64_t k,
                                         int64_t Jlen, int64_t l, size_t* bytes);
ids_status tensor_id_csc(int32_t N, const int64_t* dims, int64_t R, const int64_t* const* colptr,
                         const int32_t* const* rowind, const double* const* val, const double* lambda,
                         int64_t k, int64_t Jlen, int64_t l, const double* G, uint64_t seed, double* Y,
                         int64_t* J, double* P, double* lambda_hat, int64_t* k_eff, int32_t* status,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * Batched mixed-precision matrix ID (hierarchical-matrix style block
 * compression): nprob independent dense problems A_p (m_p x n_p, BF16,
 * row-major, stored back to back in A: A_p starts at element
 * sum_{q<p} m_q n_q), each through Algorithm 2 with a Gaussian second stage and
 * Algorithm 1 with target rank k:
 *   CountSketch of A_p to l1_p = min(m_p, l1max) rows, stream (seed, tag = p),
 *   FP32 accumulation; the sketch is split into BF16 hi + lo parts and
 *   projected by G[:, 0:l1_p] (G: l x l1max row-major BF16, shared by all
 *   problems; NULL: drawn on the device from the stream (seed, 0 | 2^63) as
 *   ids_sketch_cfg.G describes, FP64 rounded to FP32 then to BF16, in the
 *   workspace) on the BF16 matrix cores with FP32 accumulation; column-pivoted
 *   QR of the l x n_p projection with FP32 data and FP64 norms recomputed
 *   every step; FP64 back-substitution for P_p.
 * Limits: 1 <= k <= l <= 122, l <= l1max <= 512, l <= m_p <= 4096,
 * k < n_p <= 1024.  A and G need only element (2-byte) alignment; the results
 * do not depend on it (16-byte-aligned rows are merely read faster).
 *   ids_batched_plan  uploads per-problem descriptors (offsets, largest-first
 *                     schedule) into a caller-owned device buffer of
 *                     ids_batched_plan_size() bytes; synchronises `stream`
 *                     once; returns the workspace size id_batched needs.
 *                     m, n are HOST arrays.
 *   id_batched        asynchronous on `stream` (its CPQR and solve fork onto two
 *                     library-owned streams per device and join back through
 *                     events before it returns, so work queued on `stream`
 *                     afterwards sees the results); tol = 0: rank k for every problem; 0 < tol
 *                     < 1: fixed accuracy (the natural rank-revealing stop of
 *                     Algorithm 1's pivoted QR): problem p stops at the first
 *                     step t with |r_tt| <= tol |r_11| and k_eff_p = t <= k.
 *                     J int64[nprob*k] (J_p at p*k, -1 past
 *                     k_eff_p), P double[k * sum n_p] (P_p, k x n_p row-major,
 *                     at k * sum_{q<p} n_q), k_eff int64[nprob], status
 *                     int32[nprob] or NULL (per problem: IDS_OK, IDS_ERANKDEF
 *                     when a zero trailing norm stopped it before its rank,
 *                     IDS_ENONFINITE).  The plan, m and n must be the ones the
 *                     plan was built from.
 */
ids_status ids_batched_plan_size(int64_t nprob, size_t* bytes);
ids_status ids_batched_plan(int64_t nprob, const int64_t* m, const int64_t* n, int64_t k, int64_t l,
                            int64_t l1max, void* plan, size_t plan_bytes, size_t* ws_bytes,
                            void* stream);
ids_status id_batched(int64_t nprob, const int64_t* m, const int64_t* n, const void* plan, int64_t k,
                      int64_t l, int64_t l1max, uint64_t seed, double tol, const void* A, const void* G,
                      int64_t* J, double* P, int64_t* k_eff, int32_t* status, void* ws, size_t ws_bytes,
                      void* stream);

/*
 * Batched ID as a HIP graph: ids_batched_graph_create records one id_batched
 * call (the same arguments; the caller's plan, A, G, outputs and workspace
 * fixed) into a graph -- the sketch, the three concurrent width-class
 * factorisations on forked streams and the solve, with the fork and join as
 * graph edges -- and instantiates it; nothing runs yet.  Each
 * ids_batched_graph_launch replays the whole batch on `stream` as one graph
 * launch (asynchronous, results as id_batched once the stream is
 * synchronised); the recorded buffers must stay allocated and are
 * overwritten by every replay.  Replays of one graph on several streams at
 * once race on those buffers.  ids_batched_graph_destroy frees the graph
 * (not the caller's buffers).  No memset or allocation is recorded.
 */
typedef struct ids_batched_graph_s* ids_batched_graph;
ids_status ids_batched_graph_create(int64_t nprob, const int64_t* m, const int64_t* n, const void* plan,
                                    int64_t k, int64_t l, int64_t l1max, uint64_t seed, double tol,
                                    const void* A, const void* G, int64_t* J, double* P, int64_t* k_eff,
                                    int32_t* status, void* ws, size_t ws_bytes, ids_batched_graph* graph);
ids_status ids_batched_graph_launch(ids_batched_graph graph, void* stream);
void ids_batched_graph_destroy(ids_batched_graph graph);

/*
 * Stage timing.  While enabled, every call records a pair of HIP events on its
 * stream around each stage ("plan", "countsketch", "project", "cpqr", "trsm",
 * "tensorsketch", "lambda_hat").  ids_profile_read waits for the recorded
 * events and returns the summed elapsed milliseconds and the number of
 * recorded launches of a stage; ids_profile_reset waits for and recycles them.
 * Intended for measurement; off by default.  Each recorded pair costs the
 * stream a few microseconds, so ids_profile_stages restricts recording to
 * the named stages (comma-separated, e.g. "countsketch"; NULL or "" = all,
 * the default); an unknown name is IDS_EINVAL and leaves the selection as it
 * was.
 */
void ids_profile_enable(int on);
ids_status ids_profile_stages(const char* stages);
ids_status ids_profile_read(const char* stage, double* total_ms, int64_t* count);
void ids_profile_reset(void);

/*
 * ids_stream_read -- measurement utility: reads every 16-byte chunk of the
 * device buffer [p, p + bytes) once (non-temporal loads, as the dense
 * CountSketch reads A) and writes the XOR of all 32-bit words to the device
 * word *checksum.  Timed around, it gives the HBM read rate this device
 * reaches in practice -- the ceiling beside the datasheet peak for kernels
 * that stream their input once.  p and bytes must be 16-byte multiples.
 */
ids_status ids_stream_read(const void* p, size_t bytes, uint32_t* checksum, void* stream);

/*
 * Launch-shape knobs.  Each knob (a name and an integer) selects among
 * kernel variants or launch shapes that give the same results, e.g.
 * "select.gl.l128.n4k" (pivoted-QR workgroup size for sketches of 65..128
 * rows and 1025..4096 columns: 0 = 8 waves, 1 = 4 waves), "trsm.k64" (lanes
 * per column of the interpolation-matrix solve), "batched.rl512" (rows the
 * 512-thread batched factorisation keeps in LDS: 36 or 0), "project.wgs"
 * (workgroups the projection's K split aims for).  The library's defaults
 * are the table the project's autotuner (paper_1901_10559_amd/tune.py)
 * measured on the device.  ids_tune_set overrides a knob for later calls
 * (value < 0 restores the table's value); an unknown name or a value the knob
 * does not accept is IDS_EINVAL.  Process-wide; query workspace sizes after
 * changing knobs.
 */
ids_status ids_tune_set(const char* key, int64_t value);
ids_status ids_tune_get(const char* key, int64_t* value);

/* ids_finalize -- release what the library holds between calls (the side
 * streams of id_batched, the stage-timing events), after the work queued on
 * them has finished.  Optional; later calls recreate what they need.  Call it
 * before the HIP runtime is torn down (e.g. from an atexit handler). */
void ids_finalize(void);

/* Human-readable name of a status code, and the calling thread's last error
 * message (empty string when the last call succeeded). */
const char* ids_status_string(ids_status s);
const char* ids_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IDSKETCH_H */
