// Internal launch interfaces between the C-ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/idsketch.h"
#include "common.hpp"

namespace ids {

ids_status check_launch(const char* what);

// optional per-stage timing with HIP events on the launch stream
enum ProfKind { PK_PLAN = 0, PK_CS, PK_PROJ, PK_CPQR, PK_TRSM, PK_TS, PK_LHAT, PK_COUNT };
struct ProfScope {
    ProfScope(int kind, hipStream_t st);  // kind < 0: records nothing
    ~ProfScope();
    int kind;
    hipStream_t st;
    hipEvent_t a;
    bool on;
};

// largest dynamic LDS a workgroup may use on the current device
size_t lds_limit();
#define CSR_LDS_MAX_BYTES (lds_limit())

// ---- CountSketch plan: rows grouped by bucket -----------------------------
struct PlanShape {
    int64_t m, L;
    int32_t seg_rows, nseg;
};
struct PlanBufs {
    int32_t* seg;   // L x nseg counts, then per-bucket exclusive scans
    int32_t* off;   // L + 1 bucket offsets into rows
    int32_t* rows;  // m signed row codes grouped by bucket
    int32_t* tot;   // L bucket totals
};
PlanShape plan_shape(int64_t m, int64_t L);
size_t plan_bytes(const PlanShape& ps);
PlanBufs plan_carve(const PlanShape& ps, char*& p);
ids_status plan_build(const PlanShape& ps, uint64_t key, const int64_t* fr_pi, const int32_t* fr_x,
                      const PlanBufs& pb, hipStream_t st);
// several plans (plain hash) at once: one launch when all are small
ids_status plan_build_many(int count, const PlanShape* ps, const uint64_t* keys, const PlanBufs* pb,
                           hipStream_t st);

// ---- CountSketch -------------------------------------------------------------
ids_status cs_dense(int32_t dtype, int32_t acc, const void* A, int64_t lda, int64_t n, const PlanBufs& pb,
                    int64_t L, void* Y, int64_t rs, int64_t cs, hipStream_t st);
ids_status cs_csr(const int64_t* rowptr, const int32_t* colind, const double* val, int64_t m, int64_t n,
                  const PlanBufs& pb, int64_t L, double* Y, int64_t rs, int64_t cs, int32_t* scratch_bop,
                  bool ordered, int64_t nnz, char* bin_ws, hipStream_t st);
// workspace of the binned ordered CSR sketch (0: shape too wide, the unbinned
// ordered kernel runs instead)
size_t csr_bin_bytes(int64_t m, int64_t n, int64_t nnz, int64_t L);

// ---- projection GEMM (MFMA): Y(col-major, ldy) = G (l x q) * Y1 (q x n, ld1) --
ids_status project(int32_t dtype, int64_t l, int64_t q, int64_t n, const void* G, const void* Y1, int64_t ld1,
                   void* Y, int64_t ldy, hipStream_t st, bool y1_colmajor = false);
// projection with K split over S chunks (S from project_splits for about
// target_wgs workgroups; partial products in `part`, S x l x n elements of the
// dtype, then summed in chunk order)
int project_splits(int64_t l, int64_t q, int64_t n, int64_t target_wgs);
ids_status project_split(int32_t dtype, int64_t l, int64_t q, int64_t n, const void* G, const void* Y1, int64_t ld1,
                         bool y1_colmajor, void* Y, int64_t ldy, int S, void* part, hipStream_t st);

// ---- CPQR + interpolation matrix --------------------------------------------
struct SelectPlan {
    int64_t l, n, k;
    int cols, threads, nb;  // columns per workgroup, threads per workgroup, workgroups
    int nh;                 // candidate publishers per step
    int mode, S, H0;        // mailbox exchange: mode, slot stride, column box offset
    int64_t RS;             // mailbox doubles per factorisation step
    int64_t CS;             // speculative mode: doubles per set of column slots (two sets)
    int variant;            // kernel variant (tuned knob)
    int steps = 0;          // 1: columns in HBM, one kernel per pivot step
};
// P from Rt / R11c / pos for large k: blocked back-substitution on the FP64
// matrix cores, in place in P (solve_blk.hip)
ids_status solve_mfma_small(int64_t n, int64_t k, const double* Rt, const double* R11c, const int32_t* pos,
                            const int64_t* keff, double* P, hipStream_t st);  // k <= 128
ids_status solve_blocked(int64_t n, int64_t k, const double* Rt, const double* R11c, const int32_t* pos,
                         const int64_t* keff, double* P, hipStream_t st);
// the column-steps factorisation (cpqr_steps.hip): workspace bytes before Rt
size_t steps_bytes(int64_t l, int64_t n, int64_t k, int64_t* ldw);
int64_t steps_workgroups(int64_t l, int64_t n);  // workgroups of each column-steps kernel
ids_status steps_factor(const void* Y, int32_t ydt, int64_t l, int64_t n, int64_t rs, int64_t cs, int64_t k,
                        int64_t* J, int64_t* keff, int32_t* status, double* Rt, double* R11c, int32_t* pos, char* ws,
                        hipStream_t st);
ids_status select_plan(int64_t l, int64_t n, int64_t k, SelectPlan& sp);
size_t select_bytes(const SelectPlan& sp);
// status: optional device status word; prof: record stage events (when on)
ids_status select_run(const SelectPlan& sp, const void* Y, int32_t ydt, int64_t rs, int64_t cs, int64_t* J,
                      double* P, int64_t* keff, int32_t* status, char* ws, hipStream_t st, bool prof = true);
// polls before a device-wide CPQR wait gives up (< 0: the default; 0: give up
// at once, every factorisation then reports IDS_ETIMEOUT)
void set_wait_limit(int64_t polls);
// lambda_hat[t] = lambda[J[t]] * sum_r P[t][r]
ids_status lambda_hat(int64_t k, int64_t n, const double* P, const int64_t* J, const int64_t* keff,
                      const double* lambda, double* lhat, hipStream_t st);

// ---- batched mixed-precision ID --------------------------------------------
ids_status batched_plan_bytes(int64_t nprob, size_t* bytes);
// destroys the library's side streams (after their work has finished)
void batched_release();
ids_status batched_plan(int64_t nprob, const int64_t* m, const int64_t* n, int64_t k, int64_t l, int64_t l1max,
                        void* plan, size_t plan_bytes, size_t* ws_bytes, hipStream_t st);
ids_status batched_run(int64_t nprob, const void* plan, int64_t k, int64_t l, int64_t l1max, uint64_t seed,
                       double tol, const void* A, const void* G, int64_t* J, double* P, int64_t* keff,
                       int32_t* status, void* ws, size_t ws_bytes, int64_t a_elems, int64_t y_elems,
                       int64_t r_elems, hipStream_t st, bool prof = true);
// the same call captured into an instantiated HIP graph (opaque handle)
ids_status batched_graph_create(int64_t nprob, const void* plan, int64_t k, int64_t l, int64_t l1max, uint64_t seed,
                                double tol, const void* A, const void* G, int64_t* J, double* P, int64_t* keff,
                                int32_t* status, void* ws, size_t ws_bytes, int64_t a_elems, int64_t y_elems,
                                int64_t r_elems, void** out);
ids_status batched_graph_launch(void* g, hipStream_t st);
void batched_graph_destroy(void* g);

// ---- l x q N(0, 1) matrix from the stream (seed, tag | 2^63), Box-Muller ----
ids_status gaussian_fill(uint64_t seed, uint64_t tag, int64_t l, int64_t q, int32_t dtype, void* out, hipStream_t st);

// ---- finiteness scan of a sketch (l x n column-major) -> status word ---------
ids_status check_finite(int32_t dtype, const void* Y, int64_t l, int64_t n, int64_t ldy, int32_t* status,
                        hipStream_t st);
// every 16-byte chunk of [p, p + bytes) read once; XOR of the words -> *sum
ids_status stream_read(const void* p, size_t bytes, uint32_t* sum, hipStream_t st);

// ---- TensorSketch -------------------------------------------------------------
// colptr / rowind / val (non-NULL): CSC factors instead of dense ones
ids_status tensorsketch(int32_t N, const int64_t* dims, int64_t R, const double* const* factors,
                        const int64_t* ld, const double* lambda, int64_t Jlen, const PlanBufs* plans,
                        const uint64_t* keys, const double2* twiddle, double* Y, hipStream_t st,
                        const int64_t* const* colptr = nullptr, const int32_t* const* rowind = nullptr,
                        const double* const* val = nullptr);
ids_status twiddles(int64_t Jlen, double2* tw, hipStream_t st);
size_t ts_lds_bytes(int64_t J);

}  // namespace ids
