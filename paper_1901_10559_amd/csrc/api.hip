// C-ABI layer of idsketch: argument validation, workspace carving and launch
// sequencing.  Declarations and contracts: include/idsketch.h.
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "tune.hpp"

namespace ids {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

ids_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return IDS_EHIP;
    }
    return IDS_OK;
}

size_t lds_limit() {
    static std::mutex mu;
    static std::unordered_map<int, size_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    cache[dev] = (size_t)v;
    return (size_t)v;
}

// ---------------------------------------------------------------------------
// launch-shape knobs (tuned table + run-time overrides)
// ---------------------------------------------------------------------------
struct TuneKnob {
    const char* key;
    int64_t value;
};
static const TuneKnob kTuned[] = {
#include "tuned_table.inc"
};
// values each knob accepts
static bool tune_valid(const std::string& key, int64_t v) {
    if (key.rfind("select.gl.", 0) == 0) return v == 0 || v == 1;
    if (key == "trsm.k32") return v == 1 || v == 2 || v == 4;
    if (key == "trsm.k64") return v == 2 || v == 4;
    if (key == "trsm.k128") return v == 4 || v == 8;
    if (key == "batched.rl512" || key == "batched.rl256") return v == 0 || v == 36;
    if (key == "project.wgs") return v >= 32 && v <= 4096;
    if (key == "cs.dense.wpc") return v == 0 || (v >= 2 && v <= 8);
    if (key == "select.steps") return v == 0 || v == 1;
    if (key == "cs.csr.bin") return v == 0 || v == 1;
    if (key == "trsm.mfma") return v == 0 || v == 1;
    return false;
}
static std::mutex g_tune_mu;
static std::unordered_map<std::string, int64_t> g_tune_over;

int64_t tune_get(const std::string& key, int64_t dflt) {
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_over.find(key);
        if (it != g_tune_over.end()) return it->second;
    }
    for (const auto& t : kTuned)
        if (key == t.key) return t.value;
    return dflt;
}

static bool tune_known(const std::string& key) {
    for (const auto& t : kTuned)
        if (key == t.key) return true;
    return false;
}

// ---------------------------------------------------------------------------
// stage timing (HIP events recorded around each stage on its stream)
// ---------------------------------------------------------------------------
static const char* kProfNames[PK_COUNT] = {"plan", "countsketch", "project", "cpqr",
                                           "trsm", "tensorsketch", "lambda_hat"};
struct ProfRec {
    int kind;
    hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static uint32_t g_prof_mask = (1u << PK_COUNT) - 1;  // stages recorded while on
static std::vector<ProfRec> g_recs;
static std::vector<hipEvent_t> g_pool;

static hipEvent_t prof_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(int k, hipStream_t s) : kind(k), st(s), a(nullptr), on(false) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (k < 0 || !g_prof_on || !((g_prof_mask >> k) & 1u)) return;
    a = prof_event();
    if (a && hipEventRecord(a, st) == hipSuccess) on = true;
}

ProfScope::~ProfScope() {
    if (!on) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    hipEvent_t b = prof_event();
    if (b && hipEventRecord(b, st) == hipSuccess) g_recs.push_back({kind, a, b});
}

static ids_status fail(ids_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

static size_t esize(int32_t dt) { return dt == IDS_F64 ? 8 : dt == IDS_F32 ? 4 : 2; }

static bool aligned256(const void* p) { return ((uintptr_t)p & 255) == 0; }

static ids_status check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return IDS_OK;
    if (!ws) return fail(IDS_EWORKSPACE, "workspace is NULL but " + std::to_string(need) + " bytes are needed");
    if (!aligned256(ws)) return fail(IDS_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(IDS_EWORKSPACE,
                    "workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(need) + " bytes");
    return IDS_OK;
}

// ---------------------------------------------------------------------------
// sketch
// ---------------------------------------------------------------------------
static ids_status validate_sketch(const ids_matrix* A, const ids_sketch_cfg* c) {
    if (!A || !c) return fail(IDS_EINVAL, "A and cfg must be non-NULL");
    if (A->m < 1 || A->n < 1) return fail(IDS_EINVAL, "matrix must be at least 1 x 1");
    if (A->m >= (int64_t(1) << 31) - 1) return fail(IDS_EINVAL, "m must be < 2^31 - 1");
    if (A->fmt == IDS_DENSE) {
        if (!A->val) return fail(IDS_EINVAL, "dense A: val is NULL");
        if (A->ld < A->n) return fail(IDS_EINVAL, "dense A: ld < n");
        if (A->dtype != IDS_F64 && A->dtype != IDS_F32 && A->dtype != IDS_BF16)
            return fail(IDS_EDTYPE, "dense A: dtype must be IDS_F64, IDS_F32 or IDS_BF16");
    } else if (A->fmt == IDS_CSR) {
        if (!A->val || !A->rowptr || !A->colind) return fail(IDS_EINVAL, "CSR A: rowptr, colind and val required");
        if (A->dtype != IDS_F64) return fail(IDS_EDTYPE, "CSR A: dtype must be IDS_F64");
        if (A->nnz < 0) return fail(IDS_EINVAL, "CSR A: nnz < 0");
        if (A->n >= (int64_t(1) << 31)) return fail(IDS_EINVAL, "CSR A: n must be < 2^31");
    } else {
        return fail(IDS_EINVAL, "unknown matrix format");
    }
    if (c->l1 < 1 || c->l1 > 32768) return fail(IDS_EINVAL, "l1 must be in [1, 32768]");
    if (c->l < 1 || c->l > c->l1) return fail(IDS_EINVAL, "l must be in [1, l1]");
    if (c->acc != IDS_F64 && c->acc != IDS_F32) return fail(IDS_EDTYPE, "acc must be IDS_F64 or IDS_F32");
    if (A->dtype == IDS_F64 && c->acc != IDS_F64) return fail(IDS_EDTYPE, "FP64 input needs FP64 accumulation");
    if (A->fmt == IDS_CSR && c->acc != IDS_F64) return fail(IDS_EDTYPE, "CSR input needs FP64 accumulation");
    if (c->l < c->l1 && c->proj != c->acc) return fail(IDS_EDTYPE, "proj must equal acc");
    if (c->flags & ~(IDS_HASH_FULLRANK | IDS_CHECK_FINITE | IDS_DETERMINISTIC))
        return fail(IDS_EINVAL, "unknown flag bits");
    if ((c->flags & IDS_CHECK_FINITE) && !c->status) return fail(IDS_EINVAL, "IDS_CHECK_FINITE needs status");
    if ((c->flags & IDS_HASH_FULLRANK) && (!c->fr_pi || !c->fr_x))
        return fail(IDS_EINVAL, "IDS_HASH_FULLRANK needs fr_pi and fr_x");
    if (sizeof(int32_t) * (size_t)c->l1 > lds_limit()) return fail(IDS_EINVAL, "l1 too large for the LDS histogram");
    return IDS_OK;
}

struct SketchLayout {
    PlanShape ps;
    size_t plan, y1, bop, part, gdraw, bin, total;
    int splits;  // projection K split (1: one pass)
};

static SketchLayout sketch_layout(const ids_matrix* A, const ids_sketch_cfg* c) {
    SketchLayout L;
    L.ps = plan_shape(A->m, c->l1);
    L.plan = plan_bytes(L.ps);
    L.y1 = (c->l < c->l1) ? align256(esize(c->acc) * (size_t)c->l1 * A->n) : 0;
    L.bop = (A->fmt == IDS_CSR) ? align256(sizeof(int32_t) * (size_t)A->m) : 0;
    // a projection with few output tiles splits its K (the l1 sketch rows) so
    // that about 256 workgroups share it; the partial products need l x n each
    L.splits = (c->l < c->l1) ? project_splits(c->l, c->l1, A->n, tune_get("project.wgs", 256)) : 1;
    L.part = (L.splits > 1) ? align256(esize(c->acc) * (size_t)L.splits * c->l * A->n) : 0;
    // G drawn on the device when the caller passes none
    L.gdraw = (c->l < c->l1 && !c->G) ? align256(esize(c->acc) * (size_t)c->l * c->l1) : 0;
    // IDS_DETERMINISTIC on CSR input: the binned entries of the ordered sketch
    L.bin = (A->fmt == IDS_CSR && (c->flags & IDS_DETERMINISTIC)) ? csr_bin_bytes(A->m, A->n, A->nnz, c->l1) : 0;
    L.total = L.plan + L.y1 + L.bop + L.part + L.gdraw + L.bin;
    return L;
}

}  // namespace ids

using namespace ids;

extern "C" {

const char* ids_status_string(ids_status s) {
    switch (s) {
        case IDS_OK: return "IDS_OK";
        case IDS_EINVAL: return "IDS_EINVAL";
        case IDS_EDTYPE: return "IDS_EDTYPE";
        case IDS_EWORKSPACE: return "IDS_EWORKSPACE";
        case IDS_EHIP: return "IDS_EHIP";
        case IDS_ETIMEOUT: return "IDS_ETIMEOUT";
        case IDS_ERANKDEF: return "IDS_ERANKDEF";
        case IDS_ENONFINITE: return "IDS_ENONFINITE";
        default: return "IDS_UNKNOWN";
    }
}

const char* ids_last_error(void) { return g_err.c_str(); }

void ids_profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
}

ids_status ids_profile_stages(const char* stages) {
    g_err.clear();
    uint32_t mask = 0;
    if (!stages || !*stages) {
        mask = (1u << PK_COUNT) - 1;
    } else {
        std::string all(stages);
        size_t b = 0;
        while (b <= all.size()) {
            size_t e = all.find(',', b);
            if (e == std::string::npos) e = all.size();
            const std::string name = all.substr(b, e - b);
            int kind = -1;
            for (int k = 0; k < PK_COUNT; ++k)
                if (name == kProfNames[k]) kind = k;
            if (kind < 0) return fail(IDS_EINVAL, "unknown stage " + name);
            mask |= 1u << kind;
            b = e + 1;
        }
    }
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_mask = mask;
    return IDS_OK;
}

ids_status ids_profile_read(const char* stage, double* total_ms, int64_t* count) {
    g_err.clear();
    if (!stage || !total_ms || !count) return fail(IDS_EINVAL, "stage, total_ms and count must be non-NULL");
    int kind = -1;
    for (int k = 0; k < PK_COUNT; ++k)
        if (std::string(stage) == kProfNames[k]) kind = k;
    if (kind < 0) return fail(IDS_EINVAL, std::string("unknown stage ") + stage);
    std::lock_guard<std::mutex> g(g_prof_mu);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto& r : g_recs) {
        if (r.kind != kind) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(IDS_EHIP, "hipEventSynchronize failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(IDS_EHIP, "hipEventElapsedTime failed");
        tot += ms;
        ++cnt;
    }
    *total_ms = tot;
    *count = cnt;
    return IDS_OK;
}

void ids_finalize(void) {
    batched_release();
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = false;
    for (auto& r : g_recs) {
        hipEventSynchronize(r.b);
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    for (hipEvent_t e : g_pool) hipEventDestroy(e);
    g_pool.clear();
}

void ids_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto& r : g_recs) {
        hipEventSynchronize(r.b);
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
}

ids_status ids_sketch_workspace_size(const ids_matrix* A, const ids_sketch_cfg* cfg, size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(IDS_EINVAL, "bytes is NULL");
    ids_status s = validate_sketch(A, cfg);
    if (s) return s;
    *bytes = sketch_layout(A, cfg).total;
    return IDS_OK;
}

ids_status id_sketch(const ids_matrix* A, const ids_sketch_cfg* c, void* Y, int32_t ydt, int64_t ldy, void* ws,
                     size_t ws_bytes, void* stream) {
    g_err.clear();
    ids_status s = validate_sketch(A, c);
    if (s) return s;
    if (!Y) return fail(IDS_EINVAL, "Y is NULL");
    if (ydt != c->acc) return fail(IDS_EDTYPE, "ydt must equal cfg->acc");
    if (ldy < c->l) return fail(IDS_EINVAL, "ldy < l");
    SketchLayout L = sketch_layout(A, c);
    if ((s = check_ws(ws, ws_bytes, L.total))) return s;
    hipStream_t st = (hipStream_t)stream;
    char* p = (char*)ws;
    PlanBufs pb = plan_carve(L.ps, p);
    void* Y1 = p;
    p += L.y1;
    int32_t* bop = (int32_t*)p;
    p += L.bop;
    void* part = p;
    p += L.part;
    void* gdraw = p;
    p += L.gdraw;
    char* bin = L.bin ? p : nullptr;

    const bool proj = c->l < c->l1;
    const uint64_t key = stream_key(c->seed, c->tag);
    {
        ProfScope ps(PK_PLAN, st);
        s = plan_build(L.ps, key, (c->flags & IDS_HASH_FULLRANK) ? c->fr_pi : nullptr,
                       (c->flags & IDS_HASH_FULLRANK) ? c->fr_x : nullptr, pb, st);
    }
    if (s) return s;
    // CountSketch destination: row-major Y1 workspace (projection follows) or
    // the caller's column-major Y directly.
    void* dst = proj ? Y1 : Y;
    const int64_t rs = proj ? A->n : 1;
    const int64_t cs = proj ? 1 : ldy;
    {
        ProfScope ps(PK_CS, st);
        if (A->fmt == IDS_DENSE)
            s = cs_dense(A->dtype, c->acc, A->val, A->ld, A->n, pb, c->l1, dst, rs, cs, st);
        else
            s = cs_csr(A->rowptr, A->colind, (const double*)A->val, A->m, A->n, pb, c->l1, (double*)dst, rs, cs,
                       bop, (c->flags & IDS_DETERMINISTIC) != 0, A->nnz, bin, st);
    }
    if (s) return s;
    if (proj) {
        ProfScope ps(PK_PROJ, st);
        const void* G = c->G;
        if (!G) {
            s = gaussian_fill(c->seed, c->tag, c->l, c->l1, c->acc, gdraw, st);
            G = gdraw;
        }
        if (!s) s = project_split(c->acc, c->l, c->l1, A->n, G, Y1, A->n, false, Y, ldy, L.splits, part, st);
    }
    if (!s && (c->flags & IDS_CHECK_FINITE)) s = check_finite(c->acc, Y, c->l, A->n, ldy, c->status, st);
    return s;
}

ids_status id_project(int32_t dtype, int64_t l, int64_t q, int64_t n, const void* G, const void* Y1, int64_t ld1,
                      void* Y, int64_t ldy, void* stream) {
    g_err.clear();
    if (!G || !Y1 || !Y) return fail(IDS_EINVAL, "G, Y1 and Y must be non-NULL");
    if (l < 1 || q < 1 || n < 1) return fail(IDS_EINVAL, "sizes must be positive");
    if (ld1 < n || ldy < l) return fail(IDS_EINVAL, "leading dimension too small");
    if (dtype != IDS_F64 && dtype != IDS_F32) return fail(IDS_EDTYPE, "dtype must be IDS_F64 or IDS_F32");
    return project(dtype, l, q, n, G, Y1, ld1, Y, ldy, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Gaussian sketch (the comparison method)
// ---------------------------------------------------------------------------
static ids_status validate_gaussian(const ids_matrix* A, int64_t l) {
    if (!A) return fail(IDS_EINVAL, "A must be non-NULL");
    if (A->fmt != IDS_DENSE) return fail(IDS_EINVAL, "the Gaussian sketch takes a dense A");
    if (A->m < 1 || A->n < 1) return fail(IDS_EINVAL, "matrix must be at least 1 x 1");
    if (!A->val) return fail(IDS_EINVAL, "dense A: val is NULL");
    if (A->ld < A->n) return fail(IDS_EINVAL, "dense A: ld < n");
    if (A->dtype != IDS_F64 && A->dtype != IDS_F32) return fail(IDS_EDTYPE, "dtype must be IDS_F64 or IDS_F32");
    if (l < 1 || l > 4096) return fail(IDS_EINVAL, "l must be in [1, 4096]");
    return IDS_OK;
}

static int gaussian_splits(const ids_matrix* A, int64_t l) { return project_splits(l, A->m, A->n, 2048); }

ids_status ids_gaussian_workspace_size(const ids_matrix* A, int64_t l, size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(IDS_EINVAL, "bytes is NULL");
    ids_status s = validate_gaussian(A, l);
    if (s) return s;
    const int S = gaussian_splits(A, l);
    *bytes = S > 1 ? align256(esize(A->dtype) * (size_t)S * l * A->n) : 0;
    return IDS_OK;
}

ids_status id_gaussian_sketch(const ids_matrix* A, int64_t l, const void* Omega, void* Y, int64_t ldy, void* ws,
                              size_t ws_bytes, void* stream) {
    g_err.clear();
    ids_status s = validate_gaussian(A, l);
    if (s) return s;
    if (!Omega || !Y) return fail(IDS_EINVAL, "Omega and Y must be non-NULL");
    if (ldy < l) return fail(IDS_EINVAL, "ldy < l");
    const int S = gaussian_splits(A, l);
    const size_t need = S > 1 ? align256(esize(A->dtype) * (size_t)S * l * A->n) : 0;
    if ((s = check_ws(ws, ws_bytes, need))) return s;
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps(PK_PROJ, st);
    return project_split(A->dtype, l, A->m, A->n, Omega, A->val, A->ld, false, Y, ldy, S, ws, st);
}

// ---------------------------------------------------------------------------
// select
// ---------------------------------------------------------------------------
static ids_status validate_select(int64_t l, int64_t n, int64_t k) {
    if (l < 1 || n < 2) return fail(IDS_EINVAL, "need l >= 1 and n >= 2");
    if (k < 1 || k >= n) return fail(IDS_EINVAL, "k must satisfy 1 <= k < n");
    if (k > l) return fail(IDS_EINVAL, "k must be <= l");
    if (l > 4096) return fail(IDS_EINVAL, "l must be <= 4096");
    return IDS_OK;
}

ids_status ids_select_workspace_size(int64_t l, int64_t n, int64_t k, size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(IDS_EINVAL, "bytes is NULL");
    ids_status s = validate_select(l, n, k);
    if (s) return s;
    SelectPlan sp;
    if ((s = select_plan(l, n, k, sp))) return s;
    *bytes = select_bytes(sp);
    return IDS_OK;
}

void ids_set_wait_limit(int64_t polls) { set_wait_limit(polls); }

ids_status ids_tune_set(const char* key, int64_t value) {
    g_err.clear();
    if (!key || !tune_known(key)) return fail(IDS_EINVAL, std::string("unknown knob ") + (key ? key : "(null)"));
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (value < 0) {
        g_tune_over.erase(key);
        return IDS_OK;
    }
    if (!tune_valid(key, value)) return fail(IDS_EINVAL, std::string("value not accepted by knob ") + key);
    g_tune_over[key] = value;
    return IDS_OK;
}

ids_status ids_tune_get(const char* key, int64_t* value) {
    g_err.clear();
    if (!key || !value || !tune_known(key)) return fail(IDS_EINVAL, "unknown knob or NULL value");
    *value = tune_get(key, -1);
    return IDS_OK;
}

ids_status ids_stream_read(const void* p, size_t bytes, uint32_t* checksum, void* stream) {
    g_err.clear();
    if (!p || !checksum) return fail(IDS_EINVAL, "p and checksum must be non-NULL");
    if (((uintptr_t)p & 15) != 0 || (bytes & 15) != 0) return fail(IDS_EINVAL, "p and bytes must be 16-byte multiples");
    return stream_read(p, bytes, checksum, (hipStream_t)stream);
}

ids_status ids_select_plan_info(int64_t l, int64_t n, int64_t k, int32_t* info) {
    g_err.clear();
    if (!info) return fail(IDS_EINVAL, "info is NULL");
    ids_status s = validate_select(l, n, k);
    if (s) return s;
    SelectPlan sp;
    if ((s = select_plan(l, n, k, sp))) return s;
    info[0] = sp.steps ? 2 : (l <= 256 ? 0 : 1);
    info[1] = sp.steps ? 2 : sp.mode;           // the column-steps path exchanges nothing
    info[2] = sp.steps ? (int32_t)steps_workgroups(l, n) : sp.nb;  // one column per wave
    info[3] = sp.steps ? 0 : sp.nh;
    return IDS_OK;
}

ids_status id_select(const void* Y, int32_t ydt, int64_t l, int64_t n, int64_t rs, int64_t cs, int64_t k, int64_t* J,
                     double* P, int64_t* k_eff, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    ids_status s = validate_select(l, n, k);
    if (s) return s;
    if (!Y || !J || !P || !k_eff) return fail(IDS_EINVAL, "Y, J, P and k_eff must be non-NULL");
    if (ydt != IDS_F64 && ydt != IDS_F32) return fail(IDS_EDTYPE, "Y dtype must be IDS_F64 or IDS_F32");
    if (rs < 1 || cs < 1) return fail(IDS_EINVAL, "strides must be positive");
    SelectPlan sp;
    if ((s = select_plan(l, n, k, sp))) return s;
    if ((s = check_ws(ws, ws_bytes, select_bytes(sp)))) return s;
    return select_run(sp, Y, ydt, rs, cs, J, P, k_eff, status, (char*)ws, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// allocation-free select: the scratch is a static device array
// ---------------------------------------------------------------------------
// One copy per GPU, placed by the loader with the library's code object and
// held until the process ends.  In host code `scratch` names a host-side
// stand-in; the device address of each GPU's copy comes from
// hipGetSymbolAddress (with that GPU current) and is the only one passed on.
static __device__ __align__(256) unsigned char scratch[IDS_SELECT_NOALLOC_MAX_BYTES];
static std::mutex g_scr_mu;
static void* g_scr_ptr[64];

static ids_status scratch_ptr(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(IDS_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> g(g_scr_mu);
    if (!g_scr_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(IDS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scr_ptr[dev] = p;
    }
    *out = g_scr_ptr[dev];
    return IDS_OK;
}

ids_status id_select_noalloc(const void* Y, int32_t ydt, int64_t l, int64_t n, int64_t rs, int64_t cs, int64_t k,
                             int64_t* J, double* P, int64_t* k_eff, int32_t* status, void* stream) {
    g_err.clear();
    ids_status s = validate_select(l, n, k);
    if (s) return s;
    if (!Y || !J || !P || !k_eff) return fail(IDS_EINVAL, "Y, J, P and k_eff must be non-NULL");
    if (ydt != IDS_F64 && ydt != IDS_F32) return fail(IDS_EDTYPE, "Y dtype must be IDS_F64 or IDS_F32");
    if (rs < 1 || cs < 1) return fail(IDS_EINVAL, "strides must be positive");
    SelectPlan sp;
    if ((s = select_plan(l, n, k, sp))) return s;
    const size_t need = select_bytes(sp);
    if (need > (size_t)IDS_SELECT_NOALLOC_MAX_BYTES)
        return fail(IDS_EWORKSPACE, "id_select_noalloc: this shape needs " + std::to_string(need) +
                                        " bytes of scratch; the static buffer holds " +
                                        std::to_string((size_t)IDS_SELECT_NOALLOC_MAX_BYTES));
    void* scr = nullptr;
    if ((s = scratch_ptr(&scr))) return s;
    return select_run(sp, Y, ydt, rs, cs, J, P, k_eff, status, (char*)scr, (hipStream_t)stream, false);
}

// ---------------------------------------------------------------------------
// tensor
// ---------------------------------------------------------------------------
struct TensorLayout {
    PlanShape ps[8];
    size_t plans, tw, y, yp, part, gdraw, sel, total;
    int splits;
    SelectPlan sp;
};

static ids_status validate_tensor(int32_t N, const int64_t* dims, int64_t R, int64_t k, int64_t Jlen, int64_t l) {
    if (N < 1 || N > 8) return fail(IDS_EINVAL, "N must be in [1, 8]");
    if (!dims) return fail(IDS_EINVAL, "dims is NULL");
    for (int n = 0; n < N; ++n)
        if (dims[n] < 1 || dims[n] >= (int64_t(1) << 31) - 1) return fail(IDS_EINVAL, "dims[n] out of range");
    if (R < 2) return fail(IDS_EINVAL, "R must be >= 2");
    if (Jlen < 16 || Jlen > 4096 || (Jlen & (Jlen - 1))) return fail(IDS_EINVAL, "Jlen must be a power of two in [16, 4096]");
    if (k < 1 || k >= R || k > Jlen) return fail(IDS_EINVAL, "k must satisfy 1 <= k < R and k <= Jlen");
    if (l != 0 && (l < k || l > Jlen)) return fail(IDS_EINVAL, "l must be 0 (no projection) or satisfy k <= l <= Jlen");
    return IDS_OK;
}

static ids_status tensor_layout(int32_t N, const int64_t* dims, int64_t R, int64_t k, int64_t Jlen, int64_t l,
                                TensorLayout& T, bool csc = false) {
    T.plans = 0;
    for (int n = 0; n < N && !csc; ++n) {   // CSC factors need no bucket plans
        T.ps[n] = plan_shape(dims[n], Jlen);
        T.plans += plan_bytes(T.ps[n]);
    }
    T.tw = align256(sizeof(double2) * (size_t)Jlen);
    T.y = align256(sizeof(double) * (size_t)Jlen * R);
    T.yp = l ? align256(sizeof(double) * (size_t)l * R) : 0;
    T.splits = l ? project_splits(l, Jlen, R, 512) : 1;
    T.part = T.splits > 1 ? align256(sizeof(double) * (size_t)T.splits * l * R) : 0;
    T.gdraw = l ? align256(sizeof(double) * (size_t)l * Jlen) : 0;  // used when G is NULL
    ids_status s = select_plan(l ? l : Jlen, R, k, T.sp);
    if (s) return s;
    T.sel = select_bytes(T.sp);
    T.total = T.plans + T.tw + T.y + T.yp + T.part + T.gdraw + T.sel;
    return IDS_OK;
}

ids_status ids_tensor_workspace_size(int32_t N, const int64_t* dims, int64_t R, int64_t k, int64_t Jlen,
                                     int64_t l, size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(IDS_EINVAL, "bytes is NULL");
    ids_status s = validate_tensor(N, dims, R, k, Jlen, l);
    if (s) return s;
    TensorLayout T;
    if ((s = tensor_layout(N, dims, R, k, Jlen, l, T))) return s;
    *bytes = T.total;
    return IDS_OK;
}

static ids_status tensor_run(int32_t N, const int64_t* dims, int64_t R, const double* const* factors,
                             const int64_t* ld, const int64_t* const* colptr, const int32_t* const* rowind,
                             const double* const* val, const double* lambda, int64_t k, int64_t Jlen, int64_t l,
                             const double* G, uint64_t seed, double* Y, int64_t* J, double* P, double* lambda_hat,
                             int64_t* k_eff, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    const bool csc = colptr != nullptr;
    ids_status s = validate_tensor(N, dims, R, k, Jlen, l);
    if (s) return s;
    if (!lambda || !J || !P || !lambda_hat || !k_eff)
        return fail(IDS_EINVAL, "lambda, J, P, lambda_hat and k_eff must be non-NULL");
    for (int n = 0; n < N; ++n) {
        if (csc) {
            if (!colptr[n] || !rowind[n] || !val[n]) return fail(IDS_EINVAL, "colptr, rowind and val[n] required");
        } else {
            if (!factors[n]) return fail(IDS_EINVAL, "factors[n] is NULL");
            if (ld[n] < dims[n]) return fail(IDS_EINVAL, "ld[n] < dims[n]");
        }
    }
    if (ts_lds_bytes(Jlen) > lds_limit()) return fail(IDS_EINVAL, "Jlen too large for the LDS FFT on this device");
    TensorLayout T;
    if ((s = tensor_layout(N, dims, R, k, Jlen, l, T, csc))) return s;
    if ((s = check_ws(ws, ws_bytes, T.total))) return s;
    hipStream_t st = (hipStream_t)stream;
    char* p = (char*)ws;
    PlanBufs pb[8];
    for (int n = 0; n < N && !csc; ++n) pb[n] = plan_carve(T.ps[n], p);
    double2* tw = (double2*)p;
    p += T.tw;
    double* Yw = (double*)p;
    p += T.y;
    double* Yp = (double*)p;
    p += T.yp;
    double* part = (double*)p;
    p += T.part;
    double* gdraw = (double*)p;
    p += T.gdraw;
    char* sel = p;
    double* Yout = Y ? Y : Yw;
    uint64_t keys[8];
    for (int n = 0; n < N; ++n) keys[n] = stream_key(seed, (uint64_t)n + 1);
    {
        ProfScope ps(PK_PLAN, st);
        if (!csc && (s = plan_build_many(N, T.ps, keys, pb, st))) return s;
        if ((s = twiddles(Jlen, tw, st))) return s;
    }
    {
        ProfScope ps(PK_TS, st);
        if ((s = tensorsketch(N, dims, R, factors, ld, lambda, Jlen, pb, keys, tw, Yout, st, colptr, rowind, val)))
            return s;
    }
    if (l) {
        // Gaussian second stage: Yp (l x R, column-major) = G (l x Jlen) T M
        ProfScope ps(PK_PROJ, st);
        if (!G) {
            if ((s = gaussian_fill(seed, 0, l, Jlen, IDS_F64, gdraw, st))) return s;
            G = gdraw;
        }
        if ((s = project_split(IDS_F64, l, Jlen, R, G, Yout, Jlen, true, Yp, l, T.splits, part, st))) return s;
    }
    if ((s = select_run(T.sp, l ? Yp : Yout, IDS_F64, 1, l ? l : Jlen, J, P, k_eff, status, sel, st))) return s;
    ProfScope ps(PK_LHAT, st);
    return ids::lambda_hat(k, R, P, J, k_eff, lambda, lambda_hat, st);
}

ids_status tensor_id(int32_t N, const int64_t* dims, int64_t R, const double* const* factors, const int64_t* ld,
                     const double* lambda, int64_t k, int64_t Jlen, int64_t l, const double* G, uint64_t seed,
                     double* Y, int64_t* J, double* P, double* lambda_hat, int64_t* k_eff, int32_t* status,
                     void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!factors || !ld) return fail(IDS_EINVAL, "factors and ld must be non-NULL");
    return tensor_run(N, dims, R, factors, ld, nullptr, nullptr, nullptr, lambda, k, Jlen, l, G, seed, Y, J, P,
                      lambda_hat, k_eff, status, ws, ws_bytes, stream);
}

ids_status ids_tensor_csc_workspace_size(int32_t N, const int64_t* dims, int64_t R, int64_t k, int64_t Jlen,
                                         int64_t l, size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(IDS_EINVAL, "bytes is NULL");
    ids_status s = validate_tensor(N, dims, R, k, Jlen, l);
    if (s) return s;
    TensorLayout T;
    if ((s = tensor_layout(N, dims, R, k, Jlen, l, T, true))) return s;
    *bytes = T.total;
    return IDS_OK;
}

ids_status tensor_id_csc(int32_t N, const int64_t* dims, int64_t R, const int64_t* const* colptr,
                         const int32_t* const* rowind, const double* const* val, const double* lambda, int64_t k,
                         int64_t Jlen, int64_t l, const double* G, uint64_t seed, double* Y, int64_t* J, double* P,
                         double* lambda_hat, int64_t* k_eff, int32_t* status, void* ws, size_t ws_bytes,
                         void* stream) {
    g_err.clear();
    if (!colptr || !rowind || !val) return fail(IDS_EINVAL, "colptr, rowind and val must be non-NULL");
    return tensor_run(N, dims, R, nullptr, nullptr, colptr, rowind, val, lambda, k, Jlen, l, G, seed, Y, J, P,
                      lambda_hat, k_eff, status, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// batched
// ---------------------------------------------------------------------------
static ids_status validate_batched(int64_t nprob, const int64_t* m, const int64_t* n, int64_t k, int64_t l,
                                   int64_t l1max) {
    if (nprob < 1 || nprob >= (int64_t(1) << 31)) return fail(IDS_EINVAL, "nprob must be in [1, 2^31)");
    if (!m || !n) return fail(IDS_EINVAL, "m and n must be non-NULL host arrays");
    if (l < 1 || l > 122) return fail(IDS_EINVAL, "batched: l must be in [1, 122]");
    if (k < 1 || k > l) return fail(IDS_EINVAL, "batched: k must be in [1, l]");  // l <= 122 < 128
    if (l1max < l || l1max > 512) return fail(IDS_EINVAL, "batched: l1max must be in [l, 512]");
    for (int64_t q = 0; q < nprob; ++q) {
        if (m[q] < l || m[q] > 4096)
            return fail(IDS_EINVAL, "batched: problem " + std::to_string(q) + ": m must be in [l, 4096]");
        if (n[q] <= k || n[q] >= (int64_t(1) << 31))
            return fail(IDS_EINVAL, "batched: problem " + std::to_string(q) + ": n must exceed k");
        if (n[q] > 1024) return fail(IDS_EINVAL, "batched: problem " + std::to_string(q) + ": n must be <= 1024");
    }
    return IDS_OK;
}

ids_status ids_batched_plan_size(int64_t nprob, size_t* bytes) {
    g_err.clear();
    if (!bytes || nprob < 1) return fail(IDS_EINVAL, "bytes must be non-NULL and nprob >= 1");
    return batched_plan_bytes(nprob, bytes);
}

ids_status ids_batched_plan(int64_t nprob, const int64_t* m, const int64_t* n, int64_t k, int64_t l, int64_t l1max,
                            void* plan, size_t plan_bytes, size_t* ws_bytes, void* stream) {
    g_err.clear();
    ids_status s = validate_batched(nprob, m, n, k, l, l1max);
    if (s) return s;
    if (!plan || !ws_bytes) return fail(IDS_EINVAL, "plan and ws_bytes must be non-NULL");
    return batched_plan(nprob, m, n, k, l, l1max, plan, plan_bytes, ws_bytes, (hipStream_t)stream);
}

static ids_status batched_args(int64_t nprob, const int64_t* m, const int64_t* n, const void* plan, int64_t k,
                               int64_t l, int64_t l1max, double tol, const void* A, const void* G, int64_t* J,
                               double* P, int64_t* k_eff, void* ws, size_t ws_bytes, int64_t* a_elems,
                               int64_t* y_elems, int64_t* r_elems) {
    ids_status s = validate_batched(nprob, m, n, k, l, l1max);
    if (s) return s;
    if (!(tol >= 0.0 && tol < 1.0)) return fail(IDS_EINVAL, "tol must be in [0, 1)");
    if (!plan || !A || !J || !P || !k_eff) return fail(IDS_EINVAL, "plan, A, J, P and k_eff required");
    *a_elems = *y_elems = *r_elems = 0;
    for (int64_t q = 0; q < nprob; ++q) {
        *a_elems += m[q] * n[q];
        *y_elems += l * n[q];
        *r_elems += n[q];
    }
    const size_t need = align256(sizeof(float) * (size_t)*y_elems) +
                        align256(sizeof(double) * (size_t)*r_elems * k) +
                        align256(sizeof(int32_t) * (size_t)*r_elems) + align256(sizeof(double) * (size_t)nprob * k) +
                        align256(sizeof(uint16_t) * (size_t)l * l1max);
    return check_ws(ws, ws_bytes, need);
}

ids_status ids_batched_graph_create(int64_t nprob, const int64_t* m, const int64_t* n, const void* plan, int64_t k,
                                    int64_t l, int64_t l1max, uint64_t seed, double tol, const void* A,
                                    const void* G, int64_t* J, double* P, int64_t* k_eff, int32_t* status,
                                    void* ws, size_t ws_bytes, ids_batched_graph* graph) {
    g_err.clear();
    if (!graph) return fail(IDS_EINVAL, "graph is NULL");
    int64_t ae, ye, re;
    ids_status s = batched_args(nprob, m, n, plan, k, l, l1max, tol, A, G, J, P, k_eff, ws, ws_bytes, &ae, &ye, &re);
    if (s) return s;
    void* h = nullptr;
    if ((s = batched_graph_create(nprob, plan, k, l, l1max, seed, tol, A, G, J, P, k_eff, status, ws, ws_bytes, ae,
                                  ye, re, &h)))
        return s;
    *graph = (ids_batched_graph)h;
    return IDS_OK;
}

ids_status ids_batched_graph_launch(ids_batched_graph graph, void* stream) {
    g_err.clear();
    if (!graph) return fail(IDS_EINVAL, "graph is NULL");
    return batched_graph_launch((void*)graph, (hipStream_t)stream);
}

void ids_batched_graph_destroy(ids_batched_graph graph) { batched_graph_destroy((void*)graph); }

ids_status id_batched(int64_t nprob, const int64_t* m, const int64_t* n, const void* plan, int64_t k, int64_t l,
                      int64_t l1max, uint64_t seed, double tol, const void* A, const void* G, int64_t* J, double* P,
                      int64_t* k_eff, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    int64_t a_elems, y_elems, r_elems;
    ids_status s = batched_args(nprob, m, n, plan, k, l, l1max, tol, A, G, J, P, k_eff, ws, ws_bytes, &a_elems,
                                &y_elems, &r_elems);
    if (s) return s;
    return batched_run(nprob, plan, k, l, l1max, seed, tol, A, G, J, P, k_eff, status, ws, ws_bytes, a_elems,
                       y_elems, r_elems, (hipStream_t)stream);
}

}  // extern "C"
