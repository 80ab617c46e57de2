// C ABI of the condensed spectral-element Helmholtz solver (see include/semcond.h).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/semcond.h"
#include "kernels.h"
#include "layout.h"
#include "noalloc.h"
#include "pcg_persistent.h"
#include "tables.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <chrono>
#include <cstdio>
#include <map>
#include <unordered_map>

using namespace semcond;

namespace {

thread_local std::string g_last_error;

// Device copy of the 1D tables of one scalar type.
template <typename T>
struct DevTables {
    T* buf = nullptr;
    DevTab<T> tab{};
    const T* K = nullptr;  // (p+1)^2 stiffness
};

struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct semcond_ctx {
    int p = 0;
    int n[3] = {0, 0, 0};
    int64_t n_e = 0, N = 0, N_s = 0, N_free = 0;
    Layout L{};
    Tables1D t;
    std::string err;
    // device data
    DevTables<double> t64;
    DevTables<float> t32;
    double* d_widths = nullptr;  // n1 + n2 + n3
    double* d_ax = nullptr;      // [n1 + n2 + n3][2]: h/2, 4/h^2
    double* d_lam_e = nullptr;
    double* d_dcoef = nullptr;
    double* d_diag = nullptr;    // [N_s]
    double* d_pinv64 = nullptr;  // [N_s]
    float* d_pinv32 = nullptr;   // [N_s]
    Geo geo{};
    // workspace (grown on demand)
    Buffer ws_vec;      // vectors for apply / solve
    Buffer ws_scratch;  // element cubes for large p
    Buffer ws_state;    // CG scalars (device)
    Buffer ws_nodal;    // nodal right-hand sides of dual solves
    Buffer ws_persist;  // partials and barrier words of the persistent CG
    Buffer ws_lift;     // prescribed Dirichlet values (transformed) and a temporary
    Buffer ws_slots;    // per-side output slots of the CG applies (layout.h)
    int* h_active = nullptr;  // pinned host copy of CG activity flags
    int h_active_cap = 0;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};  // lagged convergence polls of the fused CG loop
    int* h_flags = nullptr;                       // pinned, written by the fused CG kernels: [kMaxRhs]
    int cg_epoch = 0;                             // numbers the fused CG loops (tags h_flags)
    // persistent CG launch configuration per (k, dtype): (S, G)
    std::map<std::pair<int, int>, std::pair<int, int>> tuned;
    // tracing: event pairs around kernel launches, with the kernel id
    bool prof = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    std::vector<int> ev_kind;    // kernel id per pair
    size_t ev_used = 0;          // events recorded since the last read
    double prof_ms[3] = {0.0, 0.0, 0.0};       // by kernel id: FP64 apply, persistent CG, FP32 apply
    int64_t prof_launches[3] = {0, 0, 0};
    int64_t prof_iters = 0;
    // deterministic assembly: every apply, condensation and CG loop sums the
    // element rows of shared nodes through per-side slots in a fixed order
    bool det = false;         // set by semcond_set_deterministic (applies, condensation, solves)
    bool det_active = false;  // in force for the current call
    // device address of the library's fixed apply workspace on this context's
    // device (semcond_apply_noalloc), looked up at create
    void* noalloc_ws = nullptr;
    // MMC variant (semcond_variant_setup): one dense Schur complement per class
    // of elements with equal metric, column-major n_B x n_B, elements in class
    // order (col_of[e]), and the class ranges of that order
    double* mmc_H = nullptr;
    int* mmc_col = nullptr;
    std::vector<int64_t> mmc_start, mmc_count;
    rocblas_handle blas = nullptr;
    Buffer ws_mmc;  // UL and VL, n_B x n_e k each
    // two-level preconditioner (solve option coarse): the inverse of the
    // trilinear coarse matrix over the free element vertices (from its Cholesky
    // factor), vertex -> coarse unknown map, the transformed 1D hats [t_0; t_1]
    bool coarse_ready = false;
    bool coarse_active = false;  // in force for the current solve
    int n0 = 0;
    double* c_L = nullptr;
    int* c_vmap = nullptr;
    double* c_tw = nullptr;
    Buffer ws_coarse;  // r0, z0 [k][n0], rz_extra [k]
    // D^-1 of the fast diagonalisation per metric class for the FP32 cube
    // applies (6 <= n_I <= 15 and at most kMaxDinvClasses classes; dinv_nc = 0:
    // none, the applies recompute it), and the class of every element
    int dinv_nc = 0;
    int dinv_cap = 0;  // classes the table has room for
    float* d_dinv32 = nullptr;
    int* d_dcls = nullptr;
    double* d_dclass = nullptr;  // [cap][4] metric coefficients of the classes
    // right-hand sides per workgroup of the batched condensation / recovery
    // kernels: fixed by semcond_set_rhs_batch (> 0; -1: the per-item kernels),
    // else timed per k on first use (rhs_tuned: k -> (condensation, recovery);
    // 0 = per-item kernels)
    int rhs_batch_fixed = 0;
    std::map<int, std::pair<int, int>> rhs_tuned;
};

namespace {

// Deterministic assembly in force for the duration of one library call.
struct DetScope {
    semcond_ctx* c;
    bool old;
    DetScope(semcond_ctx* ctx, bool on);
    ~DetScope();
};

int fail(semcond_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    g_last_error = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e__ = (call);                                                            \
        if (e__ != hipSuccess)                                                              \
            return fail((ctx), SEMCOND_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e__)); \
    } while (0)

int grow(semcond_ctx* c, Buffer& b, size_t bytes) {
    if (b.bytes >= bytes) return SEMCOND_OK;
    if (b.ptr) {
        hipDeviceSynchronize();
        hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    if (hipMalloc(&b.ptr, bytes) != hipSuccess) {
        b.ptr = nullptr;
        return fail(c, SEMCOND_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = bytes;
    return SEMCOND_OK;
}

template <typename T>
int upload_tables(semcond_ctx* c, DevTables<T>& d) {
    const Tables1D& t = c->t;
    const int NI = t.NI, n = t.p + 1;
    const size_t count = 3 * NI + 4 * (size_t)NI * NI + n + (size_t)n * n;
    std::vector<T> h(count);
    size_t o = 0;
    auto put = [&](const std::vector<double>& v) {
        for (double x : v) h[o++] = (T)x;
    };
    put(t.lam);
    put(t.a);
    put(t.b);
    put(t.S);
    for (int i = 0; i < NI; ++i)
        for (int m = 0; m < NI; ++m) h[o++] = (T)t.S[(size_t)m * NI + i];  // S^T
    put(t.Sinv);
    put(t.SinvT);
    put(t.w);
    put(t.K);
    HIPCHK(c, hipMalloc(&d.buf, count * sizeof(T)));
    HIPCHK(c, hipMemcpy(d.buf, h.data(), count * sizeof(T), hipMemcpyHostToDevice));
    T* b = d.buf;
    d.tab.lam = b;
    d.tab.a = b + NI;
    d.tab.b = b + 2 * NI;
    d.tab.S = b + 3 * NI;
    d.tab.St = d.tab.S + NI * NI;
    d.tab.Sinv = d.tab.St + NI * NI;
    d.tab.SinvT = d.tab.Sinv + NI * NI;
    d.tab.w = d.tab.SinvT + NI * NI;
    d.K = d.tab.w + n;
    d.tab.m0 = (T)t.m0;
    d.tab.K00 = (T)t.K00;
    d.tab.K0p = (T)t.K0p;
    return SEMCOND_OK;
}

DetScope::DetScope(semcond_ctx* ctx, bool on) : c(ctx), old(ctx->det_active) { c->det_active = on; }
DetScope::~DetScope() { c->det_active = old; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int check_dtype(semcond_ctx* c, int dtype) {
    if (dtype != SEMCOND_F64 && dtype != SEMCOND_F32) return fail(c, SEMCOND_EINVAL, "dtype must be F64 or F32");
    return SEMCOND_OK;
}

int check_k(semcond_ctx* c, int k) {
    if (k < 1 || k > 256) return fail(c, SEMCOND_EINVAL, "k must be in [1, 256]");
    // the apply kernels address [N_s][k] arrays with 32-bit offsets
    if (c && c->N_s * (int64_t)k >= (int64_t(1) << 31))
        return fail(c, SEMCOND_EINVAL, "N_s * k must stay below 2^31");
    return SEMCOND_OK;
}

template <typename T>
const DevTab<T>& tabs(semcond_ctx* c);

template <>
const DevTab<double>& tabs<double>(semcond_ctx* c) { return c->t64.tab; }
template <>
const DevTab<float>& tabs<float>(semcond_ctx* c) { return c->t32.tab; }


template <typename T>
const T* pinv(semcond_ctx* c);
template <>
const double* pinv<double>(semcond_ctx* c) { return c->d_pinv64; }
template <>
const float* pinv<float>(semcond_ctx* c) { return c->d_pinv32; }

// Start / end event of a traced launch of kernel `kind` on stream st.
int profile_begin(semcond_ctx* c, int kind, hipStream_t st) {
    if (c->ev_used + 2 > c->ev.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
        c->ev_kind.resize(c->ev.size() / 2);
    }
    c->ev_kind[c->ev_used / 2] = kind;
    HIPCHK(c, hipEventRecord(c->ev[c->ev_used], st));
    return SEMCOND_OK;
}

int profile_end(semcond_ctx* c, hipStream_t st) {
    HIPCHK(c, hipEventRecord(c->ev[c->ev_used + 1], st));
    c->ev_used += 2;
    return SEMCOND_OK;
}

// Apply arguments of this context (operand, result and options set by the caller).
template <typename T>
ApplyArgs<T> apply_args(semcond_ctx* c) {
    ApplyArgs<T> a;
    a.g = c->geo;
    a.tab = tabs<T>(c);
    a.u = nullptr;
    a.v = nullptr;
    a.k = 0;
    a.energy = nullptr;
    a.e_begin = 0;
    if constexpr (sizeof(T) == 4) {
        if (c->dinv_nc > 0) {
            a.dinv = c->d_dinv32;
            a.dcls = c->d_dcls;
        }
    }
    return a;
}

template <typename T>
hipError_t launch_apply(const ApplyArgs<T>& a, int64_t n_elem, hipStream_t st) {
    return launch_apply_tpt<T>(a, n_elem, st);
}

// v = H~^ u (transformed).  v is zeroed first unless v_is_zero.  energy: optional [n_e][k].
// With dir_r set, the operand is the CG direction fmadd(beta, u, pinv r) (u:
// previous direction) and q = v must be zero on entry.
// Multivector layouts: [N_s][k] (RHS innermost, the library's interface) and
// [k][N_s] (RHS-major, inside the conjugate gradients).
enum VecLayout { NODE_MAJOR = 0, RHS_MAJOR = 1 };

// The CG applies address one right-hand side's vectors and slots with 32-bit
// byte offsets: N_s and the slot length times the value size below 2^32.
template <typename T>
bool cg_offsets_fit(const semcond_ctx* c) {
    const uint64_t lim = uint64_t(1) << 32;
    return (uint64_t)c->N_s * sizeof(T) < lim && (uint64_t)slot_len(c->L) * sizeof(T) < lim;
}
const char* const cg_offsets_msg = "conjugate gradients: skeleton beyond 32-bit byte offsets per right-hand side";

// Whether the CG applies that use slots store face rows into slots as well
// (else faces are added into q; edges and vertices use slots).  Measured on
// MI355X: the FP32 loop is faster with face slots, the FP64 loop with face
// additions (fewer bytes for the step to read).
template <typename T>
constexpr int cg_face_slots() { return sizeof(T) == 4 ? 1 : 0; }

template <typename T>
int apply_transformed(semcond_ctx* c, const T* u, T* v, int k, VecLayout lay, double* energy, hipStream_t st,
                      bool v_is_zero = false, const T* dir_r = nullptr, const double* dir_beta = nullptr,
                      int read_con = 0, const CgFuse* fz = nullptr, const int* act = nullptr,
                      T* slots = nullptr, int face_slots = cg_face_slots<T>()) {
    if (c->det_active && !slots && !dir_r) {
        // deterministic plain apply: every row into its per-side slot, then the
        // fixed-order slot sums written into v (all entries)
        const int64_t qlen = slot_len(c->L);
        if (qlen * (int64_t)k >= (int64_t(1) << 31))
            return fail(c, SEMCOND_EINVAL, "deterministic apply: slot workspace beyond 2^31 entries");
        int rc = grow(c, c->ws_slots, (size_t)qlen * k * sizeof(T));
        if (rc) return rc;
        T* Q = (T*)c->ws_slots.ptr;
        HIPCHK(c, launch_fill<T>(Q, qlen * k, (T)0, st));
        rc = apply_transformed<T>(c, u, v, k, lay, energy, st, true, nullptr, nullptr, read_con, nullptr, nullptr,
                                  Q, 1);
        if (rc) return rc;
        HIPCHK(c, launch_slot_sum<T>(c->L, Q, qlen, v, k, lay == RHS_MAJOR ? 1u : (uint32_t)k,
                                     lay == RHS_MAJOR ? (uint32_t)c->N_s : 1u, st));
        return SEMCOND_OK;
    }
    if (!v_is_zero) HIPCHK(c, launch_fill<T>(v, c->N_s * k, (T)0, st));
    ApplyArgs<T> a = apply_args<T>(c);
    a.u = u;
    a.v = v;
    a.k = k;
    a.ns = lay == RHS_MAJOR ? 1u : (uint32_t)k;
    a.rs = lay == RHS_MAJOR ? (uint32_t)c->N_s : 1u;
    a.read_con = read_con;
    a.energy = energy;
    if (dir_r) {
        if (!dir_beta) return fail(c, SEMCOND_EINVAL, "fused direction needs beta");
        if (lay != RHS_MAJOR) return fail(c, SEMCOND_EINVAL, "fused direction needs RHS-major vectors");
        if (!cg_offsets_fit<T>(c)) return fail(c, SEMCOND_EINVAL, cg_offsets_msg);
        if (slots && face_slots != cg_face_slots<T>())
            return fail(c, SEMCOND_EINVAL, "CG applies keep face rows in slots exactly in FP32");
        a.dir_r = dir_r;
        a.dir_pinv = pinv<T>(c);
        a.dir_beta = dir_beta;
        if (fz) a.fz = *fz;
    }
    a.act = act;
    if (slots) {
        if (!v_is_zero) return fail(c, SEMCOND_EINVAL, "slot output needs a zeroed v");
        a.slots = slots;
        a.qlen = slot_len(c->L);
        a.face_slots = face_slots;
    }
    if (c->prof) {
        int rc = profile_begin(c, sizeof(T) == 4 ? SEMCOND_KERNEL_APPLY_F32 : SEMCOND_KERNEL_APPLY, st);
        if (rc) return rc;
        HIPCHK(c, launch_apply<T>(a, c->n_e, st));
        return profile_end(c, st);
    }
    HIPCHK(c, launch_apply<T>(a, c->n_e, st));
    return SEMCOND_OK;
}

// Accumulate the recorded event pairs into the profile totals.
int profile_flush(semcond_ctx* c) {
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        HIPCHK(c, hipEventSynchronize(c->ev[i + 1]));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        const int kind = c->ev_kind[i / 2];
        c->prof_ms[kind] += ms;
        c->prof_launches[kind] += 1;
    }
    c->ev_used = 0;
    return SEMCOND_OK;
}

template <typename T>
const T* transform_matrix(semcond_ctx* c, int direction) {
    const DevTab<T>& t = tabs<T>(c);
    switch (direction) {
        case SEMCOND_COEF_TO_TRANSFORMED: return t.Sinv;
        case SEMCOND_COEF_TO_PHYSICAL: return t.S;
        case SEMCOND_DUAL_TO_TRANSFORMED: return t.St;
        case SEMCOND_DUAL_TO_PHYSICAL: return t.SinvT;
        default: return nullptr;
    }
}

int scratch_for_cubes(semcond_ctx* c, int* grid, double** scratch) {
    bool need = false;
    *grid = rhs_grid_for_scratch(c->p, c->n_e, &need);
    *scratch = nullptr;
    if (need) {
        const size_t n = (size_t)(c->p + 1);
        int rc = grow(c, c->ws_scratch, (size_t)(*grid) * n * n * n * sizeof(double));
        if (rc) return rc;
        *scratch = (double*)c->ws_scratch.ptr;
    }
    return SEMCOND_OK;
}

// Right-hand sides per workgroup of the batched condensation (kind 0) or
// recovery (kind 1) for k right-hand sides: 0 = the per-item kernels, -1 = not
// yet timed.
int rhs_batch(const semcond_ctx* c, int k, int kind) {
    if (!rhs_batched_supported(c->L, c->N) || c->rhs_batch_fixed < 0) return 0;
    if (c->rhs_batch_fixed > 0) return std::min(c->rhs_batch_fixed, k);
    auto it = c->rhs_tuned.find(k);
    if (it == c->rhs_tuned.end()) return -1;
    return kind ? it->second.second : it->second.first;
}

// Times run(R) for the candidate batch sizes (per-item kernels, 1, 2, 4, 8,
// 16 up to k; two rounds, the faster of each) on stream st and returns the
// fastest in *best.  run must be repeatable (the callers clear what it adds
// into).
template <class Run>
int tune_rhs_batch(semcond_ctx* c, int k, hipStream_t st, Run&& run, int* best) {
    std::vector<int> cand{0};
    for (int R = 1; R <= 16 && R <= k; R *= 2) cand.push_back(R);
    std::vector<float> ms(cand.size(), 1e30f);
    hipEvent_t ev[2];
    HIPCHK(c, hipEventCreate(&ev[0]));
    HIPCHK(c, hipEventCreate(&ev[1]));
    int rc = SEMCOND_OK;
    for (int round = 0; round < 2 && !rc; ++round)
        for (size_t i = 0; i < cand.size() && !rc; ++i) {
            hipError_t e = hipEventRecord(ev[0], st);
            if (e == hipSuccess) rc = run(cand[i]);
            if (!rc && e == hipSuccess) e = hipEventRecord(ev[1], st);
            if (!rc && e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float t = 0.0f;
            if (!rc && e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
            if (!rc && e != hipSuccess) rc = fail(c, SEMCOND_EDEVICE, std::string("batch timing: ") + hipGetErrorString(e));
            if (!rc) ms[i] = std::min(ms[i], t);
        }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (rc) return rc;
    *best = cand[std::min_element(ms.begin(), ms.end()) - ms.begin()];
    return SEMCOND_OK;
}

// fhat (FP64, transformed) = condensed RHS of nodal f.
int condense_rhs64(semcond_ctx* c, const double* f, double* fhat, int k, hipStream_t st, SkelStride sk = {}) {
    int grid;
    double* scratch;
    int rc = scratch_for_cubes(c, &grid, &scratch);
    if (rc) return rc;
    // Rows go into per-side slots, summed in a fixed order afterwards, in
    // deterministic mode; otherwise they are added with atomics (measured
    // faster than slots with the batched kernels too: 2.6 against 2.7 ms plus
    // 0.4 ms of slot sums and 0.3 ms of clearing at 24^3 elements, p = 12, 16 RHS).
    const int64_t qlen = slot_len(c->L);
    if (c->det_active && qlen * (int64_t)k >= (int64_t(1) << 31))
        return fail(c, SEMCOND_EINVAL, "deterministic condensation: slot workspace beyond 2^31 entries");
    auto run = [&](int R) -> int {
        double* slots = nullptr;
        if (c->det_active) {
            int rc2 = grow(c, c->ws_slots, (size_t)qlen * k * sizeof(double));
            if (rc2) return rc2;
            slots = (double*)c->ws_slots.ptr;
            HIPCHK(c, launch_fill<double>(slots, qlen * k, 0.0, st));
        } else {
            HIPCHK(c, launch_fill<double>(fhat, c->N_s * k, 0.0, st));
        }
        HIPCHK(c, launch_condense_rhs(c->geo, c->t64.tab, f, c->N, fhat, k, scratch, grid, slots, st, sk, R));
        return SEMCOND_OK;
    };
    int R = rhs_batch(c, k, 0);
    if (R < 0) {
        rc = tune_rhs_batch(c, k, st, run, &R);
        if (rc) return rc;
        auto it = c->rhs_tuned.emplace(k, std::make_pair(-1, -1)).first;
        it->second.first = R;
    }
    return run(R);
}

// Interior recovery with the batch size of this context for k (timed on first use).
int recover_interior64(semcond_ctx* c, const double* f, const double* xs, double* u, int k, int keep,
                       hipStream_t st, SkelStride sk = {}) {
    int grid;
    double* scratch;
    int rc = scratch_for_cubes(c, &grid, &scratch);
    if (rc) return rc;
    auto run = [&](int R) -> int {
        HIPCHK(c, launch_recover_interior(c->geo, c->t64.tab, f, c->N, xs, u, k, scratch, grid, keep, st, sk, R));
        return SEMCOND_OK;
    };
    int R = rhs_batch(c, k, 1);
    if (R < 0) {
        rc = tune_rhs_batch(c, k, st, run, &R);
        if (rc) return rc;
        auto it = c->rhs_tuned.emplace(k, std::make_pair(-1, -1)).first;
        it->second.second = R;
    }
    return run(R);
}

struct CgWork {
    CgState s;
    double* partials;  // [3][vec_blocks(k)][k] (room for [3][kVecBlocks][k])
    double* energy;    // [n_e][k]
    double* epart;     // [kEnergyBlocks][k]: first-stage sums of the energies
    double* rho1;      // second slots of rho, active and the stagnation state
    int* act1;         // (fused loop, odd iterations)
    double* rrb1;
    int* stall1;
    double* alpha1;    // second alpha slot (fused loop, odd iterations)
};

// Device state layout inside ws_state: two independent CG states (slot 0 for
// the CG iteration, slot 1 for the outer refinement loop of MIXED_IR).
int cg_state(semcond_ctx* c, int k, int slot, CgWork* w) {
    const size_t nd = 11 * (size_t)k + 1;  // rho pq alpha beta rr bb (6k), rho slot 1, rrb (2 slots), tol2, xa,
                                           // alpha slot 1
    const size_t ni = 6 * (size_t)k;      // active iters status, active slot 1, stall (2 slots)
    const size_t np = 3 * (size_t)kVecBlocks * k;
    const size_t ne = (size_t)c->n_e * k;
    const size_t nep = (size_t)kEnergyBlocks * k;
    const size_t one = ((nd + np + ne + nep) * sizeof(double) + ni * sizeof(int) + 255) / 256 * 256;
    int rc = grow(c, c->ws_state, 2 * one);
    if (rc) return rc;
    double* d = (double*)((char*)c->ws_state.ptr + slot * one);
    w->s.rho = d;
    w->s.pq = d + k;
    w->s.alpha = d + 2 * k;
    w->s.beta = d + 3 * k;
    w->s.rr = d + 4 * k;
    w->s.bb = d + 5 * k;
    w->rho1 = d + 6 * k;
    w->s.rrb = d + 7 * k;
    w->rrb1 = d + 8 * k;
    w->s.tol2 = d + 9 * k;
    w->s.xa = d + 9 * k + 1;
    w->alpha1 = d + 10 * k + 1;
    w->s.window = 0;
    w->partials = d + nd;
    w->energy = w->partials + np;
    w->epart = w->energy + ne;
    int* ip = (int*)(w->epart + nep);
    w->s.active = ip;
    w->s.iters = ip + k;
    w->s.status = ip + 2 * k;
    w->act1 = ip + 3 * k;
    w->s.stall = ip + 4 * k;
    w->stall1 = ip + 5 * k;
    if (c->h_active_cap < 3 * k) {
        if (c->h_active) hipHostFree(c->h_active);
        c->h_active = nullptr;
        c->h_active_cap = 0;
        if (hipHostMalloc((void**)&c->h_active, 3 * k * sizeof(int)) != hipSuccess)
            return fail(c, SEMCOND_ENOMEM, "pinned host allocation failed");
        c->h_active_cap = 3 * k;
    }
    return SEMCOND_OK;
}

struct CgHost {
    std::vector<double> rr, bb;
    std::vector<int> iters, status, active;
};

int read_state(semcond_ctx* c, const CgWork& w, int k, CgHost* h, hipStream_t st) {
    h->rr.resize(k);
    h->bb.resize(k);
    h->iters.resize(k);
    h->status.resize(k);
    h->active.resize(k);
    HIPCHK(c, hipMemcpyAsync(h->rr.data(), w.s.rr, k * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(h->bb.data(), w.s.bb, k * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(h->iters.data(), w.s.iters, k * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(h->status.data(), w.s.status, k * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(h->active.data(), w.s.active, k * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return SEMCOND_OK;
}

// Largest n_e k for which the CG loop completes its reductions inside the
// consuming kernels.
constexpr int64_t kFusedMaxItems = 16384;

// Iterations without the residual norm halving after which an inner FP32
// solve of the iterative refinement stops (its outer step then recomputes
// the FP64 residual).
constexpr int kInnerStallWindow = 64;

// Views of the CG state for iteration parity ph (slot ph: this iteration's
// rho / active; slot 1 - ph: the previous iteration's); the apply's partial
// sums are set by the caller from the second iteration on.
CgFuse fuse_view(const CgWork& w, int k, int ph, int64_t n_e) {
    CgFuse f = {};
    double* rho[2] = {w.s.rho, w.rho1};
    int* act[2] = {w.s.active, w.act1};
    double* rrb[2] = {w.s.rrb, w.rrb1};
    int* stall[2] = {w.s.stall, w.stall1};
    f.part = w.partials;
    f.nsb = fused_step_blocks(k);
    f.energy = w.energy;
    f.n_e = n_e;
    f.rho_prev = rho[1 - ph];
    f.act_prev = act[1 - ph];
    f.rho = rho[ph];
    f.act = act[ph];
    f.beta = w.s.beta;
    f.rr = w.s.rr;
    f.iters = w.s.iters;
    f.status = w.s.status;
    f.bb = w.s.bb;
    f.tol2 = w.s.tol2;
    f.pq = w.s.pq;
    // x is read and written at odd iterations only (both steps' updates at
    // once); an even iteration's alpha waits in slot 0 for the next step, or
    // for the flush at the end of the loop
    f.alpha = ph ? w.alpha1 : w.s.alpha;
    f.alpha_prev = ph ? w.s.alpha : w.alpha1;
    f.x_mode = ph ? CG_X_FLUSH : CG_X_DEFER;
    f.rrb_prev = rrb[1 - ph];
    f.rrb = rrb[ph];
    f.stall_prev = stall[1 - ph];
    f.stall = stall[ph];
    f.window = w.s.window;
    f.host_act = nullptr;
    f.epoch2 = 0;
    return f;
}

// Start of a CG solve: tolerance, r = b - A x (x0_given) or x = 0, r = b; q = 0;
// rho = r.z, b.b, activity.  keep_dir: the direction p of the previous solve on
// these buffers is continued (first beta = r.z / the r.z that formed it), as a
// refinement step that replaces the residual without restarting the Krylov
// recurrence; otherwise p = 0.
template <typename T>
int cg_start(semcond_ctx* c, const T* b, T* x, T* r, T* p, T* q, int k, double tol, bool x0_given, bool keep_dir,
             CgWork& w, hipStream_t st) {
    const int64_t Ns = c->N_s;
    const double tol2 = tol * tol;
    HIPCHK(c, hipMemcpyAsync(w.s.tol2, &tol2, sizeof(double), hipMemcpyHostToDevice, st));
    if (x0_given) {
        int rc = apply_transformed<T>(c, x, q, k, RHS_MAJOR, nullptr, st);
        if (rc) return rc;
        HIPCHK(c, launch_cg_init<T>(b, q, pinv<T>(c), r, p, Ns, k, w.partials, st, keep_dir));
    } else {
        HIPCHK(c, launch_fill<T>(x, Ns * k, (T)0, st));
        HIPCHK(c, launch_fill<T>(q, Ns * k, (T)0, st));
        HIPCHK(c, launch_cg_init<T>(b, (T*)nullptr, pinv<T>(c), r, p, Ns, k, w.partials, st, keep_dir));
    }
    HIPCHK(c, launch_cg_reduce(w.partials, vec_blocks(k), 3, k, w.s, keep_dir ? RED_INIT_KEEP : RED_INIT, st));
    return SEMCOND_OK;
}

// Preconditioned CG on the transformed condensed system, k RHS, type T.
// b, x, r, p, q: [N_s][k] of T.  x holds the initial guess on entry (x0_given)
// or is zeroed.  Returns per-RHS iterations/status through the state.
template <typename T>
int run_cg(semcond_ctx* c, const T* b, T* x, T* r, T* p, T* q, int k, double tol, int max_iter,
           int check_every, bool x0_given, CgWork& w, hipStream_t st, bool keep_dir = false) {
    const int64_t Ns = c->N_s;
    int rc0 = cg_start<T>(c, b, x, r, p, q, k, tol, x0_given, keep_dir, w, st);
    if (rc0) return rc0;
    if (check_every < 1) check_every = 1;
    // Small problems complete both reductions inside the kernels that consume
    // them (two launches per iteration instead of four); the redundant reads
    // of the partial sums grow with n_e k.
    const bool fused = !c->det_active && c->n_e * (int64_t)k <= kFusedMaxItems;
    // In the loop with separate reductions the applies store per-side slots of
    // edges and vertices (faces too in FP32; plain stores, no atomics) that the
    // step sums in a fixed order; cleared here, so that slots no element writes
    // read 0.  Where they measured faster on MI355X: not in the small fused
    // loop (its step is latency-bound and reads fewer values with additions),
    // not at p = 2 (one node per entity: 5 % slower), and in FP64 only while one
    // wave holds an element (n_I <= 8; at p = 12 with 16 RHS 5 % slower).
    T* Q = nullptr;
    const int64_t qlen = slot_len(c->L);
    // (deterministic mode: always, so that no edge or vertex row is added by atomics)
    const bool slots = c->det_active || (!fused && c->L.NI >= 3 && (sizeof(T) == 4 || c->L.NI <= 8));
    if (c->det_active && qlen * (int64_t)k >= (int64_t(1) << 31))
        return fail(c, SEMCOND_EINVAL, "deterministic solve: slot workspace beyond 2^31 entries");
    if (slots && qlen * (int64_t)k < (int64_t(1) << 31)) {
        rc0 = grow(c, c->ws_slots, (size_t)qlen * k * sizeof(T));
        if (rc0) return rc0;
        Q = (T*)c->ws_slots.ptr;
        HIPCHK(c, launch_fill<T>(Q, qlen * k, (T)0, st));
    }
    if (fused) {
        for (hipEvent_t& e : c->poll_ev)
            if (!e) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        if (!c->h_flags && hipHostMalloc((void**)&c->h_flags, kMaxRhs * sizeof(int), hipHostMallocCoherent) !=
                               hipSuccess)
            return fail(c, SEMCOND_ENOMEM, "pinned host allocation failed");
        // a flag counts as "stopped" only when a kernel of this loop wrote it
        c->cg_epoch = (c->cg_epoch + 1) & 0x3FFFFFFF;
    }
    const int epoch2 = 2 * c->cg_epoch;
    if (fused) {
        // every flag starts as "active" in this loop's numbering: the first
        // poll with check_every = 1 reads them before any kernel of this loop
        // has written one, and a pinned buffer recycled from another context
        // may hold that context's "stopped" value of the same number (no kernel
        // writes them now: the previous solve ended with a synchronisation)
        for (int i = 0; i < k; ++i) __atomic_store_n(c->h_flags + i, epoch2 + 1, __ATOMIC_RELEASE);
    }
    auto none_active = [&](const int* h) {
        for (int i = 0; i < k; ++i)
            if (h[i]) return false;
        return true;
    };
    int n_it = 0, pending = -1;
    for (int it = 0; it < max_iter; ++it) {
        if (it % check_every == 0 && !(fused && it == 0)) {
            // (the fused loop needs no check before its first iteration: a RHS
            // that is converged from the start exits every kernel at once)
            if (fused) {
                // Lagged poll: the kernels write the flags to pinned host memory
                // as they decide them; the host waits for the event recorded one
                // check interval earlier (the queue never drains) and reads them.
                // Iterations queued after convergence exit at once.
                const int b = (it / check_every) & 1;
                HIPCHK(c, hipEventRecord(c->poll_ev[b], st));
                if (pending >= 0) {
                    HIPCHK(c, hipEventSynchronize(c->poll_ev[pending]));
                    bool stopped = true;
                    for (int i = 0; i < k; ++i) stopped &= __atomic_load_n(c->h_flags + i, __ATOMIC_ACQUIRE) == epoch2;
                    if (stopped) break;
                }
                pending = b;
            } else {
                HIPCHK(c, hipMemcpyAsync(c->h_active, w.s.active, k * sizeof(int), hipMemcpyDeviceToHost, st));
                HIPCHK(c, hipStreamSynchronize(st));
                if (none_active(c->h_active)) break;
            }
        }
        // The apply writes the slots Q and adds face rows (all rows without Q)
        // into q, which is zero here: zeroed at start and by every step.  It
        // forms the direction p = beta p + z at its gather; the step stores it.
        if (fused) {
            // slot it & 1 is this iteration's rho / active, the other the previous one's
            CgFuse f = fuse_view(w, k, it & 1, c->n_e);
            f.host_act = c->h_flags;
            f.epoch2 = epoch2;
            int rc = apply_transformed<T>(c, p, q, k, RHS_MAJOR, w.energy, st, true, r, w.s.beta, 0,
                                          it > 0 ? &f : nullptr, nullptr, Q);
            if (rc) return rc;
            HIPCHK(c, launch_cg_step_fused<T>(x, r, p, q, pinv<T>(c), Ns, k, f, w.partials, Q, qlen, c->L,
                                              cg_face_slots<T>(), st));
        } else {
            int rc = apply_transformed<T>(c, p, q, k, RHS_MAJOR, w.energy, st, true, r, w.s.beta, 0, nullptr,
                                          w.s.active, Q);
            if (rc) return rc;
            HIPCHK(c, launch_energy_pq(w.energy, c->n_e, k, w.epart, w.s, st));
            // x is read and written at odd steps only (both steps' updates at
            // once): the even step's length waits in xa, its direction in p
            const bool defer = (it & 1) == 0;
            HIPCHK(c, launch_cg_step<T>(x, r, p, q, pinv<T>(c), Ns, k, w.s, w.partials, Q, qlen, c->L,
                                        cg_face_slots<T>(), st, false, defer ? CG_X_DEFER : CG_X_FLUSH));
            HIPCHK(c, launch_cg_reduce(w.partials, vec_blocks(k), 2, k, w.s, defer ? RED_RZ_DEFER : RED_RZ, st));
        }
        n_it = it + 1;
    }
    // right-hand sides whose last step deferred its update (xa != 0)
    if (!fused && n_it > 0) HIPCHK(c, launch_cg_x_flush<T>(x, p, Ns, k, w.s, st));
    if (fused && n_it > 0) {
        // the last step's r.z reduction, then the state back in slot 0
        const bool odd = ((n_it - 1) & 1) != 0;
        CgState v = w.s;
        if (odd) {
            v.rho = w.rho1;
            v.active = w.act1;
            v.rrb = w.rrb1;
            v.stall = w.stall1;
        }
        HIPCHK(c, launch_cg_reduce(w.partials, fused_step_blocks(k), 2, k, v, RED_RZ, st));
        if (odd) {
            HIPCHK(c, hipMemcpyAsync(w.s.rho, w.rho1, k * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipMemcpyAsync(w.s.active, w.act1, k * sizeof(int), hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipMemcpyAsync(w.s.rrb, w.rrb1, k * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipMemcpyAsync(w.s.stall, w.stall1, k * sizeof(int), hipMemcpyDeviceToDevice, st));
        }
        // right-hand sides whose last step (of even index: an odd step count)
        // deferred its x update; its alpha is in slot 0, its direction in p
        HIPCHK(c, launch_cg_x_flush_parity<T>(x, p, Ns, k, w.s.iters, w.s.alpha, st));
    }
    return SEMCOND_OK;
}

// The element metric coefficients d_e as the kernels compute them, [n_e][4] on the host.
int element_metrics_host(semcond_ctx* c, hipStream_t st, std::vector<double>& hd) {
    hd.assign(4 * (size_t)c->n_e, 0.0);
    double* dd = nullptr;
    HIPCHK(c, hipMalloc(&dd, hd.size() * sizeof(double)));
    hipError_t e1 = launch_elem_metrics(c->geo, dd, st);
    hipError_t e2 =
        e1 == hipSuccess ? hipMemcpyAsync(hd.data(), dd, hd.size() * sizeof(double), hipMemcpyDeviceToHost, st) : e1;
    hipError_t e3 = e2 == hipSuccess ? hipStreamSynchronize(st) : e2;
    hipFree(dd);
    HIPCHK(c, e3);
    return SEMCOND_OK;
}

// Metric classes (elements with bitwise equal d_e) and their D^-1 tables for
// the FP32 cube applies.  Meshes with more classes than kMaxDinvClasses (for
// example per-element lambda_e) keep recomputing D^-1 at every point: a table
// per element would add n_I^3 values of traffic per element and RHS.
constexpr int kMaxDinvClasses = 64;

int build_dinv_tables(semcond_ctx* c, hipStream_t st) {
    c->dinv_nc = 0;
    const int NI = c->L.NI;
    if (NI < 6 || NI > 15) return SEMCOND_OK;
    std::vector<double> hd;
    int rc = element_metrics_host(c, st, hd);
    if (rc) return rc;
    struct Key {
        uint64_t w[4];
        bool operator==(const Key& o) const { return std::memcmp(w, o.w, sizeof(w)) == 0; }
    };
    struct KeyHash {
        size_t operator()(const Key& k) const {
            uint64_t h = 1469598103934665603ull;
            for (uint64_t x : k.w) h = (h ^ x) * 1099511628211ull;
            return (size_t)h;
        }
    };
    std::unordered_map<Key, int, KeyHash> cls;
    std::vector<int> cl(c->n_e);
    std::vector<double> coef;
    for (int64_t e = 0; e < c->n_e; ++e) {
        Key key;
        std::memcpy(key.w, hd.data() + 4 * e, sizeof(key.w));
        auto it = cls.find(key);
        if (it == cls.end()) {
            if ((int)cls.size() == kMaxDinvClasses) return SEMCOND_OK;  // too many: recompute
            it = cls.emplace(key, (int)cls.size()).first;
            coef.insert(coef.end(), hd.begin() + 4 * e, hd.begin() + 4 * e + 4);
        }
        cl[e] = it->second;
    }
    const int nc = (int)cls.size();
    const size_t n3 = (size_t)NI * NI * NI;
    if (nc > c->dinv_cap) {
        hipFree(c->d_dinv32);
        hipFree(c->d_dclass);
        c->d_dinv32 = nullptr;
        c->d_dclass = nullptr;
        c->dinv_cap = 0;
        HIPCHK(c, hipMalloc(&c->d_dinv32, nc * n3 * sizeof(float)));
        HIPCHK(c, hipMalloc(&c->d_dclass, nc * 4 * sizeof(double)));
        c->dinv_cap = nc;
    }
    if (!c->d_dcls) HIPCHK(c, hipMalloc(&c->d_dcls, c->n_e * sizeof(int)));
    HIPCHK(c, hipMemcpy(c->d_dclass, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_dcls, cl.data(), cl.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, launch_dinv_table(c->t64.tab.lam, NI, c->d_dclass, nc, c->d_dinv32, st));
    c->dinv_nc = nc;
    return SEMCOND_OK;
}

// Upload lambda / lambda_e / dcoef_e (validated by the caller) and rebuild the
// preconditioner diagonal and its inverses.
int set_coefficients(semcond_ctx* c, double lambda, const double* lambda_e, const double* dcoef_e, hipStream_t st) {
    const int64_t ne = c->n_e;
    if (lambda_e) {
        if (!c->d_lam_e) HIPCHK(c, hipMalloc(&c->d_lam_e, ne * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->d_lam_e, lambda_e, ne * sizeof(double), hipMemcpyHostToDevice));
    }
    if (dcoef_e) {
        if (!c->d_dcoef) HIPCHK(c, hipMalloc(&c->d_dcoef, 4 * ne * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->d_dcoef, dcoef_e, 4 * ne * sizeof(double), hipMemcpyHostToDevice));
    }
    c->geo.lam = lambda;
    c->coarse_ready = false;  // the coarse matrix holds the old metric
    c->geo.lam_e = lambda_e ? c->d_lam_e : nullptr;
    c->geo.dcoef = dcoef_e ? c->d_dcoef : nullptr;
    // the diagonal's rows of shared nodes are summed through per-side slots in
    // a fixed order, so every context of a mesh has bitwise the same diagonal
    const int64_t qlen = slot_len(c->L);
    int rc = grow(c, c->ws_slots, (size_t)qlen * sizeof(double));
    if (rc) return rc;
    HIPCHK(c, launch_fill<double>((double*)c->ws_slots.ptr, qlen, 0.0, st));
    HIPCHK(c, launch_precond_diag(c->geo, c->t64.tab, c->d_diag, (double*)c->ws_slots.ptr, st));
    HIPCHK(c, launch_precond_invert<double>(c->L, c->d_diag, c->d_pinv64, st));
    HIPCHK(c, launch_precond_invert<float>(c->L, c->d_diag, c->d_pinv32, st));
    return build_dinv_tables(c, st);
}

// Validation shared by create and update: returns an error message or NULL.
const char* check_coefficients(int64_t ne, unsigned mask, double lambda, const double* lambda_e, const double* dcoef_e) {
    if (!lambda_e && !dcoef_e && !(std::isfinite(lambda) && lambda >= 0.0)) return "lambda must be finite and >= 0";
    bool any_d0 = !lambda_e && !dcoef_e && lambda > 0.0;
    if (lambda_e)
        for (int64_t e = 0; e < ne; ++e) {
            if (!(std::isfinite(lambda_e[e]) && lambda_e[e] >= 0.0)) return "lambda_e must be finite and >= 0";
            any_d0 |= lambda_e[e] > 0.0;
        }
    if (dcoef_e)
        for (int64_t e = 0; e < ne; ++e) {
            const double* d = dcoef_e + 4 * e;
            if (!(std::isfinite(d[0]) && d[0] >= 0.0) || !finite_pos(d[1]) || !finite_pos(d[2]) || !finite_pos(d[3]))
                return "dcoef_e entries invalid";
            if (!lambda_e) any_d0 |= d[0] > 0.0;
        }
    if (!any_d0 && mask == 0) return "lambda = 0 everywhere needs at least one Dirichlet face";
    return nullptr;
}


template <typename T>
constexpr int dtype_of() { return sizeof(T) == 8 ? SEMCOND_F64 : SEMCOND_F32; }

// Default persistent configuration: the largest element-group count that k
// divides, and as many workgroups as are co-resident, but no more than needed
// to give every element group one element.
bool persist_default(semcond_ctx* c, int k, int dtype, int* S, int* G) {
    const int NI = c->L.NI;
    int cand[2] = {NI * NI <= 64 ? 4 : (NI * NI <= 128 ? 2 : 1), 1};
    for (int S0 : cand) {
        if (!persist_supported(NI, S0, k)) continue;
        const int mg = dtype == SEMCOND_F64 ? persist_max_grid<double>(NI, S0) : persist_max_grid<float>(NI, S0);
        if (mg <= 0) continue;
        int64_t need = (c->n_e + S0 - 1) / S0;
        *S = S0;
        *G = (int)std::min<int64_t>(mg, need);
        return true;
    }
    return false;
}

template <typename T>
int run_persistent(semcond_ctx* c, T* x, T* r, T* p, T* q, int k, double tol, int max_iter, CgWork& w, int S, int G,
                   hipStream_t st) {
    // a cooperative grid must be co-resident: reject configurations (e.g. from a
    // stale tuning cache) beyond what the device holds at once
    const int mg = persist_max_grid<T>(c->L.NI, S);
    if (!persist_supported(c->L.NI, S, k) || G < 1 || G > mg)
        return fail(c, SEMCOND_EINVAL, "persistent CG: configuration (S, G) not co-resident on this device");
    if (!cg_offsets_fit<T>(c)) return fail(c, SEMCOND_EINVAL, cg_offsets_msg);
    const size_t part_bytes = (3 * (size_t)G * k * sizeof(double) + 255) / 256 * 256;
    const size_t need = part_bytes + kBarWords * sizeof(unsigned);
    int rc = grow(c, c->ws_persist, need);
    if (rc) return rc;
    double* part = (double*)c->ws_persist.ptr;
    unsigned* bar = (unsigned*)((char*)c->ws_persist.ptr + part_bytes);
    // barrier words and error flag start at zero (bit pattern of 0.0f)
    HIPCHK(c, launch_fill<float>((float*)bar, kBarWords, 0.0f, st));
    PcgArgs<T> P;
    P.A = apply_args<T>(c);
    P.A.u = p;
    P.A.v = q;
    P.A.k = k;
    P.A.ns = 1u;  // RHS-major vectors
    P.A.rs = (uint32_t)c->N_s;
    P.A.energy = nullptr;
    P.A.e_begin = 0;
    // the kernel forms the direction at its gather from r, pinv and its own beta
    P.A.dir_r = r;
    P.A.dir_pinv = pinv<T>(c);
    P.A.dir_beta = nullptr;
    P.x = x;
    P.r = r;
    P.p = p;
    P.q = q;
    P.pinv = pinv<T>(c);
    P.Ns = c->N_s;
    P.n_e = c->n_e;
    P.k = k;
    P.part = part;
    P.rho = w.s.rho;
    P.beta = w.s.beta;
    P.rr = w.s.rr;
    P.bb = w.s.bb;
    P.active = w.s.active;
    P.iters = w.s.iters;
    P.status = w.s.status;
    P.rrb = w.s.rrb;
    P.stall = w.s.stall;
    P.window = w.s.window;
    P.tol2 = tol * tol;
    P.max_iter = max_iter;
    P.bar = bar;
    P.err = (int*)(bar + (kBarGroups + 2) * kBarSlot);
    P.spin_limit = 1u << 24;
    std::vector<int> it0;
    if (c->prof) {
        it0.resize(k);
        HIPCHK(c, hipMemcpyAsync(it0.data(), w.s.iters, k * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        rc = profile_begin(c, SEMCOND_KERNEL_PCG, st);
        if (rc) return rc;
    }
    if (!P.A.u || !P.A.v || !P.A.dir_r || !P.A.dir_pinv || !P.x || !P.r || !P.q || !P.pinv || !P.part || !P.beta)
        return fail(c, SEMCOND_EINVAL, "persistent CG: missing operand");
#ifdef SEMCOND_PCG_TRACE
    const size_t ntr = (size_t)kPcgTraceIters * 4 * G;
    HIPCHK(c, hipMalloc(&P.trace, ntr * sizeof(long long)));
    HIPCHK(c, hipMemsetAsync(P.trace, 0, ntr * sizeof(long long), st));
#endif
    HIPCHK(c, launch_pcg_persistent<T>(P, c->L.NI, S, G, st));
#ifdef SEMCOND_PCG_TRACE
    {
        std::vector<long long> tr(ntr);
        HIPCHK(c, hipMemcpyAsync(tr.data(), P.trace, ntr * sizeof(long long), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        HIPCHK(c, hipFree(P.trace));
        if (const char* fn = std::getenv("SEMCOND_PCG_TRACE_FILE")) {
            if (FILE* fp = std::fopen(fn, "a")) {
                std::fprintf(fp, "launch NI %d S %d G %d k %d\n", c->L.NI, S, G, k);
                for (size_t i = 0; i < ntr; ++i) std::fprintf(fp, "%lld%c", tr[i], (i + 1) % G ? ' ' : '\n');
                std::fclose(fp);
            }
        }
    }
#endif
    if (c->prof) {
        rc = profile_end(c, st);
        if (rc) return rc;
    }
    int herr = 0;
    HIPCHK(c, hipMemcpyAsync(&herr, P.err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (herr) return fail(c, SEMCOND_EDEVICE, "persistent CG: grid barrier wait exceeded its bound");
    if (c->prof) {
        std::vector<int> it1(k);
        HIPCHK(c, hipMemcpy(it1.data(), w.s.iters, k * sizeof(int), hipMemcpyDeviceToHost));
        int mx = 0;
        for (int i = 0; i < k; ++i) mx = std::max(mx, it1[i] - it0[i]);
        c->prof_iters += mx;
    }
    return SEMCOND_OK;
}

// CG on the transformed condensed system.  mode SEMCOND_CG_AUTO takes the
// autotuned choice for (k, type) when there is one (S = 0 meaning one launch
// per step), else one launch per step; SEMCOND_CG_PERSISTENT takes the tuned
// or default persistent grid where a persistent kernel exists.
// ---- Two-level preconditioner (vertex coarse space) -----------------------

constexpr int kMaxCoarse = 32768;

int coarse_setup(semcond_ctx* c, hipStream_t st) {
    if (c->coarse_ready) return SEMCOND_OK;
    const Layout& L = c->L;
    const int nv1 = L.n1 + 1, nv2 = L.n2 + 1, nv3 = L.n3 + 1;
    const int64_t nv = (int64_t)nv1 * nv2 * nv3;
    std::vector<int> vmap(nv, -1);
    int n0 = 0;
    for (int vz = 0; vz < nv3; ++vz)
        for (int vy = 0; vy < nv2; ++vy)
            for (int vx = 0; vx < nv1; ++vx)
                if (!xcon(L, vx) && !ycon(L, vy) && !zcon(L, vz)) vmap[vx + (int64_t)nv1 * (vy + (int64_t)nv2 * vz)] = n0++;
    if (n0 > kMaxCoarse)
        return fail(c, SEMCOND_EINVAL, "coarse space of " + std::to_string(n0) + " free vertices (limit " +
                                           std::to_string(kMaxCoarse) + ")");
    // element metrics as the kernels use them
    std::vector<double> hd;
    {
        int rc = element_metrics_host(c, st, hd);
        if (rc) return rc;
    }
    // trilinear element matrices d0 m(x)m(x)m + d1 m(x)m(x)k + d2 m(x)k(x)m +
    // d3 k(x)m(x)m with the 1D linear-element matrices on [-1, 1] (exact, the
    // GLL rule integrates these quadratics exactly for p >= 2), assembled over
    // the free vertices
    const double k1[2][2] = {{0.5, -0.5}, {-0.5, 0.5}};
    const double m1[2][2] = {{2.0 / 3.0, 1.0 / 3.0}, {1.0 / 3.0, 2.0 / 3.0}};
    std::vector<double> A((size_t)n0 * n0, 0.0);
    for (int64_t e = 0; e < c->n_e; ++e) {
        const int e1 = (int)(e % L.n1), e2 = (int)((e / L.n1) % L.n2), e3 = (int)(e / ((int64_t)L.n1 * L.n2));
        const double* d = hd.data() + 4 * e;
        int idx[8];
        for (int q = 0; q < 8; ++q)
            idx[q] = vmap[(e1 + (q & 1)) + (int64_t)nv1 * ((e2 + ((q >> 1) & 1)) + (int64_t)nv2 * (e3 + (q >> 2)))];
        for (int a = 0; a < 8; ++a) {
            if (idx[a] < 0) continue;
            const int ai = a & 1, aj = (a >> 1) & 1, ak = a >> 2;
            for (int b = 0; b < 8; ++b) {
                if (idx[b] < 0) continue;
                const int bi = b & 1, bj = (b >> 1) & 1, bk = b >> 2;
                const double v = d[0] * m1[ak][bk] * m1[aj][bj] * m1[ai][bi] + d[1] * m1[ak][bk] * m1[aj][bj] * k1[ai][bi] +
                                 d[2] * m1[ak][bk] * k1[aj][bj] * m1[ai][bi] + d[3] * k1[ak][bk] * m1[aj][bj] * m1[ai][bi];
                A[(size_t)idx[b] * n0 + idx[a]] += v;
            }
        }
    }
    // transformed hats t_a = S^-1 l_a, l_0 = (1 - x)/2, l_1 = (1 + x)/2 at the interior nodes
    const int NI = L.NI;
    std::vector<double> tw(2 * (size_t)NI, 0.0);
    for (int o = 0; o < NI; ++o)
        for (int m = 0; m < NI; ++m) {
            const double xm = c->t.x[m + 1];
            tw[o] += c->t.Sinv[(size_t)o * NI + m] * 0.5 * (1.0 - xm);
            tw[NI + o] += c->t.Sinv[(size_t)o * NI + m] * 0.5 * (1.0 + xm);
        }
    hipFree(c->c_L);
    hipFree(c->c_vmap);
    hipFree(c->c_tw);
    c->c_L = nullptr;
    c->c_vmap = nullptr;
    c->c_tw = nullptr;
    HIPCHK(c, hipMalloc(&c->c_vmap, vmap.size() * sizeof(int)));
    HIPCHK(c, hipMemcpy(c->c_vmap, vmap.data(), vmap.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMalloc(&c->c_tw, tw.size() * sizeof(double)));
    HIPCHK(c, hipMemcpy(c->c_tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice));
    if (n0 > 0) {
        HIPCHK(c, hipMalloc(&c->c_L, A.size() * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->c_L, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice));
        if (!c->blas && rocblas_create_handle(&c->blas) != rocblas_status_success) {
            c->blas = nullptr;
            return fail(c, SEMCOND_EDEVICE, "rocblas_create_handle failed");
        }
        if (rocblas_set_stream(c->blas, st) != rocblas_status_success)
            return fail(c, SEMCOND_EDEVICE, "rocblas_set_stream failed");
        int* dinfo = nullptr;
        HIPCHK(c, hipMalloc(&dinfo, sizeof(int)));
        const rocblas_status rs = rocsolver_dpotrf(c->blas, rocblas_fill_lower, n0, c->c_L, n0, dinfo);
        int info = -1;
        hipError_t he = rs == rocblas_status_success ? hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, st)
                                                     : hipErrorUnknown;
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        hipFree(dinfo);
        if (rs != rocblas_status_success || he != hipSuccess)
            return fail(c, SEMCOND_EDEVICE, "coarse Cholesky factorisation failed to run");
        if (info != 0) return fail(c, SEMCOND_EINVAL, "coarse matrix not positive definite");
        // the explicit inverse from the factor, made symmetric: each coarse
        // solve streams it once (the two triangular solves with few right-hand
        // sides measured 8 ms per CG iteration at 12167 unknowns)
        HIPCHK(c, hipMalloc(&dinfo, sizeof(int)));
        const rocblas_status ri = rocsolver_dpotri(c->blas, rocblas_fill_lower, n0, c->c_L, n0, dinfo);
        he = ri == rocblas_status_success ? hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, st)
                                          : hipErrorUnknown;
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        hipFree(dinfo);
        if (ri != rocblas_status_success || he != hipSuccess || info != 0)
            return fail(c, SEMCOND_EDEVICE, "coarse matrix inversion failed");
        HIPCHK(c, launch_symmetrize_lower(c->c_L, n0, st));
    }
    c->n0 = n0;
    c->coarse_ready = true;
    return SEMCOND_OK;
}

// The coarse part of the preconditioner for the RHS-major residual r: r0 =
// P^T r, z0 = A_0^-1 r0, rz_extra = r0 . z0.
template <typename T>
int coarse_solve(semcond_ctx* c, const T* r, int k, const int* act, double* r0, double* z0, double* rz_extra,
                 hipStream_t st) {
    const int n0 = c->n0;
    if (n0 == 0) {
        HIPCHK(c, launch_fill<double>(rz_extra, k, 0.0, st));
        return SEMCOND_OK;
    }
    HIPCHK(c, launch_fill<double>(r0, (int64_t)n0 * k, 0.0, st));
    HIPCHK(c, launch_coarse_restrict<T>(c->L, c->c_tw, c->c_vmap, n0, r, k, act, r0, st));
    HIPCHK(c, launch_fill<double>(z0, (int64_t)n0 * k, 0.0, st));
    HIPCHK(c, launch_coarse_gemv(c->c_L, n0, r0, k, z0, st));
    HIPCHK(c, launch_coarse_dot(r0, z0, n0, k, rz_extra, st));
    return SEMCOND_OK;
}

// Preconditioned CG with the two-level preconditioner P^-1 + P A_0^-1 P^T:
// the direction p = z + beta p is formed before each operator application
// (plain apply), the step updates x and r from it.  Otherwise as run_cg's
// loop with separate reductions (slots, stopped RHS skipped, polls every
// check_every iterations).
template <typename T>
int run_cg_coarse(semcond_ctx* c, const T* b, T* x, T* r, T* p, T* q, int k, double tol, int max_iter,
                  int check_every, bool x0_given, CgWork& w, hipStream_t st, bool keep_dir) {
    const int64_t Ns = c->N_s;
    int rc = coarse_setup(c, st);
    if (rc) return rc;
    rc = grow(c, c->ws_coarse, (2 * (size_t)c->n0 * k + k) * sizeof(double));
    if (rc) return rc;
    double* r0 = (double*)c->ws_coarse.ptr;
    double* z0 = r0 + (size_t)c->n0 * k;
    double* rz_extra = z0 + (size_t)c->n0 * k;
    const double tol2 = tol * tol;
    HIPCHK(c, hipMemcpyAsync(w.s.tol2, &tol2, sizeof(double), hipMemcpyHostToDevice, st));
    if (x0_given) {
        rc = apply_transformed<T>(c, x, q, k, RHS_MAJOR, nullptr, st);
        if (rc) return rc;
        HIPCHK(c, launch_cg_init<T>(b, q, pinv<T>(c), r, p, Ns, k, w.partials, st, keep_dir));
    } else {
        HIPCHK(c, launch_fill<T>(x, Ns * k, (T)0, st));
        HIPCHK(c, launch_fill<T>(q, Ns * k, (T)0, st));
        HIPCHK(c, launch_cg_init<T>(b, (T*)nullptr, pinv<T>(c), r, p, Ns, k, w.partials, st, keep_dir));
    }
    rc = coarse_solve<T>(c, r, k, nullptr, r0, z0, rz_extra, st);
    if (rc) return rc;
    CgState s = w.s;
    s.rz_extra = rz_extra;
    HIPCHK(c, launch_cg_reduce(w.partials, vec_blocks(k), 3, k, s, keep_dir ? RED_INIT_KEEP : RED_INIT, st));
    HIPCHK(c, launch_coarse_pupd<T>(c->L, c->c_tw, c->c_vmap, c->n0, z0, pinv<T>(c), r, p, k, s, st));
    if (check_every < 1) check_every = 1;
    T* Q = nullptr;
    const int64_t qlen = slot_len(c->L);
    const bool slots = c->det_active || (c->L.NI >= 3 && (sizeof(T) == 4 || c->L.NI <= 8));
    if (c->det_active && qlen * (int64_t)k >= (int64_t(1) << 31))
        return fail(c, SEMCOND_EINVAL, "deterministic solve: slot workspace beyond 2^31 entries");
    if (slots && qlen * (int64_t)k < (int64_t(1) << 31)) {
        rc = grow(c, c->ws_slots, (size_t)qlen * k * sizeof(T));
        if (rc) return rc;
        Q = (T*)c->ws_slots.ptr;
        HIPCHK(c, launch_fill<T>(Q, qlen * k, (T)0, st));
    }
    auto none_active = [&](const int* h) {
        for (int i = 0; i < k; ++i)
            if (h[i]) return false;
        return true;
    };
    for (int it = 0; it < max_iter; ++it) {
        if (it % check_every == 0) {
            HIPCHK(c, hipMemcpyAsync(c->h_active, w.s.active, k * sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (none_active(c->h_active)) break;
        }
        rc = apply_transformed<T>(c, p, q, k, RHS_MAJOR, w.energy, st, true, nullptr, nullptr, 0, nullptr, w.s.active,
                                  Q);
        if (rc) return rc;
        HIPCHK(c, launch_energy_pq(w.energy, c->n_e, k, w.epart, w.s, st));
        HIPCHK(c, launch_cg_step<T>(x, r, p, q, pinv<T>(c), Ns, k, w.s, w.partials, Q, qlen, c->L, cg_face_slots<T>(),
                                    st, true));
        rc = coarse_solve<T>(c, r, k, w.s.active, r0, z0, rz_extra, st);
        if (rc) return rc;
        HIPCHK(c, launch_cg_reduce(w.partials, vec_blocks(k), 2, k, s, RED_RZ, st));
        HIPCHK(c, launch_coarse_pupd<T>(c->L, c->c_tw, c->c_vmap, c->n0, z0, pinv<T>(c), r, p, k, s, st));
    }
    return SEMCOND_OK;
}

template <typename T>
int run_cg_any(semcond_ctx* c, const T* b, T* x, T* r, T* p, T* q, int k, double tol, int max_iter, int check_every,
               bool x0_given, int mode, CgWork& w, hipStream_t st, bool keep_dir = false) {
    if (c->coarse_active)
        return run_cg_coarse<T>(c, b, x, r, p, q, k, tol, max_iter, check_every, x0_given, w, st, keep_dir);
    int S = 0, G = 0;
    bool use = false;
    // (the persistent kernel scatters with atomics: never in deterministic mode)
    if (mode != SEMCOND_CG_STEPWISE && !c->det_active && persist_supported(c->L.NI, 1, k)) {
        auto it = c->tuned.find({k, dtype_of<T>()});
        if (it != c->tuned.end() && it->second.first > 0) {
            S = it->second.first;
            G = it->second.second;
            use = true;
        } else if (mode == SEMCOND_CG_PERSISTENT) {
            use = persist_default(c, k, dtype_of<T>(), &S, &G);
        }
    }
    if (!use) return run_cg<T>(c, b, x, r, p, q, k, tol, max_iter, check_every, x0_given, w, st, keep_dir);
    int rc = cg_start<T>(c, b, x, r, p, q, k, tol, x0_given, keep_dir, w, st);
    if (rc) return rc;
    return run_persistent<T>(c, x, r, p, q, k, tol, max_iter, w, S, G, st);
}

// Time the candidate persistent configurations, and one launch per step, for
// `iters` CG iterations on the condensed RHS b (tolerance 0, so every RHS
// stays active).  (S, G) = (0, 0) when one launch per step is fastest.
template <typename T>
int autotune_persistent(semcond_ctx* c, const T* b, T* x, T* r, T* p, T* q, int k, CgWork& w, hipStream_t st,
                        int* bestS, int* bestG) {
    const int NI = c->L.NI;
    const int smax = NI * NI <= 64 ? 4 : (NI * NI <= 128 ? 2 : 1);
    std::vector<std::pair<int, int>> cands = {{0, 0}};
    for (int S : {smax, 1}) {
        if (!persist_supported(NI, S, k)) continue;
        const int mg = persist_max_grid<T>(NI, S);
        const int64_t need = (c->n_e + S - 1) / S;
        for (int div : {1, 2, 4, 8}) {
            int G = (int)std::min<int64_t>(mg / div, need);
            if (G < 1) continue;
            bool dup = false;
            for (auto& cc : cands) dup |= cc.first == S && cc.second == G;
            if (!dup) cands.push_back({S, G});
        }
        if (S == 1 && smax == 1) break;
    }
    const int iters = 12;
    double best = 1e300;
    for (auto& cc : cands) {
        double t_best = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            HIPCHK(c, launch_fill<T>(x, c->N_s * k, (T)0, st));
            HIPCHK(c, launch_fill<T>(q, c->N_s * k, (T)0, st));
            HIPCHK(c, launch_cg_init<T>(b, (T*)nullptr, pinv<T>(c), r, p, c->N_s, k, w.partials, st));
            HIPCHK(c, launch_cg_reduce(w.partials, vec_blocks(k), 3, k, w.s, RED_INIT, st));
            HIPCHK(c, hipStreamSynchronize(st));
            auto t0 = std::chrono::steady_clock::now();
            int rc;
            if (cc.first == 0) {
                rc = run_cg<T>(c, b, x, r, p, q, k, 0.0, iters, iters + 1, false, w, st);
                if (!rc) HIPCHK(c, hipStreamSynchronize(st));
            } else {
                rc = run_persistent<T>(c, x, r, p, q, k, 0.0, iters, w, cc.first, cc.second, st);
            }
            if (rc) return rc;
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            t_best = std::min(t_best, dt);
        }
        if (t_best < best) {
            best = t_best;
            *bestS = cc.first;
            *bestG = cc.second;
        }
    }
    return SEMCOND_OK;
}

// The library's apply on [N_s][k] arrays: the element kernels run on
// RHS-major copies when k > 1 (per-RHS gathers and scatters stay coalesced);
// the physical basis adds S^-1 before and S^-T after (Sec. 6).  Temporaries:
// ws_vec, 2 N_s k values.
template <typename T>
int apply_public(semcond_ctx* c, const T* u, T* v, int k, int basis, T* ws, hipStream_t st) {
    // ws: 2 N_s k values
    const int64_t Ns = c->N_s;
    T* t1 = ws;
    T* t2 = t1 + Ns * k;
    const DevTab<T>& tb = tabs<T>(c);
    const T* in = u;
    if (basis == SEMCOND_PHYSICAL) {
        HIPCHK(c, launch_transform<T>(c->L, tb.Sinv, u, t1, k, st));
        in = t1;
    }
    if (k == 1) {
        int rc = apply_transformed<T>(c, in, t2, k, NODE_MAJOR, nullptr, st);
        if (rc) return rc;
    } else {
        T* tin = in == t1 ? t2 : t1;
        HIPCHK(c, launch_transpose<T>(in, tin, Ns, k, st));
        T* tout = tin == t1 ? t2 : t1;
        int rc = apply_transformed<T>(c, tin, tout, k, RHS_MAJOR, nullptr, st);
        if (rc) return rc;
        if (basis == SEMCOND_TRANSFORMED) {
            HIPCHK(c, launch_transpose<T>(tout, v, k, Ns, st));
            return SEMCOND_OK;
        }
        HIPCHK(c, launch_transpose<T>(tout, tin, k, Ns, st));
        HIPCHK(c, launch_transform<T>(c->L, tb.SinvT, tin, v, k, st));
        return SEMCOND_OK;
    }
    HIPCHK(c, launch_transform<T>(c->L, tb.SinvT, t2, v, k, st));
    return SEMCOND_OK;
}

int create_context(const semcond_mesh* m, void* stream, semcond_ctx** out, bool needs_definite);

}  // namespace

extern "C" {

const char* semcond_version(void) { return "semcond 0.1 (gfx950)"; }

const char* semcond_last_error(const semcond_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

int semcond_host_tables(int p, double* x, double* w, double* K, double* Sm, double* lam) {
    Tables1D t;
    if (!build_tables(p, &t)) return fail(nullptr, SEMCOND_EINVAL, "p must be in [2, 32]");
    if (x) std::memcpy(x, t.x.data(), t.x.size() * sizeof(double));
    if (w) std::memcpy(w, t.w.data(), t.w.size() * sizeof(double));
    if (K) std::memcpy(K, t.K.data(), t.K.size() * sizeof(double));
    if (Sm) std::memcpy(Sm, t.S.data(), t.S.size() * sizeof(double));
    if (lam) std::memcpy(lam, t.lam.data(), t.lam.size() * sizeof(double));
    return SEMCOND_OK;
}

int semcond_destroy(semcond_ctx* c) {
    if (!c) return SEMCOND_OK;
    hipDeviceSynchronize();
    hipFree(c->t64.buf);
    hipFree(c->t32.buf);
    hipFree(c->d_widths);
    hipFree(c->d_ax);
    hipFree(c->d_lam_e);
    hipFree(c->d_dcoef);
    hipFree(c->d_diag);
    hipFree(c->d_pinv64);
    hipFree(c->d_pinv32);
    hipFree(c->ws_vec.ptr);
    hipFree(c->ws_scratch.ptr);
    hipFree(c->ws_state.ptr);
    hipFree(c->ws_nodal.ptr);
    hipFree(c->ws_persist.ptr);
    hipFree(c->ws_lift.ptr);
    hipFree(c->ws_slots.ptr);
    if (c->h_active) hipHostFree(c->h_active);
    if (c->h_flags) hipHostFree(c->h_flags);
    for (hipEvent_t e : c->poll_ev)
        if (e) hipEventDestroy(e);
    for (hipEvent_t e : c->ev) hipEventDestroy(e);
    hipFree(c->mmc_H);
    hipFree(c->mmc_col);
    hipFree(c->ws_mmc.ptr);
    hipFree(c->c_L);
    hipFree(c->c_vmap);
    hipFree(c->c_tw);
    hipFree(c->ws_coarse.ptr);
    hipFree(c->d_dinv32);
    hipFree(c->d_dcls);
    hipFree(c->d_dclass);
    if (c->blas) rocblas_destroy_handle(c->blas);
    delete c;
    return SEMCOND_OK;
}

int semcond_profile_enable(semcond_ctx* c, int enable) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    int rc = profile_flush(c);
    if (rc) return rc;
    c->prof = enable != 0;
    c->prof_ms[0] = c->prof_ms[1] = c->prof_ms[2] = 0.0;
    c->prof_launches[0] = c->prof_launches[1] = c->prof_launches[2] = 0;
    c->prof_iters = 0;
    return SEMCOND_OK;
}

int semcond_profile_read(semcond_ctx* c, int kernel, double* ms, int64_t* launches, int64_t* iters) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (kernel != SEMCOND_KERNEL_APPLY && kernel != SEMCOND_KERNEL_PCG && kernel != SEMCOND_KERNEL_APPLY_F32)
        return fail(c, SEMCOND_EINVAL, "bad kernel id");
    int rc = profile_flush(c);
    if (rc) return rc;
    if (ms) *ms = c->prof_ms[kernel];
    if (launches) *launches = c->prof_launches[kernel];
    if (iters) *iters = kernel == SEMCOND_KERNEL_PCG ? c->prof_iters : 0;
    return SEMCOND_OK;
}

int semcond_create(const semcond_mesh* m, void* stream, semcond_ctx** out) {
    return create_context(m, stream, out, true);
}

}  // extern "C"

namespace {

// semcond_create; without the check that a problem with lambda = 0
// everywhere has a Dirichlet face (one-element contexts whose operator is
// only applied, never solved: the MMC class matrices)
int create_context(const semcond_mesh* m, void* stream, semcond_ctx** out, bool needs_definite) {
    if (!out) return fail(nullptr, SEMCOND_EINVAL, "out is NULL");
    *out = nullptr;
    if (!m) return fail(nullptr, SEMCOND_EINVAL, "mesh is NULL");
    if (m->p < 2 || m->p > kMaxP) return fail(nullptr, SEMCOND_EINVAL, "p must be in [2, 32]");
    int64_t ne = 1;
    for (int a = 0; a < 3; ++a) {
        if (m->n[a] < 1) return fail(nullptr, SEMCOND_EINVAL, "n[a] must be >= 1");
        if (!m->widths[a]) return fail(nullptr, SEMCOND_EINVAL, "widths[a] is NULL");
        for (int i = 0; i < m->n[a]; ++i)
            if (!finite_pos(m->widths[a][i])) return fail(nullptr, SEMCOND_EINVAL, "widths must be positive and finite");
        ne *= m->n[a];
    }
    if (ne > (int64_t(1) << 26)) return fail(nullptr, SEMCOND_EINVAL, "too many elements (max 2^26)");
    if (m->dirichlet_mask > 63u) return fail(nullptr, SEMCOND_EINVAL, "dirichlet_mask has bits above 5");
    if (const char* msg = check_coefficients(ne, needs_definite ? m->dirichlet_mask : 1u, m->lambda, m->lambda_e,
                                             m->dcoef_e))
        return fail(nullptr, SEMCOND_EINVAL, msg);

    semcond_ctx* c = new (std::nothrow) semcond_ctx();
    if (!c) return fail(nullptr, SEMCOND_ENOMEM, "host allocation failed");
    c->p = m->p;
    for (int a = 0; a < 3; ++a) c->n[a] = m->n[a];
    c->n_e = ne;
    if (!build_tables(m->p, &c->t)) {
        delete c;
        return fail(nullptr, SEMCOND_EINVAL, "table construction failed");
    }
    c->L = make_layout(m->p, m->n, m->dirichlet_mask);
    c->N_s = c->L.Ns;
    c->N = (int64_t)(m->n[0] * (int64_t)m->p + 1) * (m->n[1] * (int64_t)m->p + 1) * (m->n[2] * (int64_t)m->p + 1);
    int64_t nfree = 0;
    for (int64_t s = 0; s < c->N_s; ++s) {
        int I1, I2, I3;
        bool con;
        skeleton_node(c->L, s, &I1, &I2, &I3, &con);
        nfree += con ? 0 : 1;
    }
    c->N_free = nfree;
    hipStream_t st = S(stream);
    auto bail = [&](int rc) {
        std::string msg = c->err;
        semcond_destroy(c);
        g_last_error = msg;
        return rc;
    };
    int rc = upload_tables<double>(c, c->t64);
    if (!rc) rc = upload_tables<float>(c, c->t32);
    if (rc) return bail(rc);
    const int nw = m->n[0] + m->n[1] + m->n[2];
    std::vector<double> hw;
    for (int a = 0; a < 3; ++a) hw.insert(hw.end(), m->widths[a], m->widths[a] + m->n[a]);
#define CHK(call)                                                                          \
    do {                                                                                   \
        hipError_t e__ = (call);                                                           \
        if (e__ != hipSuccess) {                                                           \
            fail(c, SEMCOND_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e__));  \
            return bail(SEMCOND_EDEVICE);                                                  \
        }                                                                                  \
    } while (0)
    {
        // the fixed workspace of semcond_apply_noalloc on this device
        int dev = 0;
        CHK(hipGetDevice(&dev));
        CHK(noalloc_scratch_init());
        c->noalloc_ws = noalloc_scratch(dev);
        if (!c->noalloc_ws) {
            fail(c, SEMCOND_EDEVICE, "fixed apply workspace: no device address");
            return bail(SEMCOND_EDEVICE);
        }
    }
    CHK(hipMalloc(&c->d_widths, nw * sizeof(double)));
    CHK(hipMemcpy(c->d_widths, hw.data(), nw * sizeof(double), hipMemcpyHostToDevice));
    c->geo.L = c->L;
    c->geo.hx = c->d_widths;
    c->geo.hy = c->d_widths + m->n[0];
    c->geo.hz = c->d_widths + m->n[0] + m->n[1];
    {
        // per axis and element: h/2 and 4/h^2
        std::vector<double> ax(2 * (size_t)nw);
        for (int i = 0; i < nw; ++i) {
            ax[2 * i] = 0.5 * hw[i];
            ax[2 * i + 1] = 4.0 / (hw[i] * hw[i]);
        }
        CHK(hipMalloc(&c->d_ax, ax.size() * sizeof(double)));
        CHK(hipMemcpy(c->d_ax, ax.data(), ax.size() * sizeof(double), hipMemcpyHostToDevice));
        c->geo.ax = c->d_ax;
    }
    CHK(hipMalloc(&c->d_diag, c->N_s * sizeof(double)));
    CHK(hipMalloc(&c->d_pinv64, c->N_s * sizeof(double)));
    CHK(hipMalloc(&c->d_pinv32, c->N_s * sizeof(float)));
    rc = set_coefficients(c, m->lambda, m->lambda_e, m->dcoef_e, st);
    if (rc) return bail(rc);
    CHK(hipStreamSynchronize(st));
#undef CHK
    *out = c;
    return SEMCOND_OK;
}

}  // namespace

extern "C" {

int semcond_sizes(const semcond_ctx* c, int64_t* N, int64_t* N_s, int64_t* N_free, int64_t* n_e) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (N) *N = c->N;
    if (N_s) *N_s = c->N_s;
    if (N_free) *N_free = c->N_free;
    if (n_e) *n_e = c->n_e;
    return SEMCOND_OK;
}

int semcond_skeleton_coords(const semcond_ctx* c, int32_t* ijk, uint8_t* free_mask) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    for (int64_t s = 0; s < c->N_s; ++s) {
        int I1, I2, I3;
        bool con;
        skeleton_node(c->L, s, &I1, &I2, &I3, &con);
        if (ijk) {
            ijk[3 * s] = I1;
            ijk[3 * s + 1] = I2;
            ijk[3 * s + 2] = I3;
        }
        if (free_mask) free_mask[s] = con ? 0 : 1;
    }
    return SEMCOND_OK;
}

int semcond_apply(semcond_ctx* c, const void* u, void* v, int k, int dtype, int basis, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!u || !v) return fail(c, SEMCOND_EINVAL, "u and v must be device pointers");
    if (u == v) return fail(c, SEMCOND_EINVAL, "u and v must not overlap");
    int rc = check_dtype(c, dtype);
    if (!rc) rc = check_k(c, k);
    if (rc) return rc;
    if (basis != SEMCOND_PHYSICAL && basis != SEMCOND_TRANSFORMED) return fail(c, SEMCOND_EINVAL, "bad basis");
    hipStream_t st = S(stream);
    DetScope det(c, c->det);
    const size_t es = dtype == SEMCOND_F64 ? sizeof(double) : sizeof(float);
    if (basis == SEMCOND_TRANSFORMED && k == 1) {
        if (dtype == SEMCOND_F64) return apply_transformed<double>(c, (const double*)u, (double*)v, k, NODE_MAJOR, nullptr, st);
        return apply_transformed<float>(c, (const float*)u, (float*)v, k, NODE_MAJOR, nullptr, st);
    }
    rc = grow(c, c->ws_vec, 2 * es * (size_t)c->N_s * k);
    if (rc) return rc;
    if (dtype == SEMCOND_F64) return apply_public<double>(c, (const double*)u, (double*)v, k, basis, (double*)c->ws_vec.ptr, st);
    return apply_public<float>(c, (const float*)u, (float*)v, k, basis, (float*)c->ws_vec.ptr, st);
}

int semcond_apply_noalloc(semcond_ctx* c, const void* u, void* v, int k, int dtype, int basis, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!u || !v) return fail(c, SEMCOND_EINVAL, "u and v must be device pointers");
    if (u == v) return fail(c, SEMCOND_EINVAL, "u and v must not overlap");
    int rc = check_dtype(c, dtype);
    if (!rc) rc = check_k(c, k);
    if (rc) return rc;
    if (basis != SEMCOND_PHYSICAL && basis != SEMCOND_TRANSFORMED) return fail(c, SEMCOND_EINVAL, "bad basis");
    if (c->det) return fail(c, SEMCOND_EINVAL, "semcond_apply_noalloc: deterministic mode needs the slot workspace");
    if (!c->noalloc_ws) return fail(c, SEMCOND_EDEVICE, "semcond_apply_noalloc: fixed workspace not set up");
    const size_t es = dtype == SEMCOND_F64 ? sizeof(double) : sizeof(float);
    if (2 * es * (size_t)c->N_s * (size_t)k > kNoAllocScratchBytes)
        return fail(c, SEMCOND_EINVAL, "semcond_apply_noalloc: 2 N_s k values exceed the fixed workspace (32 MiB)");
    hipStream_t st = S(stream);
    DetScope det(c, false);
    // no profiling events either (their creation may allocate)
    const bool prof = c->prof;
    c->prof = false;
    if (basis == SEMCOND_TRANSFORMED && k == 1) {
        rc = dtype == SEMCOND_F64
                 ? apply_transformed<double>(c, (const double*)u, (double*)v, k, NODE_MAJOR, nullptr, st)
                 : apply_transformed<float>(c, (const float*)u, (float*)v, k, NODE_MAJOR, nullptr, st);
    } else if (dtype == SEMCOND_F64) {
        rc = apply_public<double>(c, (const double*)u, (double*)v, k, basis, (double*)c->noalloc_ws, st);
    } else {
        rc = apply_public<float>(c, (const float*)u, (float*)v, k, basis, (float*)c->noalloc_ws, st);
    }
    c->prof = prof;
    return rc;
}

int semcond_transform(semcond_ctx* c, const void* in, void* out, int k, int dtype, int direction, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!in || !out || in == out) return fail(c, SEMCOND_EINVAL, "in/out must be distinct device pointers");
    int rc = check_dtype(c, dtype);
    if (!rc) rc = check_k(c, k);
    if (rc) return rc;
    if (direction < 0 || direction > 3) return fail(c, SEMCOND_EINVAL, "bad direction");
    hipStream_t st = S(stream);
    if (dtype == SEMCOND_F64)
        HIPCHK(c, launch_transform<double>(c->L, transform_matrix<double>(c, direction), (const double*)in,
                                           (double*)out, k, st));
    else
        HIPCHK(c, launch_transform<float>(c->L, transform_matrix<float>(c, direction), (const float*)in,
                                          (float*)out, k, st));
    return SEMCOND_OK;
}

int semcond_precond_diag(semcond_ctx* c, void* diag, int dtype, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!diag) return fail(c, SEMCOND_EINVAL, "diag is NULL");
    int rc = check_dtype(c, dtype);
    if (rc) return rc;
    hipStream_t st = S(stream);
    if (dtype == SEMCOND_F64)
        HIPCHK(c, hipMemcpyAsync(diag, c->d_diag, c->N_s * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
        HIPCHK(c, (launch_convert<double, float>(c->d_diag, (float*)diag, c->N_s, st)));
    return SEMCOND_OK;
}

int semcond_condense_rhs(semcond_ctx* c, const void* f, void* fhat, int k, int dtype, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!f || !fhat) return fail(c, SEMCOND_EINVAL, "f and fhat must be device pointers");
    int rc = check_dtype(c, dtype);
    if (!rc) rc = check_k(c, k);
    if (rc) return rc;
    hipStream_t st = S(stream);
    DetScope det(c, c->det);
    if (dtype == SEMCOND_F64) return condense_rhs64(c, (const double*)f, (double*)fhat, k, st);
    rc = grow(c, c->ws_vec, sizeof(double) * (size_t)c->N_s * k);
    if (rc) return rc;
    double* t = (double*)c->ws_vec.ptr;
    rc = condense_rhs64(c, (const double*)f, t, k, st);
    if (rc) return rc;
    HIPCHK(c, (launch_convert<double, float>(t, (float*)fhat, c->N_s * k, st)));
    return SEMCOND_OK;
}

int semcond_skeleton_to_nodal(semcond_ctx* c, const void* skel, void* nodal, int k, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!skel || !nodal) return fail(c, SEMCOND_EINVAL, "NULL pointer");
    int rc = check_k(c, k);
    if (rc) return rc;
    HIPCHK(c, launch_skel_to_nodal(c->L, (const double*)skel, (double*)nodal, c->N, k, 0, S(stream)));
    return SEMCOND_OK;
}

int semcond_nodal_to_skeleton(semcond_ctx* c, const void* nodal, void* skel, int k, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!skel || !nodal) return fail(c, SEMCOND_EINVAL, "NULL pointer");
    int rc = check_k(c, k);
    if (rc) return rc;
    HIPCHK(c, launch_nodal_to_skel(c->L, (const double*)nodal, (double*)skel, c->N, k, S(stream)));
    return SEMCOND_OK;
}

int semcond_update_coefficients(semcond_ctx* c, double lambda, const double* lambda_e, const double* dcoef_e,
                                void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (const char* msg = check_coefficients(c->n_e, c->L.mask, lambda, lambda_e, dcoef_e))
        return fail(c, SEMCOND_EINVAL, msg);
    hipStream_t st = S(stream);
    int rc = set_coefficients(c, lambda, lambda_e, dcoef_e, st);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(st));
    return SEMCOND_OK;
}

int semcond_nodal_mass(semcond_ctx* c, void* mass, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!mass) return fail(c, SEMCOND_EINVAL, "mass is NULL");
    HIPCHK(c, launch_nodal_mass(c->geo, c->t64.tab.w, (double*)mass, c->N, S(stream)));
    return SEMCOND_OK;
}

int semcond_set_rhs_batch(semcond_ctx* c, int R) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (R < -1 || R > kMaxRhs) return fail(c, SEMCOND_EINVAL, "R must be in [-1, 256]");
    c->rhs_batch_fixed = R;
    return SEMCOND_OK;
}

int semcond_get_rhs_batch(const semcond_ctx* c, int k, int* R_condense, int* R_recover) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (k < 1 || k > kMaxRhs) return fail(const_cast<semcond_ctx*>(c), SEMCOND_EINVAL, "k must be in [1, 256]");
    if (R_condense) *R_condense = rhs_batch(c, k, 0);
    if (R_recover) *R_recover = rhs_batch(c, k, 1);
    return SEMCOND_OK;
}

int semcond_autotune(semcond_ctx* c, int k, int dtype, const char* cache_path, int* S_out, int* G_out) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    int rc = check_k(c, k);
    if (!rc) rc = check_dtype(c, dtype);
    if (rc) return rc;
    if (!persist_supported(c->L.NI, 1, k)) return fail(c, SEMCOND_EINVAL, "no persistent kernel for this degree and k");
    char key[160];
    std::snprintf(key, sizeof key, "%d %d %d %d %d %d", c->p, c->n[0], c->n[1], c->n[2], k, dtype);
    int S = 0, G = 0;
    bool found = false;
    if (cache_path) {
        if (FILE* fh = std::fopen(cache_path, "r")) {
            char line[256];
            while (std::fgets(line, sizeof line, fh)) {
                int a[6], s0, g0;
                if (std::sscanf(line, "%d %d %d %d %d %d %d %d", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5], &s0, &g0) == 8) {
                    char k2[160];
                    std::snprintf(k2, sizeof k2, "%d %d %d %d %d %d", a[0], a[1], a[2], a[3], a[4], a[5]);
                    if (std::strcmp(k2, key) == 0 &&
                        ((s0 == 0 && g0 == 0) || (persist_supported(c->L.NI, s0, k) && g0 > 0))) {
                        S = s0;
                        G = g0;
                        found = true;
                    }
                }
            }
            std::fclose(fh);
        }
    }
    hipStream_t st = nullptr;
    if (!found) {
        // tune on a synthetic right-hand side in the workspace: b = 1 on every slot
        const size_t nv = (size_t)c->N_s * k;
        const size_t es = dtype == SEMCOND_F64 ? sizeof(double) : sizeof(float);
        rc = grow(c, c->ws_vec, 5 * nv * es);
        if (rc) return rc;
        CgWork w;
        rc = cg_state(c, k, 0, &w);
        if (rc) return rc;
        if (dtype == SEMCOND_F64) {
            double* b = (double*)c->ws_vec.ptr;
            HIPCHK(c, launch_fill<double>(b, nv, 1.0, st));
            rc = autotune_persistent<double>(c, b, b + nv, b + 2 * nv, b + 3 * nv, b + 4 * nv, k, w, st, &S, &G);
        } else {
            float* b = (float*)c->ws_vec.ptr;
            HIPCHK(c, launch_fill<float>(b, nv, 1.0f, st));
            rc = autotune_persistent<float>(c, b, b + nv, b + 2 * nv, b + 3 * nv, b + 4 * nv, k, w, st, &S, &G);
        }
        if (rc) return rc;
        if (cache_path) {
            if (FILE* fh = std::fopen(cache_path, "a")) {
                std::fprintf(fh, "%s %d %d\n", key, S, G);
                std::fclose(fh);
            }
        }
    }
    c->tuned[{k, dtype}] = {S, G};
    if (S_out) *S_out = S;
    if (G_out) *G_out = G;
    return SEMCOND_OK;
}

int semcond_mass_apply(semcond_ctx* c, const void* in, void* out, int k, int inverse, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!in || !out) return fail(c, SEMCOND_EINVAL, "NULL pointer");
    if (k < 1 || k > 256) return fail(c, SEMCOND_EINVAL, "k must be in [1, 256]");
    HIPCHK(c, launch_mass_apply(c->geo, c->t64.tab.w, (const double*)in, (double*)out, c->N, k, inverse, S(stream)));
    return SEMCOND_OK;
}

int semcond_element_grads(semcond_ctx* c, const void* u, const void* a, void* grad, int k, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!u || !a || !grad) return fail(c, SEMCOND_EINVAL, "NULL pointer");
    if (k < 1 || k > 256) return fail(c, SEMCOND_EINVAL, "k must be in [1, 256]");
    HIPCHK(c, launch_element_grads(c->geo, c->t64.tab.w, c->t64.K, (const double*)u, (const double*)a, c->N, k,
                                   (double*)grad, false, S(stream)));
    return SEMCOND_OK;
}

int semcond_element_grads_rhs(semcond_ctx* c, const void* u, const void* a, void* grad, int k, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!u || !a || !grad) return fail(c, SEMCOND_EINVAL, "NULL pointer");
    if (k < 1 || k > 256) return fail(c, SEMCOND_EINVAL, "k must be in [1, 256]");
    HIPCHK(c, launch_element_grads(c->geo, c->t64.tab.w, c->t64.K, (const double*)u, (const double*)a, c->N, k,
                                   (double*)grad, true, S(stream)));
    return SEMCOND_OK;
}

void semcond_solve_opts_default(semcond_solve_opts* o) {
    if (!o) return;
    o->tol = 1e-10;
    o->max_iter = 20000;
    o->precision = SEMCOND_PREC_F64;
    o->check_every = 8;
    o->recover_interior = 1;
    o->x0 = nullptr;
    o->skel_out = nullptr;
    o->inner_tol = 3e-3;
    o->max_outer = 30;
    o->rhs_dual = 0;
    o->persistent = SEMCOND_CG_AUTO;
    o->g_dirichlet = nullptr;
    o->ir_restart = 0;
    o->deterministic = 0;
    o->coarse = 0;
}

int semcond_set_deterministic(semcond_ctx* c, int on) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    c->det = on != 0;
    return SEMCOND_OK;
}

int semcond_recover_interior(semcond_ctx* c, const void* f, const void* u_skel, void* u, int k, int dtype,
                             void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!f || !u_skel || !u) return fail(c, SEMCOND_EINVAL, "f, u_skel and u must be device pointers");
    if (dtype != SEMCOND_F64) return fail(c, SEMCOND_EINVAL, "interior recovery is FP64 only");
    int rc = check_k(c, k);
    if (rc) return rc;
    hipStream_t st = S(stream);
    const size_t nv = (size_t)c->N_s * k;
    rc = grow(c, c->ws_vec, nv * sizeof(double));
    if (rc) return rc;
    double* phys = (double*)c->ws_vec.ptr;
    // skeleton nodes: u = T u~ (Dirichlet entities keep the values given in u_skel);
    // interior nodes: u_I = (S(x)S(x)S) D^-1 (F~_I - H~_IB u~_B) (Algorithm 4, second loop)
    HIPCHK(c, launch_transform<double>(c->L, c->t64.tab.S, (const double*)u_skel, phys, k, st));
    HIPCHK(c, launch_skel_to_nodal(c->L, phys, (double*)u, c->N, k, 1, st));
    return recover_interior64(c, (const double*)f, (const double*)u_skel, (double*)u, k, 1, st);
}

int semcond_reserve(semcond_ctx* c, int k_max, int dtype) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (dtype != SEMCOND_F64 && dtype != SEMCOND_F32) return fail(c, SEMCOND_EINVAL, "dtype must be F64 or F32");
    int rc = check_k(c, k_max);
    if (rc) return rc;
    const int k = k_max;
    const size_t nv = (size_t)c->N_s * k;
    // solve vectors (FP64 b x r p q, FP32 ones for F32 / MIXED_IR), which also
    // cover the applies' and transforms' temporaries (at most 2 N_s k values)
    rc = grow(c, c->ws_vec, 5 * nv * sizeof(double) + (dtype == SEMCOND_F32 ? 5 * nv * sizeof(float) : 0));
    if (rc) return rc;
    CgWork w;
    rc = cg_state(c, k, 0, &w);  // both state slots, pinned activity copy
    if (rc) return rc;
    const int64_t qlen = slot_len(c->L);
    if (qlen * (int64_t)k < (int64_t(1) << 31)) {
        rc = grow(c, c->ws_slots, (size_t)qlen * k * sizeof(double));
        if (rc) return rc;
    }
    int grid;
    double* scratch;
    rc = scratch_for_cubes(c, &grid, &scratch);
    if (rc) return rc;
    rc = grow(c, c->ws_lift, 2 * nv * sizeof(double));  // prescribed Dirichlet values
    if (rc) return rc;
    rc = grow(c, c->ws_nodal, (size_t)c->N * k * sizeof(double));  // assembled (dual) right-hand sides
    if (rc) return rc;
    // persistent CG: partial sums for the largest co-resident grid, barrier words
    size_t pb = 0;
    for (int S0 : {1, 2, 4}) {
        if (!persist_supported(c->L.NI, S0, k)) continue;
        const int mg = dtype == SEMCOND_F64 ? persist_max_grid<double>(c->L.NI, S0)
                                            : std::max(persist_max_grid<double>(c->L.NI, S0),
                                                       persist_max_grid<float>(c->L.NI, S0));
        pb = std::max(pb, (3 * (size_t)std::max(mg, 0) * k * sizeof(double) + 255) / 256 * 256);
    }
    if (pb) {
        rc = grow(c, c->ws_persist, pb + kBarWords * sizeof(unsigned));
        if (rc) return rc;
    }
    // host side of the fused CG loop's convergence polls
    for (hipEvent_t& e : c->poll_ev)
        if (!e) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (!c->h_flags && hipHostMalloc((void**)&c->h_flags, kMaxRhs * sizeof(int), hipHostMallocCoherent) != hipSuccess)
        return fail(c, SEMCOND_ENOMEM, "pinned host allocation failed");
    HIPCHK(c, hipDeviceSynchronize());
    return SEMCOND_OK;
}

int semcond_solve(semcond_ctx* c, const void* f, void* u, int k, const semcond_solve_opts* opts,
                  semcond_solve_info* info, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!f || !u) return fail(c, SEMCOND_EINVAL, "f and u must be device pointers");
    int rc = check_k(c, k);
    if (rc) return rc;
    semcond_solve_opts o;
    if (opts)
        o = *opts;
    else
        semcond_solve_opts_default(&o);
    if (!(o.tol > 0.0) || o.max_iter < 0) return fail(c, SEMCOND_EINVAL, "tol must be > 0 and max_iter >= 0");
    if (o.precision < SEMCOND_PREC_F64 || o.precision > SEMCOND_PREC_MIXED_IR)
        return fail(c, SEMCOND_EINVAL, "unknown precision mode");
    if (o.precision == SEMCOND_PREC_MIXED_IR && (!(o.inner_tol > 0.0 && o.inner_tol < 1.0) || o.max_outer < 1))
        return fail(c, SEMCOND_EINVAL, "MIXED_IR needs 0 < inner_tol < 1 and max_outer >= 1");
    hipStream_t st = S(stream);
    DetScope det(c, c->det || o.deterministic != 0);
    struct CoarseScope {
        semcond_ctx* c;
        CoarseScope(semcond_ctx* ctx, bool on) : c(ctx) { c->coarse_active = on; }
        ~CoarseScope() { c->coarse_active = false; }
    } coarse_scope(c, o.coarse != 0);
    const int64_t Ns = c->N_s;
    const size_t nv = (size_t)Ns * k;
    if (o.rhs_dual) {
        // an assembled right-hand side g equals M_G f' for the nodal values f' = g / M_G
        rc = grow(c, c->ws_nodal, (size_t)c->N * k * sizeof(double));
        if (rc) return rc;
        HIPCHK(c, launch_mass_apply(c->geo, c->t64.tab.w, (const double*)f, (double*)c->ws_nodal.ptr, c->N, k, 1, st));
        f = c->ws_nodal.ptr;
    }
    // FP64 vectors b x r p q, then FP32 vectors b x r p q
    rc = grow(c, c->ws_vec, 5 * nv * sizeof(double) + (o.precision == SEMCOND_PREC_F64 ? 0 : 5 * nv * sizeof(float)));
    if (rc) return rc;
    double* b = (double*)c->ws_vec.ptr;
    double* x = b + nv;
    double* r = x + nv;
    double* p = r + nv;
    double* q = p + nv;
    float* b32 = (float*)(q + nv);
    float* x32 = b32 + nv;
    float* r32 = x32 + nv;
    float* p32 = r32 + nv;
    float* q32 = p32 + nv;
    CgWork w;
    rc = cg_state(c, k, 0, &w);
    if (rc) return rc;
    // Without prescribed Dirichlet values the condensed right-hand side is
    // written RHS-major [k][N_s] straight away (the layout of the conjugate
    // gradients), and the post-processing reads the solution in that layout.
    const bool rmaj = k > 1 && !o.g_dirichlet;
    const SkelStride rm{1, Ns};
    rc = condense_rhs64(c, (const double*)f, b, k, st, rmaj ? rm : SkelStride{});
    if (rc) return rc;
    // Prescribed Dirichlet values: g~ = T^-1 g on the Dirichlet entities (zero
    // elsewhere; the transform keeps every entity to itself), and the lift
    // F^~_free -= (H~^ g~)_free with the apply reading the Dirichlet entities.
    double* gl = nullptr;
    if (o.g_dirichlet) {
        rc = grow(c, c->ws_lift, 2 * nv * sizeof(double));
        if (rc) return rc;
        gl = (double*)c->ws_lift.ptr;
        double* tmp = gl + nv;
        HIPCHK(c, launch_nodal_to_skel(c->L, (const double*)o.g_dirichlet, tmp, c->N, k, st));
        HIPCHK(c, launch_mask_nodes(c->L, tmp, k, KEEP_CONSTRAINED, st));
        HIPCHK(c, launch_transform<double>(c->L, c->t64.tab.Sinv, tmp, gl, k, st));
        rc = apply_transformed<double>(c, gl, tmp, k, NODE_MAJOR, nullptr, st, false, nullptr, nullptr, 1);
        if (rc) return rc;
        HIPCHK(c, launch_axpy(b, tmp, -1.0, (int64_t)nv, st));
    }
    // the initial guess holds unknowns only (entries on Dirichlet entities are ignored)
    if (o.x0) {
        HIPCHK(c, hipMemcpyAsync(q, o.x0, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(c, launch_mask_nodes(c->L, q, k, KEEP_FREE, st));
    }
    // the conjugate gradients run on RHS-major vectors [k][N_s]
    if (k > 1 && !rmaj) {
        HIPCHK(c, launch_transpose<double>(b, p, Ns, k, st));
        std::swap(b, p);
    }
    if (o.x0) {
        if (k > 1)
            HIPCHK(c, launch_transpose<double>(q, x, Ns, k, st));
        else
            HIPCHK(c, hipMemcpyAsync(x, q, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    }

    std::vector<int> iters(k, 0), status(k, 0), outer(k, 0);
    std::vector<double> relres(k, 0.0);
    CgHost h;
    if (o.precision == SEMCOND_PREC_F64) {
        rc = run_cg_any<double>(c, b, x, r, p, q, k, o.tol, o.max_iter, o.check_every, o.x0 != nullptr,
                                o.persistent, w, st);
        if (rc) return rc;
        rc = read_state(c, w, k, &h, st);
        if (rc) return rc;
        for (int i = 0; i < k; ++i) {
            iters[i] = h.iters[i];
            status[i] = h.status[i] == 0 && h.active[i] ? SEMCOND_ENOTCONV : h.status[i];
            relres[i] = h.bb[i] > 0 ? std::sqrt(h.rr[i] / h.bb[i]) : 0.0;
        }
    } else if (o.precision == SEMCOND_PREC_F32) {
        // FP32 operator and vectors, FP64 dot products; no refinement
        HIPCHK(c, (launch_convert<double, float>(b, b32, nv, st)));
        if (o.x0) HIPCHK(c, (launch_convert<double, float>(x, x32, nv, st)));
        rc = run_cg_any<float>(c, b32, x32, r32, p32, q32, k, o.tol, o.max_iter, o.check_every, o.x0 != nullptr,
                               o.persistent, w, st);
        if (rc) return rc;
        HIPCHK(c, (launch_convert<float, double>(x32, x, nv, st)));
        rc = read_state(c, w, k, &h, st);
        if (rc) return rc;
        for (int i = 0; i < k; ++i) {
            iters[i] = h.iters[i];
            status[i] = h.status[i] == 0 && h.active[i] ? SEMCOND_ENOTCONV : h.status[i];
        }
        // report the FP64 residual of the FP32 solution
        CgWork wo;
        rc = cg_state(c, k, 1, &wo);
        if (rc) return rc;
        const double tol2 = o.tol * o.tol;
        HIPCHK(c, hipMemcpyAsync(wo.s.tol2, &tol2, sizeof(double), hipMemcpyHostToDevice, st));
        rc = apply_transformed<double>(c, x, q, k, RHS_MAJOR, nullptr, st);
        if (rc) return rc;
        HIPCHK(c, launch_cg_init<double>(b, q, c->d_pinv64, r, p, Ns, k, wo.partials, st));
        HIPCHK(c, launch_cg_reduce(wo.partials, vec_blocks(k), 3, k, wo.s, RED_INIT, st));
        CgHost ho;
        rc = read_state(c, wo, k, &ho, st);
        if (rc) return rc;
        for (int i = 0; i < k; ++i) relres[i] = ho.bb[i] > 0 ? std::sqrt(ho.rr[i] / ho.bb[i]) : 0.0;
    } else {
        // Iterative refinement: outer FP64 residual r = b - A64 x, inner FP32
        // CG on A32 d = r (FP64 dot products), x += d, until ||r|| <= tol ||b||.
        CgWork wo;
        rc = cg_state(c, k, 1, &wo);
        if (rc) return rc;
        const double tol2 = o.tol * o.tol;
        HIPCHK(c, hipMemcpyAsync(wo.s.tol2, &tol2, sizeof(double), hipMemcpyHostToDevice, st));
        if (!o.x0) HIPCHK(c, launch_fill<double>(x, nv, 0.0, st));
        HIPCHK(c, launch_fill<double>(q, nv, 0.0, st));
        int step = 0;
        double prev_worst = 0.0;
        bool keep = false;  // continue the inner direction in this step
        for (;; ++step) {
            // r = b - A64 x (q holds A64 x; zeroed again by cg_init), convergence per RHS
            if (step > 0 || o.x0) {
                rc = apply_transformed<double>(c, x, q, k, RHS_MAJOR, nullptr, st, true);
                if (rc) return rc;
            }
            HIPCHK(c, launch_cg_init<double>(b, q, c->d_pinv64, r, p, Ns, k, wo.partials, st));
            HIPCHK(c, launch_cg_reduce(wo.partials, vec_blocks(k), 3, k, wo.s, RED_INIT, st));
            CgHost ho;
            rc = read_state(c, wo, k, &ho, st);
            if (rc) return rc;
            bool any = false;
            for (int i = 0; i < k; ++i) {
                relres[i] = ho.bb[i] > 0 ? std::sqrt(ho.rr[i] / ho.bb[i]) : 0.0;
                if (ho.status[i] < 0) status[i] = ho.status[i];
                if (ho.active[i] && status[i] >= 0) {
                    any = true;
                    outer[i] = step + 1;
                }
            }
            if (!any) break;
            if (step >= o.max_outer) {
                for (int i = 0; i < k; ++i)
                    if (ho.active[i] && status[i] == 0) status[i] = SEMCOND_ENOTCONV;
                break;
            }
            // Inner tolerance: inner_tol, or a looser one when a smaller reduction
            // (with a factor 4 margin) takes every active RHS to tol.
            double worst = 0.0, need = 0.5;
            for (int i = 0; i < k; ++i)
                if (ho.active[i] && status[i] >= 0) {
                    worst = std::max(worst, relres[i]);
                    if (relres[i] > 0.0) need = std::min(need, 0.25 * o.tol / relres[i]);
                }
            // ... but never below what the FP32 operator can reach: its face rows
            // cancel K_00 against the 1D Schur value 1/2 (Sec. 6 transformed
            // primary part), so its rounding error relative to the residual is
            // about 2 K_00 FP32 units; a margin of 8 on top.
            const double fp32_floor = 8.0 * 0x1p-24 * 2.0 * c->t.K00;
            const double run_tol = std::max(std::max(o.inner_tol, need), fp32_floor);
            // The FP32 CG continues its search direction across refinement steps
            // (only the residual is replaced by the FP64 one) unless restarts are
            // asked for, or the last step did not halve the worst residual.
            keep = step > 0 && !o.ir_restart && worst < 0.5 * prev_worst;
            prev_worst = worst;
            HIPCHK(c, launch_convert_masked(r, r32, nv, k, wo.s.active, st));
            w.s.window = kInnerStallWindow;  // an inner solve that stops halving its residual ends
            rc = run_cg_any<float>(c, r32, x32, b32, p32, q32, k, run_tol, o.max_iter, o.check_every, false,
                                   o.persistent, w, st, keep);
            w.s.window = 0;
            if (rc) return rc;
            CgHost hi;
            rc = read_state(c, w, k, &hi, st);
            if (rc) return rc;
            for (int i = 0; i < k; ++i) {
                iters[i] += hi.iters[i];
                if (hi.status[i] < 0 && status[i] == 0) status[i] = hi.status[i];
            }
            HIPCHK(c, launch_add_mixed(x, x32, nv, st));
        }
    }

    // the physical basis and the nodal array (Algorithm 4, second loop), from the
    // RHS-major solution, or from its [N_s][k] copy with prescribed values
    double* xs = x;
    SkelStride xl{};
    if (rmaj) {
        xl = rm;
    } else if (k > 1) {
        HIPCHK(c, launch_transpose<double>(x, q, k, Ns, st));
        xs = q;
    }
    if (gl) HIPCHK(c, launch_axpy(xs, gl, 1.0, (int64_t)nv, st));  // u~ = unknowns + g~
    const int keep = gl ? 1 : 0;
    HIPCHK(c, launch_transform<double>(c->L, c->t64.tab.S, xs, p, k, st, xl));
    HIPCHK(c, launch_skel_to_nodal(c->L, p, (double*)u, c->N, k, keep, st, xl));
    if (o.recover_interior) {
        rc = recover_interior64(c, (const double*)f, xs, (double*)u, k, keep, st, xl);
        if (rc) return rc;
    }
    if (o.skel_out) {
        if (rmaj)
            HIPCHK(c, launch_transpose<double>(xs, (double*)o.skel_out, k, Ns, st));
        else
            HIPCHK(c, hipMemcpyAsync(o.skel_out, xs, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(c, hipStreamSynchronize(st));
    int worst = SEMCOND_OK;
    for (int i = 0; i < k; ++i) {
        if (info) {
            info[i].iters = iters[i];
            info[i].outer = outer[i];
            info[i].rel_res = relres[i];
            info[i].status = status[i];
        }
        if (status[i] < 0) worst = status[i];
        else if (status[i] == SEMCOND_ENOTCONV && worst == SEMCOND_OK) worst = status[i];
    }
    if (worst != SEMCOND_OK) fail(c, worst, "solve did not converge for every right-hand side");
    return worst;
}

// ---------------------------------------------------------------------------
// Operator variants of Sec. 7 (physical basis, FP64)
// ---------------------------------------------------------------------------

int semcond_variant_setup(semcond_ctx* c, int variant, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (variant == SEMCOND_VARIANT_TPC) return SEMCOND_OK;  // nothing beyond the 1D tables
    if (variant != SEMCOND_VARIANT_MMC) return fail(c, SEMCOND_EINVAL, "unknown operator variant");
    hipStream_t st = S(stream);
    const int NI = c->L.NI;
    const int64_t nB = 6 * (int64_t)NI * NI + 12 * NI + 8;
    // element classes: equal metric coefficients (the device's own values)
    std::vector<double> hd;
    {
        int rc = element_metrics_host(c, st, hd);
        if (rc) return rc;
    }
    std::map<std::vector<double>, int> cls;
    std::vector<int> cl(c->n_e);
    std::vector<std::vector<double>> keys;
    for (int64_t e = 0; e < c->n_e; ++e) {
        std::vector<double> key(hd.begin() + 4 * e, hd.begin() + 4 * e + 4);
        auto it = cls.find(key);
        if (it == cls.end()) {
            it = cls.emplace(key, (int)keys.size()).first;
            keys.push_back(key);
        }
        cl[e] = it->second;
    }
    const int nc = (int)keys.size();
    const double mbytes = (double)nc * nB * nB * sizeof(double);
    if (mbytes > 16.0 * (1 << 30))
        return fail(c, SEMCOND_EINVAL, "MMC: the element matrices of " + std::to_string(nc) + " classes would need " +
                                           std::to_string(mbytes / (1 << 30)) + " GiB (limit 16)");
    std::vector<int64_t> start(nc, 0), count(nc, 0);
    for (int64_t e = 0; e < c->n_e; ++e) ++count[cl[e]];
    for (int q = 1; q < nc; ++q) start[q] = start[q - 1] + count[q - 1];
    std::vector<int> col(c->n_e);
    {
        std::vector<int64_t> next = start;
        for (int64_t e = 0; e < c->n_e; ++e) col[e] = (int)next[cl[e]]++;
    }
    hipFree(c->mmc_H);
    hipFree(c->mmc_col);
    c->mmc_H = nullptr;
    c->mmc_col = nullptr;
    HIPCHK(c, hipMalloc(&c->mmc_H, (size_t)mbytes));
    HIPCHK(c, hipMalloc(&c->mmc_col, col.size() * sizeof(int)));
    HIPCHK(c, hipMemcpy(c->mmc_col, col.data(), col.size() * sizeof(int), hipMemcpyHostToDevice));
    // Each class's matrix: the condensed operator of one element with that
    // metric and no Dirichlet face, applied in the physical basis to the unit
    // vectors of its n_B boundary nodes (a one-element skeleton lists them in
    // the local slot order of the gather).
    const int kc = (int)std::min<int64_t>(nB, 256);
    double *dU = nullptr, *dV = nullptr;
    HIPCHK(c, hipMalloc(&dU, (size_t)nB * kc * sizeof(double)));
    HIPCHK(c, hipMalloc(&dV, (size_t)nB * kc * sizeof(double)));
    std::vector<double> hU((size_t)nB * kc);
    int rc = SEMCOND_OK;
    for (int q = 0; q < nc && rc == SEMCOND_OK; ++q) {
        double w2[1] = {2.0};
        semcond_mesh m1{};
        m1.p = c->p;
        m1.n[0] = m1.n[1] = m1.n[2] = 1;
        m1.widths[0] = m1.widths[1] = m1.widths[2] = w2;
        m1.lambda = 0.0;
        m1.lambda_e = nullptr;
        m1.dcoef_e = keys[q].data();
        m1.dirichlet_mask = 0;
        semcond_ctx* one = nullptr;
        rc = create_context(&m1, stream, &one, false);
        if (rc) {
            fail(c, rc, "MMC: element context: " + g_last_error);
            break;
        }
        double* Hq = c->mmc_H + (size_t)q * nB * nB;
        for (int64_t j0 = 0; j0 < nB && rc == SEMCOND_OK; j0 += kc) {
            const int kk = (int)std::min<int64_t>(kc, nB - j0);
            std::fill(hU.begin(), hU.end(), 0.0);
            for (int t = 0; t < kk; ++t) hU[(size_t)(j0 + t) * kk + t] = 1.0;
            hipError_t he = hipMemcpyAsync(dU, hU.data(), (size_t)nB * kk * sizeof(double), hipMemcpyHostToDevice, st);
            if (he != hipSuccess) {
                rc = fail(c, SEMCOND_EDEVICE, "MMC: upload failed");
                break;
            }
            rc = semcond_apply(one, dU, dV, kk, SEMCOND_F64, SEMCOND_PHYSICAL, stream);
            if (rc) {
                fail(c, rc, "MMC: element apply: " + std::string(semcond_last_error(one)));
                break;
            }
            he = launch_transpose<double>(dV, Hq + (size_t)j0 * nB, nB, kk, st);
            if (he == hipSuccess) he = hipStreamSynchronize(st);
            if (he != hipSuccess) rc = fail(c, SEMCOND_EDEVICE, "MMC: column copy failed");
        }
        semcond_destroy(one);
    }
    hipFree(dU);
    hipFree(dV);
    if (rc) return rc;
    c->mmc_start = start;
    c->mmc_count = count;
    if (!c->blas && rocblas_create_handle(&c->blas) != rocblas_status_success) {
        c->blas = nullptr;
        return fail(c, SEMCOND_EDEVICE, "rocblas_create_handle failed");
    }
    return SEMCOND_OK;
}

int semcond_apply_variant(semcond_ctx* c, const void* u, void* v, int k, int variant, void* stream) {
    if (!c) return fail(nullptr, SEMCOND_EINVAL, "ctx is NULL");
    if (!u || !v) return fail(c, SEMCOND_EINVAL, "u and v must be device pointers");
    if (u == v) return fail(c, SEMCOND_EINVAL, "u and v must not overlap");
    int rc = check_k(c, k);
    if (rc) return rc;
    hipStream_t st = S(stream);
    const int64_t Ns = c->N_s;
    if (variant == SEMCOND_VARIANT_TPC) {
        HIPCHK(c, launch_fill<double>((double*)v, Ns * k, 0.0, st));
        HIPCHK(c, launch_apply_tpc(c->geo, c->t64.tab, c->t64.K, (const double*)u, (double*)v, k, st));
        return SEMCOND_OK;
    }
    if (variant != SEMCOND_VARIANT_MMC) return fail(c, SEMCOND_EINVAL, "unknown operator variant");
    if (!c->mmc_H) return fail(c, SEMCOND_EINVAL, "MMC: call semcond_variant_setup first");
    const int NI = c->L.NI;
    const int64_t nB = 6 * (int64_t)NI * NI + 12 * NI + 8;
    const size_t cols = (size_t)c->n_e * k;
    rc = grow(c, c->ws_mmc, 2 * nB * cols * sizeof(double));
    if (rc) return rc;
    double* UL = (double*)c->ws_mmc.ptr;
    double* VL = UL + nB * cols;
    HIPCHK(c, launch_mmc_gather(c->L, c->mmc_col, (const double*)u, UL, k, st));
    if (rocblas_set_stream(c->blas, st) != rocblas_status_success)
        return fail(c, SEMCOND_EDEVICE, "rocblas_set_stream failed");
    const double one = 1.0, zero = 0.0;
    for (size_t q = 0; q < c->mmc_start.size(); ++q) {
        const int64_t c0 = c->mmc_start[q] * k, nq = c->mmc_count[q] * k;
        if (nq == 0) continue;
        if (rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)nB, (rocblas_int)nq,
                          (rocblas_int)nB, &one, c->mmc_H + (size_t)q * nB * nB, (rocblas_int)nB, UL + c0 * nB,
                          (rocblas_int)nB, &zero, VL + c0 * nB, (rocblas_int)nB) != rocblas_status_success)
            return fail(c, SEMCOND_EDEVICE, "rocblas_dgemm failed");
    }
    HIPCHK(c, launch_fill<double>((double*)v, Ns * k, 0.0, st));
    HIPCHK(c, launch_mmc_scatter(c->L, c->mmc_col, VL, (double*)v, k, st));
    return SEMCOND_OK;
}

}  // extern "C"
