// fj_api.hip -- the extern "C" entry points of libfjgpu (declared in include/fj.h).
//
// Host side of the hot path: argument checks, plan and workspace carving,
// kernel launches on the caller's stream, and the CG driver. One CG
// iteration is four launches: the SpMV with its dot products, a one-workgroup
// kernel that forms alpha and beta, the fused vector update, and a
// one-workgroup kernel that forms the new residual norms. The driver
// enqueues CG iterations in chunks and copies the 1 KiB control block to
// pinned host memory after each chunk; while the GPU runs one chunk the host
// reads the status of the previous one and, from the residual history,
// predicts how many more iterations the stopping test needs. Kernels whose
// control block says "done" return at once, so overshoot costs only empty
// launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/fj.h"
#include "fj_kernels.hpp"

using namespace fj;

namespace {

constexpr size_t ALIGN = 256;
constexpr int NSLOT = 4;
constexpr int FIRST_CHUNK = 6;
constexpr int MAX_PASSES = 5;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

thread_local char g_last_error[256] = "";

void set_error(const char* what, hipError_t e) {
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(call)                              \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) {                   \
            set_error(#call, e_);                 \
            return FJ_ERR_HIP;                    \
        }                                         \
    } while (0)

// ---------------------------------------------------------------- layouts

struct PlanLayout {
    int K;            // number of row windows
    size_t blk_row;   // int[K + 1]
    size_t desc;      // WinDesc[K]
    size_t minv;      // float[n]
    size_t flags;     // int[64] scratch for validation
    size_t total;
};

PlanLayout plan_layout(const fj_csr* g) {
    PlanLayout L{};
    const int64_t keys = static_cast<int64_t>(g->n) + g->nnz;
    L.K = static_cast<int>((keys + WIN - 1) / WIN);
    size_t off = 0;
    L.blk_row = off;
    off = align_up(off + sizeof(int) * (static_cast<size_t>(L.K) + 1));
    L.desc = off;
    off = align_up(off + sizeof(WinDesc) * static_cast<size_t>(L.K));
    L.minv = off;
    off = align_up(off + sizeof(float) * static_cast<size_t>(g->n));
    L.flags = off;
    off = align_up(off + sizeof(int) * 64);
    L.total = off;
    return L;
}

struct WsLayout {
    size_t x, r, p, q, part, ctrl, total;
};

WsLayout ws_layout(const fj_csr* g, int k) {
    WsLayout L{};
    const size_t vec = align_up(sizeof(double) * static_cast<size_t>(g->n) * static_cast<size_t>(k));
    size_t off = 0;
    L.x = off; off += vec;
    L.r = off; off += vec;
    L.p = off; off += vec;
    L.q = off; off += vec;
    L.part = off; off = align_up(off + sizeof(double) * GMAX * NPART);
    L.ctrl = off; off = align_up(off + sizeof(Ctrl) * static_cast<size_t>(k));
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- device facts

struct DeviceFacts {
    int cus = 0;
    std::map<const void*, int> per_cu;  // resident workgroups per CU, per kernel
};

std::mutex g_dev_mu;
std::map<int, DeviceFacts> g_dev;

int current_device(int* dev) {
    HIPCHK(hipGetDevice(dev));
    return FJ_OK;
}

// Persistent grid: as many workgroups as fit on the device at once, capped
// by the amount of work and by GMAX.
template <typename Kern>
int grid_for(Kern kernel, int64_t work_units, int* grid) {
    int dev = 0;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lock(g_dev_mu);
    DeviceFacts& f = g_dev[dev];
    if (f.cus == 0) HIPCHK(hipDeviceGetAttribute(&f.cus, hipDeviceAttributeMultiprocessorCount, dev));
    const void* key = reinterpret_cast<const void*>(kernel);
    auto it = f.per_cu.find(key);
    if (it == f.per_cu.end()) {
        int nb = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, WG, 0));
        it = f.per_cu.emplace(key, std::max(nb, 1)).first;
    }
    const int64_t full = static_cast<int64_t>(f.cus) * it->second;
    *grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>({full, static_cast<int64_t>(GMAX), work_units})));
    return FJ_OK;
}

// ---------------------------------------------------------------- host slots

struct HostSlots {
    Ctrl* h = nullptr;                 // pinned, NSLOT + 1 control-block copies
    hipEvent_t ev[NSLOT + 1] = {};
    std::vector<hipEvent_t> prof;      // FJ_PROFILE event pairs
};

thread_local std::map<int, HostSlots> tl_slots;

int host_slots(HostSlots** out) {
    int dev = 0;
    if (int rc = current_device(&dev)) return rc;
    HostSlots& hs = tl_slots[dev];
    if (!hs.h) {
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hs.h), sizeof(Ctrl) * (NSLOT + 1), hipHostMallocDefault));
        for (auto& e : hs.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    *out = &hs;
    return FJ_OK;
}

int profile_events(HostSlots& hs, size_t pairs) {
    while (hs.prof.size() < 2 * pairs) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        hs.prof.push_back(e);
    }
    return FJ_OK;
}

// ---------------------------------------------------------------- dispatch

template <typename F>
int with_graph(const fj_csr* g, F&& f) {
    switch (g->val_type) {
        case FJ_VAL_UNIT:
            return f(Csr<Unit>{g->n, static_cast<int>(g->nnz), g->row_ptr, g->col_idx, nullptr});
        case FJ_VAL_F32:
            return f(Csr<float>{g->n, static_cast<int>(g->nnz), g->row_ptr, g->col_idx, static_cast<const float*>(g->val)});
        case FJ_VAL_F64:
            return f(Csr<double>{g->n, static_cast<int>(g->nnz), g->row_ptr, g->col_idx, static_cast<const double*>(g->val)});
        default:
            return FJ_ERR_INVALID_ARG;
    }
}

int check_graph_args(const fj_csr* g) {
    if (!g || g->n < 0 || g->nnz < 0 || g->nnz >= (int64_t(1) << 31)) return FJ_ERR_INVALID_ARG;
    if (g->n > 0 && (!g->row_ptr || (g->nnz > 0 && !g->col_idx))) return FJ_ERR_INVALID_ARG;
    if (g->n == 0 && g->nnz != 0) return FJ_ERR_INVALID_GRAPH;
    if (g->val_type == FJ_VAL_UNIT) {
        if (g->val) return FJ_ERR_INVALID_ARG;
    } else if (g->val_type == FJ_VAL_F32 || g->val_type == FJ_VAL_F64) {
        if (!g->val && g->nnz > 0) return FJ_ERR_INVALID_ARG;
    } else {
        return FJ_ERR_INVALID_ARG;
    }
    return FJ_OK;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) % ALIGN) == 0; }

int check_opts(const fj_opts* o) {
    if (!o) return FJ_ERR_INVALID_ARG;
    if (!(o->eps > 0.0 && o->eps < 0.5)) return FJ_ERR_INVALID_ARG;
    if (!(o->rtol >= 0.0 && o->rtol < 1.0)) return FJ_ERR_INVALID_ARG;
    if (o->max_iter < 0 || o->reserved != 0) return FJ_ERR_INVALID_ARG;
    if (o->precision != FJ_FP64) return FJ_ERR_INVALID_ARG;  // FJ_MIXED: see the mixed driver
    return FJ_OK;
}

int status_of(int done) {
    switch (done) {
        case CONVERGED: return FJ_OK;
        case ITER_CAP: return FJ_ERR_NOT_CONVERGED;
        case BREAKDOWN: return FJ_ERR_BREAKDOWN;
        case BAD_INPUT: return FJ_ERR_OPINION_RANGE;
        default: return FJ_ERR_NOT_CONVERGED;
    }
}

// ---------------------------------------------------------------- one solve

struct Solver {
    const fj_csr* g;
    PlanLayout pl;
    const char* plan;
    WsLayout wl;
    char* ws;
    hipStream_t st;
    HostSlots* hs;
    bool profile;
    int grid_win = 1, grid_vec = 1;
    size_t n_prof = 0;  // event pairs used

    double* x() const { return reinterpret_cast<double*>(ws + wl.x); }
    double* r() const { return reinterpret_cast<double*>(ws + wl.r); }
    double* p() const { return reinterpret_cast<double*>(ws + wl.p); }
    double* q() const { return reinterpret_cast<double*>(ws + wl.q); }
    double* part() const { return reinterpret_cast<double*>(ws + wl.part); }
    Ctrl* ctrl() const { return reinterpret_cast<Ctrl*>(ws + wl.ctrl); }
    const WinDesc* desc() const { return reinterpret_cast<const WinDesc*>(plan + pl.desc); }
    const float* minv() const { return reinterpret_cast<const float*>(plan + pl.minv); }

    int setup() {
        int rc = with_graph(g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            return grid_for(k_cg_spmv<Vc>, pl.K, &grid_win);
        });
        if (rc) return rc;
        return grid_for(k_cg_update, (static_cast<int64_t>(g->n) + 2 * WG - 1) / (2 * WG), &grid_vec);
    }

    int init(const double* s, int64_t lds, int mode, double rtol, int max_iter, bool range_check) {
        if (mode == 0) {
            k_ctrl_reset<<<1, WG, 0, st>>>(ctrl(), 1);
            HIPCHK(hipGetLastError());
        }
        k_cg_init<<<grid_vec, WG, 0, st>>>(g->n, s, lds, x(), r(), p(), minv(), mode, part());
        HIPCHK(hipGetLastError());
        k_fin_init<<<1, WG, 0, st>>>(grid_vec, g->n, part(), mode, rtol * rtol, max_iter, range_check ? 1 : 0,
                                     ctrl());
        HIPCHK(hipGetLastError());
        return FJ_OK;
    }

    int launch_iteration() {
        int rc = with_graph(g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            if (profile) {
                if (int e = profile_events(*hs, n_prof + 1)) return e;
                HIPCHK(hipEventRecord(hs->prof[2 * n_prof], st));
            }
            k_cg_spmv<Vc><<<grid_win, WG, 0, st>>>(G, desc(), pl.K, p(), r(), minv(), q(), part(), ctrl());
            HIPCHK(hipGetLastError());
            if (profile) {
                HIPCHK(hipEventRecord(hs->prof[2 * n_prof + 1], st));
                ++n_prof;
            }
            return FJ_OK;
        });
        if (rc) return rc;
        k_fin_spmv<<<1, WG, 0, st>>>(grid_win, part(), ctrl());
        HIPCHK(hipGetLastError());
        k_cg_update<<<grid_vec, WG, 0, st>>>(g->n, x(), r(), p(), q(), minv(), part(), ctrl());
        HIPCHK(hipGetLastError());
        k_fin_update<<<1, WG, 0, st>>>(grid_vec, part(), ctrl());
        HIPCHK(hipGetLastError());
        return FJ_OK;
    }

    // Run CG until the control block says done. `start` = iterations already
    // done before this pass. Leaves the final status copy in *out.
    int run(int start, int max_iter, Ctrl* out) {
        int queued = start;
        int slot_next = 0;
        std::deque<int> pending;
        auto enqueue = [&](int cnt) -> int {
            for (int t = 0; t < cnt; ++t)
                if (int rc = launch_iteration()) return rc;
            queued += cnt;
            const int sl = slot_next++ % NSLOT;
            HIPCHK(hipMemcpyAsync(&hs->h[sl], ctrl(), sizeof(Ctrl), hipMemcpyDeviceToHost, st));
            HIPCHK(hipEventRecord(hs->ev[sl], st));
            pending.push_back(sl);
            return FJ_OK;
        };
        for (int c = 0; c < 2 && queued < max_iter; ++c)
            if (int rc = enqueue(std::min(FIRST_CHUNK, max_iter - queued))) return rc;
        if (pending.empty()) {  // nothing to do: report the state after init
            HIPCHK(hipMemcpyAsync(out, ctrl(), sizeof(Ctrl), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            return FJ_OK;
        }
        while (!pending.empty()) {
            const int sl = pending.front();
            pending.pop_front();
            HIPCHK(hipEventSynchronize(hs->ev[sl]));
            const Ctrl& c = hs->h[sl];
            if (c.done != RUNNING || c.iters >= max_iter) {
                std::memcpy(out, &c, sizeof(Ctrl));
                // later chunks are empty launches; let them drain before returning
                HIPCHK(hipStreamSynchronize(st));
                if (!pending.empty()) std::memcpy(out, &hs->h[pending.back()], sizeof(Ctrl));
                return FJ_OK;
            }
            int need = predict(c, start);
            need = std::min(need, max_iter);
            if (need > queued) {
                if (int rc = enqueue(need - queued)) return rc;
            } else if (pending.empty() && queued < max_iter) {
                if (int rc = enqueue(1)) return rc;
            }
        }
        HIPCHK(hipMemcpyAsync(out, ctrl(), sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return FJ_OK;
    }

    // Absolute iteration count at which rr is expected to reach tol2, from the
    // geometric rate of the last few iterations.
    static int predict(const Ctrl& c, int start) {
        const int t = c.iters;
        const int m = std::min(4, t - start);
        if (m <= 0 || !(c.rr > 0.0)) return t + FIRST_CHUNK;
        const double prev = c.hist[(t - m) % HIST];
        const double f = std::pow(c.rr / prev, 1.0 / m);
        if (!(f < 0.999) || !(f > 0.0)) return t + FIRST_CHUNK;
        const double more = std::ceil(std::log(c.tol2 / c.rr) / std::log(f));
        if (!(more >= 1.0)) return t + 1;
        return t + static_cast<int>(std::min(more, 200.0));
    }

    int epilogue(const double* s, int64_t lds, Ctrl* out) {
        int rc = with_graph(g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            k_epilogue<Vc><<<grid_win, WG, 0, st>>>(G, desc(), pl.K, x(), s, lds, r(), part(), ctrl());
            HIPCHK(hipGetLastError());
            return FJ_OK;
        });
        if (rc) return rc;
        k_fin_epilogue<<<1, WG, 0, st>>>(grid_win, g->n, part(), ctrl());
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&hs->h[NSLOT], ctrl(), sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::memcpy(out, &hs->h[NSLOT], sizeof(Ctrl));
        return FJ_OK;
    }

    int profile_total(fj_info* info) {
        if (!profile || !info) return FJ_OK;
        double tot = 0.0;
        for (size_t i = 0; i < n_prof; ++i) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, hs->prof[2 * i], hs->prof[2 * i + 1]));
            tot += ms;
        }
        info->ms_spmv = tot;
        info->n_spmv = static_cast<int32_t>(n_prof);
        return FJ_OK;
    }
};

// Smallest residual norm for which every index still meets eps/2, from the
// current index values (inverse of the certificate in k_epilogue).
double needed_rho(const Ctrl& c, double eps) {
    double need = INFINITY;
    const double scale[4] = {1.0, 2.0, 1.0, 1.0};  // D's error is bounded by rho / 2
    for (int i = 0; i < 4; ++i) {
        const double x = c.res[i];
        if (x > 0.0) need = std::min(need, scale[i] * 0.25 * eps * std::sqrt(x));
    }
    if (c.res[4] > 0.0 && c.res[3] > 0.0) need = std::min(need, 0.5 * eps * c.res[4] / std::sqrt(c.res[3]));
    return need;
}

// FP64 single right-hand side: PCG passes until certified (indices) or until
// the true relative residual meets rtol (solve).
int solve_fp64(Solver& S, const double* s, int64_t lds, const fj_opts& o, bool want_indices,
               fj_indices_t* out, fj_info* info) {
    const int max_iter = o.max_iter > 0 ? o.max_iter : 2000;
    double rtol = o.rtol > 0.0 ? o.rtol : o.eps * 1e-2;
    const bool range_check = !(o.flags & FJ_NO_RANGE_CHECK);
    Ctrl c{};
    int passes = 0;
    int status = FJ_OK;
    double prev_rho = INFINITY;
    if (int rc = S.init(s, lds, 0, rtol, max_iter, range_check)) return rc;
    for (;;) {
        ++passes;
        if (int rc = S.run(passes == 1 ? 0 : c.iters, max_iter, &c)) return rc;
        if (c.done == BAD_INPUT || c.done == BREAKDOWN) {
            status = status_of(c.done);
            break;
        }
        if (int rc = S.epilogue(s, lds, &c)) return rc;
        const double snorm = c.res[6];
        const double rho = c.res[5];
        const double rel = snorm > 0.0 ? rho / snorm : 0.0;
        bool ok;
        if (want_indices) {
            ok = true;
            for (int i = 0; i < 5; ++i) ok = ok && (c.bound[i] <= o.eps);
        } else {
            ok = rel <= rtol;
        }
        if (ok) {
            status = FJ_OK;
            break;
        }
        if (c.done == ITER_CAP || c.iters >= max_iter) {
            status = FJ_ERR_NOT_CONVERGED;
            break;
        }
        if (passes >= MAX_PASSES || !(rho < 0.5 * prev_rho)) {
            // the residual no longer drops: an index is too close to zero
            bool any_inf = false;
            for (int i = 0; i < 5; ++i) any_inf = any_inf || !(c.bound[i] < INFINITY);
            status = (want_indices && any_inf) ? FJ_ERR_UNCERTIFIABLE : FJ_ERR_NOT_CONVERGED;
            break;
        }
        prev_rho = rho;
        double next = rtol * 0.1;
        if (want_indices && snorm > 0.0) next = std::min(next, 0.5 * needed_rho(c, o.eps) / snorm);
        rtol = std::max(next, 1e-16);
        if (int rc = S.init(s, lds, 1, rtol, max_iter, range_check)) return rc;
    }
    if (out) {
        out->internal_conflict = c.res[0];
        out->disagreement = c.res[1];
        out->polarization = c.res[2];
        out->controversy = c.res[3];
        out->dc_index = c.res[4];
    }
    if (info) {
        info->status = status;
        info->iters = c.iters;
        info->passes = passes;
        info->outer_iters = 0;
        info->rel_residual = c.res[6] > 0.0 ? c.res[5] / c.res[6] : 0.0;
        for (int i = 0; i < 5; ++i) info->bound[i] = c.bound[i];
        if (int rc = S.profile_total(info)) return rc;
    }
    return status;
}

int make_solver(const fj_csr* g, const void* plan, void* ws, size_t ws_bytes, int k, void* stream,
                const fj_opts* o, Solver* S) {
    if (!plan || !ws || !aligned(plan) || !aligned(ws)) return FJ_ERR_WORKSPACE;
    S->g = g;
    S->pl = plan_layout(g);
    S->plan = static_cast<const char*>(plan);
    S->wl = ws_layout(g, k);
    if (ws_bytes < S->wl.total) return FJ_ERR_WORKSPACE;
    S->ws = static_cast<char*>(ws);
    S->st = static_cast<hipStream_t>(stream);
    S->profile = (o->flags & FJ_PROFILE) != 0;
    if (int rc = host_slots(&S->hs)) return rc;
    return S->setup();
}

}  // namespace

// ==================================================================== C ABI

extern "C" {

void fj_default_opts(fj_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->eps = 1e-6;
    o->precision = FJ_FP64;
}

const char* fj_status_string(int status) {
    switch (status) {
        case FJ_OK: return "ok";
        case FJ_ERR_INVALID_ARG: return "invalid argument";
        case FJ_ERR_INVALID_GRAPH: return "graph violates the CSR contract";
        case FJ_ERR_OPINION_RANGE: return "opinion outside [0,1] or NaN";
        case FJ_ERR_WORKSPACE: return "plan or workspace too small or misaligned";
        case FJ_ERR_NOT_CONVERGED: return "not converged within max_iter";
        case FJ_ERR_BREAKDOWN: return "CG breakdown";
        case FJ_ERR_UNCERTIFIABLE: return "an index is too close to zero to certify a relative error";
        case FJ_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* fj_last_error(void) { return g_last_error; }

size_t fj_plan_bytes(const fj_csr* g) {
    if (check_graph_args(g)) return 0;
    return plan_layout(g).total;
}

size_t fj_workspace_bytes(const fj_csr* g, int32_t k, const fj_opts* opts) {
    (void)opts;
    if (check_graph_args(g) || k < 1) return 0;
    return ws_layout(g, k).total;
}

int fj_prepare(const fj_csr* g, const fj_opts* opts, void* plan, size_t plan_bytes, void* stream) {
    if (int rc = check_graph_args(g)) return rc;
    const PlanLayout pl = plan_layout(g);
    if (!plan || !aligned(plan) || plan_bytes < pl.total) return FJ_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* P = static_cast<char*>(plan);
    int* blk_row = reinterpret_cast<int*>(P + pl.blk_row);
    WinDesc* desc = reinterpret_cast<WinDesc*>(P + pl.desc);
    float* minv = reinterpret_cast<float*>(P + pl.minv);
    int* flags = reinterpret_cast<int*>(P + pl.flags);
    if (g->n == 0) return FJ_OK;
    if (opts && (opts->flags & FJ_VALIDATE_GRAPH)) {
        HIPCHK(hipMemsetAsync(flags, 0, sizeof(int), st));
        int rc = with_graph(g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            const int64_t units = (std::max<int64_t>(g->nnz, g->n + 1) + WG - 1) / WG;
            const int grid = static_cast<int>(std::min<int64_t>(units, 8192));
            k_validate<Vc><<<grid, WG, 0, st>>>(G, g->nnz, flags);
            HIPCHK(hipGetLastError());
            return FJ_OK;
        });
        if (rc) return rc;
        int h = 0;
        HIPCHK(hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (h != 0) {
            std::snprintf(g_last_error, sizeof g_last_error, "CSR contract violated (flags 0x%x)", h);
            return FJ_ERR_INVALID_GRAPH;
        }
    }
    {
        const int grid = static_cast<int>(std::min<int64_t>((pl.K + 1 + WG - 1) / WG, 4096));
        k_windows<<<grid, WG, 0, st>>>(g->n, g->row_ptr, pl.K, blk_row);
        HIPCHK(hipGetLastError());
        k_window_desc<<<grid, WG, 0, st>>>(g->n, g->row_ptr, pl.K, blk_row, desc);
        HIPCHK(hipGetLastError());
    }
    return with_graph(g, [&](auto G) -> int {
        using Vc = typename decltype(G)::value_type;
        int grid = 1;
        if (int rc = grid_for(k_diag<Vc>, pl.K, &grid)) return rc;
        k_diag<Vc><<<grid, WG, 0, st>>>(G, desc, pl.K, minv);
        HIPCHK(hipGetLastError());
        return FJ_OK;
    });
}

int fj_apply(const fj_csr* g, const void* plan, const double* x, double* y, void* stream) {
    if (int rc = check_graph_args(g)) return rc;
    if (!plan || !aligned(plan)) return FJ_ERR_WORKSPACE;
    if (g->n == 0) return FJ_OK;
    if (!x || !y || x == y) return FJ_ERR_INVALID_ARG;
    const PlanLayout pl = plan_layout(g);
    const WinDesc* desc = reinterpret_cast<const WinDesc*>(static_cast<const char*>(plan) + pl.desc);
    hipStream_t st = static_cast<hipStream_t>(stream);
    return with_graph(g, [&](auto G) -> int {
        using Vc = typename decltype(G)::value_type;
        int grid = 1;
        if (int rc = grid_for(k_apply<Vc>, pl.K, &grid)) return rc;
        k_apply<Vc><<<grid, WG, 0, st>>>(G, desc, pl.K, x, y);
        HIPCHK(hipGetLastError());
        return FJ_OK;
    });
}

int fj_solve(const fj_csr* g, const void* plan, int32_t k, const double* S, int64_t lds, double* Z,
             int64_t ldz, const fj_opts* opts, void* ws, size_t ws_bytes, void* stream, fj_info* info) {
    if (int rc = check_graph_args(g)) return rc;
    if (int rc = check_opts(opts)) return rc;
    if (k != 1 || lds < k || ldz < k || !S || !Z) return FJ_ERR_INVALID_ARG;
    if (g->n == 0) return FJ_OK;
    Solver sv{};
    if (int rc = make_solver(g, plan, ws, ws_bytes, k, stream, opts, &sv)) return rc;
    const int status = solve_fp64(sv, S, lds, *opts, false, nullptr, info);
    if (status == FJ_ERR_HIP || status == FJ_ERR_OPINION_RANGE) return status;
    HIPCHK(hipMemcpy2DAsync(Z, sizeof(double) * ldz, sv.x(), sizeof(double), sizeof(double), g->n,
                            hipMemcpyDeviceToDevice, sv.st));
    HIPCHK(hipStreamSynchronize(sv.st));
    return status;
}

int fj_indices(const fj_csr* g, const void* plan, int32_t k, const double* S, int64_t lds,
               const fj_opts* opts, void* ws, size_t ws_bytes, void* stream, fj_indices_t* out,
               fj_info* info) {
    if (int rc = check_graph_args(g)) return rc;
    if (int rc = check_opts(opts)) return rc;
    if (k != 1 || lds < k || !S || !out) return FJ_ERR_INVALID_ARG;
    if (g->n == 0) return FJ_ERR_INVALID_ARG;
    Solver sv{};
    if (int rc = make_solver(g, plan, ws, ws_bytes, k, stream, opts, &sv)) return rc;
    return solve_fp64(sv, S, lds, *opts, true, out, info);
}

}  // extern "C"
