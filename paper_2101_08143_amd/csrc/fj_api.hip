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
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <utility>
#include <vector>

#include "../../include/fj.h"
#include "fj_guard.hpp"
#include "fj_kernels.hpp"
#include "fj_batched.hpp"
#include "fj_blockcg.hpp"
#include "fj_multilevel.hpp"
#include "fj_phased.hpp"

using namespace fj;

// The aggregation hierarchy of FJ_MULTILEVEL (see fj_hierarchy_create): levels
// 0 .. levels-2 each with a coarser level, then the last level.
struct fj_hierarchy {
    int dev = 0;
    int n0 = 0;
    int64_t nnz0 = 0;
    int levels = 0;
    MlLevel lv[ML_MAXL];
    int n[ML_MAXL] = {};
    int64_t nnz[ML_MAXL] = {};
    int nL = 0;                        // the last level: nodes,
    const double* inv = nullptr;       // its dense inverse (row-major, nL x nL) or null,
    const double* ainvL = nullptr;     // its 1 / a
    double* rbuf[ML_MAXL] = {};        // right-hand side of level l >= 1
    double* xbuf[ML_MAXL] = {};        // V-cycle result of level l >= 1
    double* ybuf[ML_MAXL] = {};        // D^-1 times the right-hand side, every level
    const double* ainvs[ML_MAXL] = {}; // 1 / a, every level
    void* mem = nullptr;               // one device allocation holding all of it
};

namespace {

constexpr size_t ALIGN = 256;
constexpr int NSLOT = 4;
constexpr int FIRST_CHUNK = 6;
constexpr int MAX_PASSES = 5;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

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
    size_t mate;      // int[n]: partner in the heavy-edge matching, -1 if none
    size_t pc;        // float2[n]: coefficients of the 2x2 block preconditioner
    size_t prop;      // int[n], float[n]: matching scratch (proposals, their weights)
    size_t pw;
    size_t flags;     // int[64] scratch for validation
    PhasedPlan ph;    // the time-phased entry layout (fj_phased.hpp), when ph.s.ok
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
    L.mate = off;
    off = align_up(off + sizeof(int) * static_cast<size_t>(g->n));
    L.pc = off;
    off = align_up(off + sizeof(float2) * static_cast<size_t>(g->n));
    L.prop = off;
    off = align_up(off + sizeof(int) * static_cast<size_t>(g->n));
    L.pw = off;
    off = align_up(off + sizeof(float) * static_cast<size_t>(g->n));
    L.flags = off;
    off = align_up(off + sizeof(int) * 64);
    L.ph.s = phased_shape(g->n, g->nnz);
    if (L.ph.s.ok) {
        const PhasedShape& S = L.ph.s;
        const size_t vb = g->val_type == FJ_VAL_F64 ? 8 : g->val_type == FJ_VAL_F32 ? 4 : 0;
        L.ph.ps = off;
        off = align_up(off + sizeof(int) * static_cast<size_t>(S.W) * (S.P + 1));
        L.ph.rs = off;
        off = align_up(off + sizeof(int) * (static_cast<size_t>(S.W) + 1));
        L.ph.row = off;
        off = align_up(off + sizeof(int) * static_cast<size_t>(g->n));
        L.ph.deg = off;
        off = align_up(off + sizeof(double) * static_cast<size_t>(g->n));
        L.ph.key = off;
        off = align_up(off + sizeof(unsigned short) * static_cast<size_t>(S.nnzp));
        L.ph.col = off;
        off = align_up(off + sizeof(int) * static_cast<size_t>(S.nnzp));
        L.ph.val = off;
        off = align_up(off + vb * static_cast<size_t>(S.nnzp));
    }
    L.total = off;
    return L;
}

struct WsLayout {
    int kp;                     // columns per block (1, or a power of two 2..KMAX)
    size_t x, r, p, q;          // FP64 vectors (p, q only for FJ_FP64)
    size_t z, mq;               // one vector: M^{-1} r and M^{-1} q of the block preconditioner (FP64)
    size_t z32, mq32;           // the same for the FP32 inner solve of FJ_MIXED
    size_t x32, r32, p32, q32;  // FP32 vectors of the inner solve (FJ_MIXED only)
    size_t sblk;                // FJ_TWO_SOLVE: the block [s, s - mean(s)]
    size_t zb, gpart, gm, wm, cm, zmean;  // FJ_BLOCK_CG: Z block, Gram partials, KB x KB matrices, column data
    size_t part, ctrl, total;   // partial sums; control blocks (outer kp, inner kp)
};

int padded_columns(int k) {
    int kp = 2;
    while (kp < k) kp *= 2;
    return kp;
}

// Columns handled by one batched solve: a single right-hand side runs alone
// (kp = 1) unless Algorithm 1 is asked for literally (two columns); more than
// KMAX columns are solved KMAX at a time. Block CG works on blocks of at
// least 16 columns (its KB x KB products use 16 x 16 matrix-core tiles).
int block_columns(int k, uint32_t flags) {
    if (flags & FJ_BLOCK_CG) return std::max(16, padded_columns(std::min(k, KMAX)));
    if (k == 1) return (flags & FJ_TWO_SOLVE) ? 2 : 1;
    return padded_columns(std::min(k, KMAX));
}

WsLayout ws_layout(const fj_csr* g, int k, int precision, uint32_t flags) {
    WsLayout L{};
    L.kp = block_columns(k, flags);
    const size_t nk = static_cast<size_t>(g->n) * static_cast<size_t>(L.kp);
    const size_t v64 = align_up(sizeof(double) * nk);
    const size_t v32 = align_up(sizeof(float) * nk);
    const bool mixed = precision == FJ_MIXED;
    size_t off = 0;
    L.x = off; off += v64;
    L.r = off; off += v64;
    if (!mixed) {
        L.p = off; off += v64;
        L.q = off; off += v64;
        if (L.kp == 1) {
            L.z = off; off += v64;
            L.mq = off; off += v64;
        }
    } else {
        L.x32 = off; off += v32;
        L.r32 = off; off += v32;
        L.p32 = off; off += v32;
        L.q32 = off; off += v32;
        if (L.kp == 1) {
            L.z32 = off; off += v32;
            L.mq32 = off; off += v32;
        }
    }
    if (k == 1 && (flags & FJ_TWO_SOLVE)) {
        L.sblk = off;
        off += align_up(sizeof(double) * 2 * static_cast<size_t>(g->n));
    }
    if (flags & FJ_BLOCK_CG) {
        const size_t kk = static_cast<size_t>(L.kp) * L.kp;
        L.zb = off; off += v64;
        L.gpart = off; off += align_up(sizeof(double) * GRAM_G * 2 * kk);
        L.gm = off; off += align_up(sizeof(double) * 2 * kk);  // [P^T Q, P^T R], or Q^T Z
        L.wm = off; off += align_up(sizeof(double) * kk);      // W = (P^T Q)^+
        L.cm = off; off += align_up(sizeof(double) * (kk + 2 * L.kp));  // alpha or beta, then column totals
        L.zmean = off; off += align_up(sizeof(double) * 2 * L.kp);
    }
    L.part = off; off = align_up(off + sizeof(double) * GMAX * std::max(NPART, BPART * L.kp));
    L.ctrl = off; off = align_up(off + sizeof(Ctrl) * 2 * static_cast<size_t>(L.kp));
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
    Ctrl* h = nullptr;                 // pinned, NSLOT + 1 slots of KMAX control blocks
    hipEvent_t ev[NSLOT + 1] = {};
    std::vector<hipEvent_t> prof;      // FJ_PROFILE event pairs
    Ctrl* slot(int i) { return h + static_cast<size_t>(i) * KMAX; }
};

thread_local std::map<int, HostSlots> tl_slots;

int host_slots(HostSlots** out) {
    int dev = 0;
    if (int rc = current_device(&dev)) return rc;
    HostSlots& hs = tl_slots[dev];
    if (!hs.h) {
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hs.h), sizeof(Ctrl) * KMAX * (NSLOT + 1),
                             hipHostMallocDefault));
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
    if ((o->flags & FJ_BLOCK_CG) &&
        (o->precision != FJ_FP64 || (o->flags & (FJ_TWO_SOLVE | FJ_WARM_START)))) {
        std::snprintf(g_last_error, sizeof g_last_error,
                      "FJ_BLOCK_CG needs FJ_FP64 and neither FJ_TWO_SOLVE nor FJ_WARM_START");
        return FJ_ERR_INVALID_ARG;
    }
    if ((o->flags & FJ_MULTILEVEL) &&
        (o->precision != FJ_FP64 || !o->hierarchy || (o->flags & (FJ_DIAG_PRECOND | FJ_BLOCK_CG | FJ_TWO_SOLVE)))) {
        std::snprintf(g_last_error, sizeof g_last_error,
                      "FJ_MULTILEVEL needs FJ_FP64, a hierarchy and none of FJ_DIAG_PRECOND, FJ_BLOCK_CG, "
                      "FJ_TWO_SOLVE");
        return FJ_ERR_INVALID_ARG;
    }
    if ((o->flags & FJ_WINDOW_SPMV) && (o->flags & FJ_PHASED_SPMV)) {
        std::snprintf(g_last_error, sizeof g_last_error, "FJ_WINDOW_SPMV and FJ_PHASED_SPMV exclude each other");
        return FJ_ERR_INVALID_ARG;
    }
    if (!(o->eps > 0.0 && o->eps < 0.5)) return FJ_ERR_INVALID_ARG;
    if (!(o->rtol >= 0.0 && o->rtol < 1.0)) return FJ_ERR_INVALID_ARG;
    if (o->max_iter < 0 || o->reserved != 0) return FJ_ERR_INVALID_ARG;
    if (o->precision != FJ_FP64 && o->precision != FJ_MIXED) return FJ_ERR_INVALID_ARG;
    return FJ_OK;
}

// FJ_MULTILEVEL: one vector, and the hierarchy built for this graph on this device.
int check_ml(const fj_csr* g, int k, const fj_opts* o) {
    if (!(o->flags & FJ_MULTILEVEL)) return FJ_OK;
    const fj_hierarchy* h = o->hierarchy;
    int dev = 0;
    if (int rc = current_device(&dev)) return rc;
    if (k != 1 || h->n0 != g->n || h->nnz0 != g->nnz || h->dev != dev) {
        std::snprintf(g_last_error, sizeof g_last_error,
                      "FJ_MULTILEVEL needs k = 1 and the hierarchy of this graph on this device");
        return FJ_ERR_INVALID_ARG;
    }
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

// One CG state: vectors of type T, its control block, the shared partials.
template <typename T>
struct CgState {
    T *x, *r, *p, *q;
    Ctrl* ctrl;
    double* part;
    const double* s_est = nullptr;  // FP64 only: s (contiguous) for the on-device index estimates
    T* z = nullptr;                 // with the 2x2 block preconditioner: M^{-1} r, M^{-1} q
    T* mq = nullptr;
    bool pairs = false;
    const fj_hierarchy* ml = nullptr;  // FJ_MULTILEVEL (FP64): z = V-cycle(r) instead of the 2x2 blocks
};

// What every launch of a solve needs.
struct Ctx {
    const fj_csr* g;
    PlanLayout pl;
    const char* plan;
    hipStream_t st;
    HostSlots* hs;
    bool profile;
    bool use_ph = false;  // the one-vector SpMV runs on the time-phased layout
    size_t n_prof = 0;  // FJ_PROFILE event pairs used
    int grid_vec = 1;
    const WinDesc* desc() const { return reinterpret_cast<const WinDesc*>(plan + pl.desc); }
    const float* minv() const { return reinterpret_cast<const float*>(plan + pl.minv); }
    const int* mate() const { return reinterpret_cast<const int*>(plan + pl.mate); }
    const float2* pc() const { return reinterpret_cast<const float2*>(plan + pl.pc); }

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

template <typename T>
int cg_init(Ctx& c, CgState<T>& S, const double* s, int64_t lds, int mode, double rtol, int max_iter,
            bool range_check, double eps_stop = 0.0, int deflate = 0) {
    const int n = c.g->n;
    if (mode != 1) {
        k_ctrl_reset<<<1, WG, 0, c.st>>>(S.ctrl, 1);
        HIPCHK(hipGetLastError());
    }
    k_cg_init<T><<<c.grid_vec, WG, 0, c.st>>>(n, s, lds, S.x, S.r, S.p, c.minv(), mode, S.part);
    HIPCHK(hipGetLastError());
    k_fin_init<<<1, WG, 0, c.st>>>(c.grid_vec, n, S.part, mode, rtol * rtol, max_iter, range_check ? 1 : 0,
                                   S.ctrl, eps_stop, deflate);
    HIPCHK(hipGetLastError());
    return FJ_OK;
}

// x = V b: one V-cycle of the hierarchy (see fj_multilevel.hpp). With ctrl,
// every launch returns at once once the solve has stopped.
int vcycle(hipStream_t st, const fj_hierarchy* h, const double* b, double* x, const Ctrl* ctrl) {
    auto rows_grid = [](auto kern, int n, int nlong, int* grid) -> int {
        const int64_t units = (static_cast<int64_t>(n) * ML_GW + static_cast<int64_t>(nlong) * 64 + WG - 1) / WG;
        return grid_for(kern, std::max<int64_t>(units, 1), grid);
    };
    int grid = 1;
    const double* bl = b;
    if (h->levels > 1) {
        if (int rc = grid_for(k_ml_scale, (static_cast<int64_t>(h->n0) + WG - 1) / WG, &grid)) return rc;
        k_ml_scale<<<grid, WG, 0, st>>>(h->n0, b, h->ainvs[0], h->ybuf[0], ctrl);
        HIPCHK(hipGetLastError());
    }
    for (int l = 0; l + 1 < h->levels; ++l) {
        const MlLevel& L = h->lv[l];
        if (int rc = rows_grid(k_ml_rows<OpPre>, L.n, L.nlong, &grid)) return rc;
        k_ml_rows<OpPre><<<grid, WG, 0, st>>>(L.n, L.rp, L.col, L.w, L.longs, L.nlong,
                                              OpPre{bl, h->ybuf[l], L.t}, ctrl);
        HIPCHK(hipGetLastError());
        if (int rc = rows_grid(k_ml_rows<OpSum>, L.nc, L.nclong, &grid)) return rc;
        k_ml_rows<OpSum><<<grid, WG, 0, st>>>(L.nc, L.mrp, L.mem, nullptr, L.clongs, L.nclong,
                                              OpSum{L.t, h->ainvs[l + 1], h->rbuf[l + 1], h->ybuf[l + 1]}, ctrl);
        HIPCHK(hipGetLastError());
        bl = h->rbuf[l + 1];
    }
    const int last = h->levels - 1;
    double* xl = last == 0 ? x : h->xbuf[last];
    if (h->inv) {
        if (int rc = grid_for(k_ml_coarse, (static_cast<int64_t>(h->nL) * 64 + WG - 1) / WG, &grid)) return rc;
    } else {
        if (int rc = grid_for(k_ml_coarse, (static_cast<int64_t>(h->nL) + WG - 1) / WG, &grid)) return rc;
    }
    k_ml_coarse<<<grid, WG, 0, st>>>(h->nL, h->inv, h->ainvL, bl, xl, ctrl);
    HIPCHK(hipGetLastError());
    for (int l = last - 1; l >= 0; --l) {
        const MlLevel& L = h->lv[l];
        const double* b_l = l == 0 ? b : h->rbuf[l];
        double* out = l == 0 ? x : h->xbuf[l];
        if (int rc = grid_for(k_ml_prolong, (static_cast<int64_t>(L.n) + WG - 1) / WG, &grid)) return rc;
        k_ml_prolong<<<grid, WG, 0, st>>>(L.n, h->ybuf[l], L.agg, h->xbuf[l + 1], L.t, ctrl);
        HIPCHK(hipGetLastError());
        if (int rc = rows_grid(k_ml_rows<OpPost>, L.n, L.nlong, &grid)) return rc;
        k_ml_rows<OpPost><<<grid, WG, 0, st>>>(L.n, L.rp, L.col, L.w, L.longs, L.nlong,
                                               OpPost{b_l, L.t, L.a, L.ainv, out}, ctrl);
        HIPCHK(hipGetLastError());
    }
    return FJ_OK;
}

// One CG step with the 2x2 block preconditioner or the V-cycle (one vector).
template <typename T>
int cg_iteration_pair(Ctx& c, CgState<T>& S) {
    int grid_win = 1;
    int rc = with_graph(c.g, [&](auto G) -> int {
        using Vc = typename decltype(G)::value_type;
        const bool lng = c.pl.ph.s.rmax == PH_RMAX_LONG;
        const int64_t chunk_waves = (c.pl.ph.s.W + NWAVE - 1) / NWAVE;
        if (c.use_ph) {
            if (int e = lng ? grid_for(k_cg_spmv_pq_ph<Vc, T, PH_RMAX_LONG>, chunk_waves, &grid_win)
                            : grid_for(k_cg_spmv_pq_ph<Vc, T, PH_RMAX_SHORT>, chunk_waves, &grid_win))
                return e;
        } else {
            if (int e = grid_for(k_cg_spmv_pq<Vc, T>, c.pl.K, &grid_win)) return e;
        }
        if (c.profile) {
            if (int e = profile_events(*c.hs, c.n_prof + 1)) return e;
            HIPCHK(hipEventRecord(c.hs->prof[2 * c.n_prof], c.st));
        }
        if (c.use_ph && lng)
            k_cg_spmv_pq_ph<Vc, T, PH_RMAX_LONG><<<grid_win, WG, 0, c.st>>>(phased_view<Vc>(c.plan, c.pl.ph), S.p,
                                                                            S.q, S.part, S.ctrl);
        else if (c.use_ph)
            k_cg_spmv_pq_ph<Vc, T, PH_RMAX_SHORT><<<grid_win, WG, 0, c.st>>>(phased_view<Vc>(c.plan, c.pl.ph), S.p,
                                                                             S.q, S.part, S.ctrl);
        else
            k_cg_spmv_pq<Vc, T><<<grid_win, WG, 0, c.st>>>(G, c.desc(), c.pl.K, S.p, S.q, S.part, S.ctrl);
        HIPCHK(hipGetLastError());
        if (c.profile) {
            HIPCHK(hipEventRecord(c.hs->prof[2 * c.n_prof + 1], c.st));
            ++c.n_prof;
        }
        return FJ_OK;
    });
    if (rc) return rc;
    const int n = c.g->n;
    if constexpr (std::is_same<T, double>::value) {
        if (S.ml) {
            if (int e = vcycle(c.st, S.ml, S.q, S.mq, S.ctrl)) return e;
            k_ml_dots<<<c.grid_vec, WG, 0, c.st>>>(n, S.q, S.z, S.mq, S.part, S.ctrl);
        } else {
            k_pair_dots<T><<<c.grid_vec, WG, 0, c.st>>>(n, S.q, S.z, c.mate(), c.pc(), S.mq, S.part, S.ctrl);
        }
    } else {
        k_pair_dots<T><<<c.grid_vec, WG, 0, c.st>>>(n, S.q, S.z, c.mate(), c.pc(), S.mq, S.part, S.ctrl);
    }
    HIPCHK(hipGetLastError());
    k_fin_pair<<<1, WG, 0, c.st>>>(grid_win, c.grid_vec, S.part, S.ctrl);
    HIPCHK(hipGetLastError());
    bool est = false;
    if constexpr (std::is_same<T, double>::value) est = S.s_est != nullptr;
    if (est) {
        if constexpr (std::is_same<T, double>::value) {
            k_cg_update_pair<T, true><<<c.grid_vec, WG, 0, c.st>>>(n, S.x, S.r, S.p, S.q, S.z, S.mq, S.s_est, S.part,
                                                                  S.ctrl);
            HIPCHK(hipGetLastError());
            k_fin_update<true><<<1, WG, 0, c.st>>>(c.grid_vec, n, S.part, S.ctrl);
        }
    } else {
        k_cg_update_pair<T, false><<<c.grid_vec, WG, 0, c.st>>>(n, S.x, S.r, S.p, S.q, S.z, S.mq, nullptr, S.part,
                                                                 S.ctrl);
        HIPCHK(hipGetLastError());
        k_fin_update<false><<<1, WG, 0, c.st>>>(c.grid_vec, n, S.part, S.ctrl);
    }
    HIPCHK(hipGetLastError());
    return FJ_OK;
}

template <typename T>
int cg_iteration(Ctx& c, CgState<T>& S) {
    if (S.pairs || S.ml) return cg_iteration_pair(c, S);
    int grid_win = 1;
    int rc = with_graph(c.g, [&](auto G) -> int {
        using Vc = typename decltype(G)::value_type;
        const bool lng = c.pl.ph.s.rmax == PH_RMAX_LONG;
        const int64_t chunk_waves = (c.pl.ph.s.W + NWAVE - 1) / NWAVE;
        if (c.use_ph) {
            if (int e = lng ? grid_for(k_cg_spmv_ph<Vc, T, PH_RMAX_LONG>, chunk_waves, &grid_win)
                            : grid_for(k_cg_spmv_ph<Vc, T, PH_RMAX_SHORT>, chunk_waves, &grid_win))
                return e;
        } else {
            if (int e = grid_for(k_cg_spmv<Vc, T>, c.pl.K, &grid_win)) return e;
        }
        if (c.profile) {
            if (int e = profile_events(*c.hs, c.n_prof + 1)) return e;
            HIPCHK(hipEventRecord(c.hs->prof[2 * c.n_prof], c.st));
        }
        if (c.use_ph && lng)
            k_cg_spmv_ph<Vc, T, PH_RMAX_LONG><<<grid_win, WG, 0, c.st>>>(phased_view<Vc>(c.plan, c.pl.ph), S.p, S.r,
                                                                         c.minv(), S.q, S.part, S.ctrl);
        else if (c.use_ph)
            k_cg_spmv_ph<Vc, T, PH_RMAX_SHORT><<<grid_win, WG, 0, c.st>>>(phased_view<Vc>(c.plan, c.pl.ph), S.p, S.r,
                                                                          c.minv(), S.q, S.part, S.ctrl);
        else
            k_cg_spmv<Vc, T><<<grid_win, WG, 0, c.st>>>(G, c.desc(), c.pl.K, S.p, S.r, c.minv(), S.q, S.part,
                                                        S.ctrl);
        HIPCHK(hipGetLastError());
        if (c.profile) {
            HIPCHK(hipEventRecord(c.hs->prof[2 * c.n_prof + 1], c.st));
            ++c.n_prof;
        }
        return FJ_OK;
    });
    if (rc) return rc;
    k_fin_spmv<<<1, WG, 0, c.st>>>(grid_win, S.part, S.ctrl);
    HIPCHK(hipGetLastError());
    bool est = false;
    if constexpr (std::is_same<T, double>::value) est = S.s_est != nullptr;
    if (est) {
        if constexpr (std::is_same<T, double>::value) {
            k_cg_update<T, true><<<c.grid_vec, WG, 0, c.st>>>(c.g->n, S.x, S.r, S.p, S.q, c.minv(), S.s_est, S.part,
                                                             S.ctrl);
            HIPCHK(hipGetLastError());
            k_fin_update<true><<<1, WG, 0, c.st>>>(c.grid_vec, c.g->n, S.part, S.ctrl);
            HIPCHK(hipGetLastError());
        }
    } else {
        k_cg_update<T, false><<<c.grid_vec, WG, 0, c.st>>>(c.g->n, S.x, S.r, S.p, S.q, c.minv(), nullptr, S.part,
                                                          S.ctrl);
        HIPCHK(hipGetLastError());
        k_fin_update<false><<<1, WG, 0, c.st>>>(c.grid_vec, c.g->n, S.part, S.ctrl);
        HIPCHK(hipGetLastError());
    }
    return FJ_OK;
}

// Chunks of iterations in flight, each with its control-block slot. A
// completed chunk queues at most one more, so at most two are pending; the
// ring holds NSLOT (no host allocation on the solve path).
struct Pending {
    int q[NSLOT] = {};
    int head = 0, count = 0;
    bool empty() const { return count == 0; }
    int front() const { return q[head]; }
    int back() const { return q[(head + count - 1) % NSLOT]; }
    void pop_front() {
        head = (head + 1) % NSLOT;
        --count;
    }
    bool push_back(int v) {
        if (count == NSLOT) return false;
        q[(head + count) % NSLOT] = v;
        ++count;
        return true;
    }
};

// Absolute iteration count at which rr is expected to reach tol2, from the
// geometric rate of the last few iterations.
int predict(const Ctrl& c, int start) {
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

// Run CG until its control block says done. `start` = iterations already done
// before this pass. Leaves the final control block in *out.
template <typename T>
int cg_run(Ctx& c, CgState<T>& S, int start, int max_iter, Ctrl* out) {
    int queued = start;
    int slot_next = 0;
    Pending pending;
    auto enqueue = [&](int cnt) -> int {
        for (int t = 0; t < cnt; ++t)
            if (int rc = cg_iteration(c, S)) return rc;
        queued += cnt;
        const int sl = slot_next++ % NSLOT;
        HIPCHK(hipMemcpyAsync(c.hs->slot(sl), S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipEventRecord(c.hs->ev[sl], c.st));
        if (!pending.push_back(sl)) return FJ_ERR_INTERNAL;
        return FJ_OK;
    };
    for (int k = 0; k < 2 && queued < max_iter; ++k)
        if (int rc = enqueue(std::min(FIRST_CHUNK, max_iter - queued))) return rc;
    while (!pending.empty()) {
        const int sl = pending.front();
        pending.pop_front();
        HIPCHK(hipEventSynchronize(c.hs->ev[sl]));
        const Ctrl& cc = *c.hs->slot(sl);
        if (cc.done != RUNNING || cc.iters >= max_iter) {
            std::memcpy(out, &cc, sizeof(Ctrl));
            // later chunks are empty launches; let them drain before returning
            HIPCHK(hipStreamSynchronize(c.st));
            if (!pending.empty()) std::memcpy(out, c.hs->slot(pending.back()), sizeof(Ctrl));
            return FJ_OK;
        }
        const int need = std::min(predict(cc, start), max_iter);
        if (need > queued) {
            if (int rc = enqueue(need - queued)) return rc;
        } else if (pending.empty() && queued < max_iter) {
            if (int rc = enqueue(1)) return rc;
        }
    }
    HIPCHK(hipMemcpyAsync(out, S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    return FJ_OK;
}

// Epilogue at z = S.x: residual into S.r, indices and bounds into S.ctrl;
// synchronises and copies the control block to *out.
int epilogue(Ctx& c, CgState<double>& S, const double* s, int64_t lds, Ctrl* out) {
    int grid_win = 1;
    int rc = with_graph(c.g, [&](auto G) -> int {
        using Vc = typename decltype(G)::value_type;
        if (int e = grid_for(k_epilogue<Vc>, c.pl.K, &grid_win)) return e;
        k_epilogue<Vc><<<grid_win, WG, 0, c.st>>>(G, c.desc(), c.pl.K, S.x, s, lds, S.r, S.part, S.ctrl);
        HIPCHK(hipGetLastError());
        return FJ_OK;
    });
    if (rc) return rc;
    k_fin_epilogue<<<1, WG, 0, c.st>>>(grid_win, c.g->n, S.part, S.ctrl);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c.hs->slot(NSLOT), S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    std::memcpy(out, c.hs->slot(NSLOT), sizeof(Ctrl));
    return FJ_OK;
}

// Smallest residual norm for which every index still meets eps/2, from the
// current index values (inverse of the certificate in k_fin_epilogue).
constexpr unsigned ALL_INDICES = 0x1Fu;

double needed_rho(const Ctrl& c, double eps, unsigned which = ALL_INDICES) {
    double need = INFINITY;
    const double scale[4] = {1.0, 2.0, 1.0, 1.0};  // D's error is bounded by rho / 2
    for (int i = 0; i < 4; ++i) {
        const double x = c.res[i];
        if (((which >> i) & 1u) && x > 0.0) need = std::min(need, scale[i] * 0.25 * eps * std::sqrt(x));
    }
    if ((which & 16u) && c.res[4] > 0.0 && c.res[3] > 0.0)
        need = std::min(need, 0.5 * eps * c.res[4] / std::sqrt(c.res[3]));
    return need;
}

bool certified(const Ctrl& c, double eps, unsigned which = ALL_INDICES) {
    for (int i = 0; i < 5; ++i)
        if (((which >> i) & 1u) && !(c.bound[i] <= eps)) return false;
    return true;
}

int stalled_status(const Ctrl& c, bool want_indices, unsigned which = ALL_INDICES) {
    bool any_inf = false;
    for (int i = 0; i < 5; ++i) any_inf = any_inf || (((which >> i) & 1u) && !(c.bound[i] < INFINITY));
    return (want_indices && any_inf) ? FJ_ERR_UNCERTIFIABLE : FJ_ERR_NOT_CONVERGED;
}

// Absolute error bound of each index from the same certificate as the
// relative bounds: |sqrt(X) - sqrt(X~)| <= rho_X gives
// |X - X~| <= rho_X (2 sqrt(X~) + rho_X), and |s^T e| <= (||z~|| + rho) rho;
// finite even where X~ is too close to 0 for a relative bound.
void abs_bounds(const Ctrl& c, double* ab) {
    const double rho = c.res[5];
    const double rh[4] = {rho, 0.5 * rho, rho, rho};
    for (int i = 0; i < 4; ++i) {
        const double rx = std::sqrt(std::max(c.res[i], 0.0));
        ab[i] = rh[i] * (2.0 * rx + rh[i]) + 1e-13 * std::fabs(c.res[i]);
    }
    ab[4] = (std::sqrt(std::max(c.res[3], 0.0)) + rho) * rho + 1e-13 * std::fabs(c.res[4]);
}

void fill_outputs(const Ctrl& c, int status, int passes, int outer, fj_indices_t* out, fj_info* info) {
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
        info->outer_iters = outer;
        info->rel_residual = c.res[6] > 0.0 ? c.res[5] / c.res[6] : 0.0;
        info->residual_norm = c.res[5];
        for (int i = 0; i < 5; ++i) info->bound[i] = c.bound[i];
        abs_bounds(c, info->abs_bound);
    }
}

// FP64: PCG passes until certified (indices) or until the true relative
// residual meets rtol (solve); each further pass restarts from the true
// residual with a tighter target.
// Warm start: z = z0 (device, stride ldz), then the true residual and the
// certificate of z0 itself; CG runs only if z0 does not already meet the
// target. Returns 1 in *done when z0 is accepted as it is.
int warm_start(Ctx& c, CgState<double>& S, const double* s, int64_t lds, const double* z0, int64_t ldz, Ctrl* cc) {
    HIPCHK(hipMemcpy2DAsync(S.x, sizeof(double), z0, sizeof(double) * ldz, sizeof(double), c.g->n,
                            hipMemcpyDeviceToDevice, c.st));
    return epilogue(c, S, s, lds, cc);
}

int solve_fp64(Ctx& c, CgState<double>& S, const double* s, int64_t lds, const fj_opts& o, bool want_indices,
               fj_indices_t* out, fj_info* info, const double* z0 = nullptr, int64_t ldz = 0) {
    const int max_iter = o.max_iter > 0 ? o.max_iter : 2000;
    double rtol = o.rtol > 0.0 ? o.rtol : o.eps * 1e-2;
    const bool range_check = !(o.flags & FJ_NO_RANGE_CHECK);
    Ctrl cc{};
    int passes = 0;
    int status = FJ_OK;
    double prev_rho = INFINITY;
    // Default target: also stop as soon as the on-device estimates of all five
    // indices at the current x meet 0.8 eps (the epilogue then certifies; the
    // estimates differ from the certified values only at the order of rho).
    const bool packable = lds == 1 && reinterpret_cast<uintptr_t>(s) % 16 == 0;  // read in 16-byte packs
    const double eps_stop = (want_indices && o.rtol == 0.0 && packable && !z0) ? 0.8 * o.eps : 0.0;
    S.s_est = eps_stop > 0.0 ? s : nullptr;
    if (int rc = cg_init(c, S, s, lds, 0, rtol, max_iter, range_check, eps_stop)) return rc;
    // deflated CG: move the start by mean(r) (from 0: to mean(s) 1) and keep
    // every step centred (k_cg_shift)
    const int deflate = (o.flags & FJ_ZERO_START) ? 0 : 1;
    auto shift_start = [&]() -> int {
        k_cg_shift<double><<<c.grid_vec, WG, 0, c.st>>>(c.g->n, S.x, S.r, S.p, c.minv(), S.ctrl, S.part);
        HIPCHK(hipGetLastError());
        k_fin_init<<<1, WG, 0, c.st>>>(c.grid_vec, c.g->n, S.part, 1, rtol * rtol, max_iter, range_check ? 1 : 0,
                                       S.ctrl, eps_stop, 1);
        HIPCHK(hipGetLastError());
        return FJ_OK;
    };
    // 2x2 block preconditioner on the plan's heavy-edge matching (default):
    // z = M^{-1} r and p = z replace the Jacobi start every start leaves
    // or the V-cycle of FJ_MULTILEVEL: z = V r, p = z
    S.ml = (o.flags & FJ_MULTILEVEL) && S.z != nullptr ? o.hierarchy : nullptr;
    S.pairs = !S.ml && S.z != nullptr && !(o.flags & FJ_DIAG_PRECOND) && c.g->n >= PAIR_MIN_N;
    auto pair_start = [&](double stop) -> int {
        if (!S.pairs && !S.ml) return FJ_OK;
        if (S.ml) {
            if (int rc = vcycle(c.st, S.ml, S.r, S.z, nullptr)) return rc;
            k_ml_start<<<c.grid_vec, WG, 0, c.st>>>(c.g->n, S.r, S.z, S.p, S.part);
        } else {
            k_pair_start<double><<<c.grid_vec, WG, 0, c.st>>>(c.g->n, S.r, S.z, S.p, c.mate(), c.pc(), S.part);
        }
        HIPCHK(hipGetLastError());
        k_fin_init<<<1, WG, 0, c.st>>>(c.grid_vec, c.g->n, S.part, 1, rtol * rtol, max_iter, range_check ? 1 : 0,
                                       S.ctrl, stop, deflate);
        HIPCHK(hipGetLastError());
        return FJ_OK;
    };
    if (deflate && !z0)
        if (int rc = shift_start()) return rc;
    if (!z0)
        if (int rc = pair_start(eps_stop)) return rc;
    if (z0) {
        if (int rc = warm_start(c, S, s, lds, z0, ldz, &cc)) return rc;
        const double snorm = cc.res[6], rho = cc.res[5];
        if (cc.done == BAD_INPUT) {
            status = FJ_ERR_OPINION_RANGE;
        } else if (want_indices ? certified(cc, o.eps) : (snorm == 0.0 || rho <= rtol * snorm)) {
            status = FJ_OK;
        } else {
            status = -1;  // iterate from z0
            prev_rho = rho;
            if (int rc = cg_init(c, S, s, lds, 1, rtol, max_iter, range_check)) return rc;
            if (deflate)
                if (int rc = shift_start()) return rc;
            if (int rc = pair_start(eps_stop)) return rc;
        }
        if (status >= 0) {
            cc.iters = 0;
            fill_outputs(cc, status, 0, 0, out, info);
            return status;
        }
        status = FJ_OK;
    }
    for (;;) {
        ++passes;
        if (int rc = cg_run(c, S, passes == 1 ? 0 : cc.iters, max_iter, &cc)) return rc;
        if (cc.done == BAD_INPUT || cc.done == BREAKDOWN) {
            status = status_of(cc.done);
            break;
        }
        if (int rc = epilogue(c, S, s, lds, &cc)) return rc;
        const double snorm = cc.res[6];
        const double rho = cc.res[5];
        const double rel = snorm > 0.0 ? rho / snorm : 0.0;
        if (want_indices ? certified(cc, o.eps) : rel <= rtol) {
            status = FJ_OK;
            break;
        }
        if (cc.done == ITER_CAP || cc.iters >= max_iter) {
            status = FJ_ERR_NOT_CONVERGED;
            break;
        }
        if (passes >= MAX_PASSES || !(rho < 0.5 * prev_rho)) {  // the residual no longer drops
            status = stalled_status(cc, want_indices);
            break;
        }
        prev_rho = rho;
        double next = rtol * 0.1;
        if (want_indices && snorm > 0.0) next = std::min(next, 0.5 * needed_rho(cc, o.eps) / snorm);
        rtol = std::max(next, 1e-16);
        S.s_est = nullptr;  // a restart runs to its residual target
        // (still deflated: x keeps mean(s), so the true residual is centred up to rounding)
        if (int rc = cg_init(c, S, s, lds, 1, rtol, max_iter, range_check, 0.0, deflate)) return rc;
        if (int rc = pair_start(0.0)) return rc;
    }
    fill_outputs(cc, status, passes, 0, out, info);
    if (info)
        if (int rc = c.profile_total(info)) return rc;
    return status;
}

// FJ_MIXED: FP64 residual-and-correction refinement around FP32 inner CG.
// Outer step: r32 = f32(r / ||r||); inner CG on (I+L) d = r32 to relative
// residual tau; z += ||r|| d in FP64; FP64 epilogue (true residual, indices,
// certificate). tau is chosen so that the next step should certify.
int solve_mixed(Ctx& c, CgState<double>& S, CgState<float>& I, const double* s, int64_t lds, const fj_opts& o,
                bool want_indices, fj_indices_t* out, fj_info* info, const double* z0 = nullptr, int64_t ldz = 0) {
    const int max_iter = o.max_iter > 0 ? o.max_iter : 2000;
    const double target = o.rtol > 0.0 ? o.rtol : o.eps * 1e-2;  // solve: relative residual to reach
    const bool range_check = !(o.flags & FJ_NO_RANGE_CHECK);
    const int n = c.g->n;
    Ctrl cc{}, ci{};
    // FP64 start: x = 0, r = s and the statistics of s (no CG iteration runs on it)
    if (int rc = cg_init(c, S, s, lds, 0, 1.0, max_iter, range_check)) return rc;
    HIPCHK(hipMemcpyAsync(&cc, S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    if (cc.done == BAD_INPUT) {
        fill_outputs(cc, FJ_ERR_OPINION_RANGE, 0, 0, out, info);
        return FJ_ERR_OPINION_RANGE;
    }
    const double snorm = std::sqrt(cc.ss);
    double rho = snorm;
    double tau = 1e-4;
    const bool deflate = !(o.flags & FJ_ZERO_START);
    I.pairs = I.z != nullptr && !(o.flags & FJ_DIAG_PRECOND) && n >= PAIR_MIN_N &&
              c.g->nnz >= static_cast<int64_t>(PAIR_MIN_DEGREE_FP32) * n;
    int inner_total = 0, outer = 0, status = FJ_ERR_NOT_CONVERGED;
    if (z0) {  // start the refinement from z0 and its true residual
        if (int rc = warm_start(c, S, s, lds, z0, ldz, &cc)) return rc;
        rho = cc.res[5];
        if (want_indices ? certified(cc, o.eps) : (snorm == 0.0 || rho <= target * snorm)) {
            cc.iters = 0;
            fill_outputs(cc, FJ_OK, 0, 0, out, info);
            return FJ_OK;
        }
        const double goal = want_indices ? needed_rho(cc, o.eps) : target * snorm;
        tau = std::min(1e-2, std::max(1e-5, 0.5 * goal / rho));
    }
    while (outer < 8 && inner_total < max_iter) {
        ++outer;
        const int mode = (outer == 1 && !z0) ? 0 : 1;
        k_mixed_cast<<<c.grid_vec, WG, 0, c.st>>>(n, S.r, I.r, mode, S.ctrl);
        HIPCHK(hipGetLastError());
        if (int rc = cg_init(c, I, nullptr, 0, 2, tau, max_iter - inner_total, false)) return rc;
        if (deflate) {  // inner CG from mean(r32) 1, deflated (see k_cg_shift)
            k_cg_shift<float><<<c.grid_vec, WG, 0, c.st>>>(n, I.x, I.r, I.p, c.minv(), I.ctrl, I.part);
            HIPCHK(hipGetLastError());
            k_fin_init<<<1, WG, 0, c.st>>>(c.grid_vec, n, I.part, 1, tau * tau, max_iter - inner_total, 0, I.ctrl,
                                           0.0, 1);
            HIPCHK(hipGetLastError());
        }
        if (I.pairs) {  // the 2x2 block preconditioner, as in the FP64 solve
            k_pair_start<float><<<c.grid_vec, WG, 0, c.st>>>(n, I.r, I.z, I.p, c.mate(), c.pc(), I.part);
            HIPCHK(hipGetLastError());
            k_fin_init<<<1, WG, 0, c.st>>>(c.grid_vec, n, I.part, 1, tau * tau, max_iter - inner_total, 0, I.ctrl,
                                           0.0, deflate ? 1 : 0);
            HIPCHK(hipGetLastError());
        }
        if (int rc = cg_run(c, I, 0, max_iter - inner_total, &ci)) return rc;
        inner_total += ci.iters;
        if (ci.done == BREAKDOWN) {
            status = FJ_ERR_BREAKDOWN;
            break;
        }
        k_mixed_refine<<<c.grid_vec, WG, 0, c.st>>>(n, S.x, I.x, mode, S.ctrl);
        HIPCHK(hipGetLastError());
        if (int rc = epilogue(c, S, s, lds, &cc)) return rc;
        const double new_rho = cc.res[5];
        const bool ok = want_indices ? certified(cc, o.eps) : (snorm == 0.0 || new_rho <= target * snorm);
        if (ok) {
            status = FJ_OK;
            break;
        }
        if (!(new_rho < 0.5 * rho)) {  // refinement no longer reduces the residual
            status = stalled_status(cc, want_indices);
            break;
        }
        rho = new_rho;
        const double goal = want_indices ? needed_rho(cc, o.eps) : target * snorm;
        tau = std::min(1e-2, std::max(1e-5, 0.5 * goal / rho));
    }
    cc.iters = inner_total;
    fill_outputs(cc, status, outer, outer, out, info);
    if (info)
        if (int rc = c.profile_total(info)) return rc;
    return status;
}

int make_ctx(const fj_csr* g, const void* plan, void* ws, size_t ws_bytes, int k, void* stream,
             const fj_opts* o, Ctx* c, WsLayout* wl, HostSlots* slots = nullptr) {
    if (!plan || !ws || !aligned(plan) || !aligned(ws)) return FJ_ERR_WORKSPACE;
    c->g = g;
    c->pl = plan_layout(g);
    c->plan = static_cast<const char*>(plan);
    *wl = ws_layout(g, k, o->precision, o->flags);
    if (ws_bytes < wl->total) return FJ_ERR_WORKSPACE;
    c->st = static_cast<hipStream_t>(stream);
    c->profile = (o->flags & FJ_PROFILE) != 0;
    c->use_ph = c->pl.ph.s.ok && ((o->flags & FJ_PHASED_SPMV) ||
                                  (g->n >= PH_MIN_N && !(o->flags & FJ_WINDOW_SPMV)));
    if (slots) c->hs = slots;
    else if (int rc = host_slots(&c->hs)) return rc;
    return grid_for(k_cg_update<double, true>, (static_cast<int64_t>(g->n) + 2 * WG - 1) / (2 * WG), &c->grid_vec);
}

// Single right-hand side, either precision. Z (may be null) receives z.
int solve_one(const fj_csr* g, const void* plan, const double* S, int64_t lds, double* Z, int64_t ldz,
              const fj_opts& o, void* ws, size_t ws_bytes, void* stream, bool want_indices, fj_indices_t* out,
              fj_info* info, HostSlots* slots = nullptr) {
    Ctx c{};
    WsLayout wl{};
    if (int rc = make_ctx(g, plan, ws, ws_bytes, 1, stream, &o, &c, &wl, slots)) return rc;
    char* W = static_cast<char*>(ws);
    Ctrl* ctrls = reinterpret_cast<Ctrl*>(W + wl.ctrl);
    double* part = reinterpret_cast<double*>(W + wl.part);
    const bool mixed = o.precision == FJ_MIXED;  // FP64 side of FJ_MIXED keeps only x and r
    const bool warm = Z && (o.flags & FJ_WARM_START);
    CgState<double> S64{reinterpret_cast<double*>(W + wl.x), reinterpret_cast<double*>(W + wl.r),
                        mixed ? nullptr : reinterpret_cast<double*>(W + wl.p),
                        mixed ? nullptr : reinterpret_cast<double*>(W + wl.q), &ctrls[0], part};
    if (!mixed) {
        S64.z = reinterpret_cast<double*>(W + wl.z);
        S64.mq = reinterpret_cast<double*>(W + wl.mq);
    }
    int status;
    if (o.precision == FJ_MIXED) {
        CgState<float> S32{reinterpret_cast<float*>(W + wl.x32), reinterpret_cast<float*>(W + wl.r32),
                           reinterpret_cast<float*>(W + wl.p32), reinterpret_cast<float*>(W + wl.q32), &ctrls[1],
                           part};
        S32.z = reinterpret_cast<float*>(W + wl.z32);
        S32.mq = reinterpret_cast<float*>(W + wl.mq32);
        status = solve_mixed(c, S64, S32, S, lds, o, want_indices, out, info, warm ? Z : nullptr, ldz);
    } else {
        status = solve_fp64(c, S64, S, lds, o, want_indices, out, info, warm ? Z : nullptr, ldz);
    }
    if (Z && status != FJ_ERR_HIP && status != FJ_ERR_OPINION_RANGE) {
        HIPCHK(hipMemcpy2DAsync(Z, sizeof(double) * ldz, S64.x, sizeof(double), sizeof(double), g->n,
                                hipMemcpyDeviceToDevice, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
    }
    return status;
}

// ---------------------------------------------------------------- SpMM tuner

// The batched SpMM has two launch parameters that trade lanes per row for
// rows in flight: CPL columns per lane (a row is owned by KB / CPL lanes, so
// a wave64 works on 64 * CPL / KB rows at once, each gather a CPL-wide vector
// load) and the persistent grid (every workgroup that fits, or half as many).
// The first batched solve of a (graph, KB, vector precision) on a device
// times each candidate on its own vectors and keeps the fastest for the life
// of the process; FJ_NO_TUNE pins CPL = 1 and the full grid. The row sums do
// not depend on the choice; the order in which the per-column dot products
// are added does (so two processes that tune differently may differ in the
// last bits, while every call within a process sees the same choice).
struct SpmmKey {
    int dev, kb, tbytes, vt, n;
    int64_t nnz;
    const void *rp, *col, *val;
    bool operator<(const SpmmKey& o) const {
        return std::tie(dev, kb, tbytes, vt, n, nnz, rp, col, val) <
               std::tie(o.dev, o.kb, o.tbytes, o.vt, o.n, o.nnz, o.rp, o.col, o.val);
    }
};
struct SpmmChoice {
    int cpl = 1, grid = 1;
    bool split = true;  // merge-path item split over lane groups, or one group per row
    int passes = 1;     // column passes (rows design): 2 or 4 for 32- and 64-column blocks
};

// A shape the SpMM can run: column passes need the rows design, a pass of at
// least 16 columns (2 or 4 of them) and CPL dividing the pass width.
bool spmm_shape_ok(int kb, int cpl, bool split, int passes) {
    if (cpl != 1 && cpl != 2 && cpl != 4) return false;
    if (passes == 1) return kb % cpl == 0;
    if (passes != 2 && passes != 4) return false;
    return !split && cpl <= 2 && kb / passes >= 16 && (kb / passes) % cpl == 0;
}
std::mutex g_tune_mu;
std::map<SpmmKey, SpmmChoice> g_tune;

int spmm_key(const fj_csr* g, int kb, int tbytes, SpmmKey* k) {
    int dev = 0;
    if (int rc = current_device(&dev)) return rc;
    *k = SpmmKey{dev, kb, tbytes, g->val_type, g->n, g->nnz, g->row_ptr, g->col_idx, g->val};
    return FJ_OK;
}

template <typename Vc, typename T, int KB>
struct Spmm {
    template <int CPL>
    static int grid_of(bool split, int K, int* grid) {
        return split ? grid_for(k_spmm_cg<Vc, T, KB, CPL, true>, K, grid)
                     : grid_for(k_spmm_cg<Vc, T, KB, CPL, false>, K, grid);
    }
    // grid of a column pass of KB / NP columns (rows design)
    template <int NP, int CPL>
    static int grid_pass(int K, int* grid) {
        if constexpr (NP > 1 && KB / NP >= 16 && (KB / NP) % CPL == 0)
            return grid_for(k_spmm_cg<Vc, T, KB / NP, CPL, false, KB>, K, grid);
        return FJ_ERR_INVALID_ARG;
    }
    static int full_grid(int cpl, bool split, int K, int* grid, int passes = 1) {
        if (passes == 2) return cpl == 2 ? grid_pass<2, 2>(K, grid) : grid_pass<2, 1>(K, grid);
        if (passes == 4) return cpl == 2 ? grid_pass<4, 2>(K, grid) : grid_pass<4, 1>(K, grid);
        if constexpr (KB % 4 == 0)
            if (cpl == 4) return grid_of<4>(split, K, grid);
        if constexpr (KB % 2 == 0)
            if (cpl == 2) return grid_of<2>(split, K, grid);
        return grid_of<1>(split, K, grid);
    }
    template <int CPL>
    static int go(const SpmmChoice& ch, hipStream_t st, const Csr<Vc>& G, const WinDesc* desc, int K,
                  const T* P, const T* R, const float* minv, T* Q, double* part, const Ctrl* ctrl) {
        if (ch.split) k_spmm_cg<Vc, T, KB, CPL, true><<<ch.grid, WG, 0, st>>>(G, desc, K, P, R, minv, Q, part, ctrl);
        else k_spmm_cg<Vc, T, KB, CPL, false><<<ch.grid, WG, 0, st>>>(G, desc, K, P, R, minv, Q, part, ctrl);
        HIPCHK(hipGetLastError());
        return FJ_OK;
    }
    // NP passes of KB / NP columns over the CSR (partials land in the KB-wide layout)
    template <int NP, int CPL>
    static int go_passes(const SpmmChoice& ch, hipStream_t st, const Csr<Vc>& G, const WinDesc* desc, int K,
                         const T* P, const T* R, const float* minv, T* Q, double* part, const Ctrl* ctrl) {
        if constexpr (NP > 1 && KB / NP >= 16 && (KB / NP) % CPL == 0) {
            constexpr int KP = KB / NP;
            for (int j = 0; j < NP; ++j) {
                k_spmm_cg<Vc, T, KP, CPL, false, KB><<<ch.grid, WG, 0, st>>>(G, desc, K, P, R, minv, Q, part, ctrl,
                                                                             j * KP);
                HIPCHK(hipGetLastError());
            }
            return FJ_OK;
        }
        return FJ_ERR_INVALID_ARG;
    }
    static int launch(const SpmmChoice& ch, hipStream_t st, const Csr<Vc>& G, const WinDesc* desc, int K,
                      const T* P, const T* R, const float* minv, T* Q, double* part, const Ctrl* ctrl) {
        if (ch.passes == 2)
            return ch.cpl == 2 ? go_passes<2, 2>(ch, st, G, desc, K, P, R, minv, Q, part, ctrl)
                               : go_passes<2, 1>(ch, st, G, desc, K, P, R, minv, Q, part, ctrl);
        if (ch.passes == 4)
            return ch.cpl == 2 ? go_passes<4, 2>(ch, st, G, desc, K, P, R, minv, Q, part, ctrl)
                               : go_passes<4, 1>(ch, st, G, desc, K, P, R, minv, Q, part, ctrl);
        if constexpr (KB % 4 == 0)
            if (ch.cpl == 4) return go<4>(ch, st, G, desc, K, P, R, minv, Q, part, ctrl);
        if constexpr (KB % 2 == 0)
            if (ch.cpl == 2) return go<2>(ch, st, G, desc, K, P, R, minv, Q, part, ctrl);
        return go<1>(ch, st, G, desc, K, P, R, minv, Q, part, ctrl);
    }
    // The launch shape for this graph: cached, or tuned now on the caller's
    // vectors (Q and part are overwritten; the next SpMM recomputes them).
    static int choose(const fj_csr* g, hipStream_t st, const Csr<Vc>& G, const WinDesc* desc, int K,
                      const T* P, const T* R, const float* minv, T* Q, double* part, bool tune,
                      SpmmChoice* out) {
        if (!tune) {
            out->cpl = 1;
            out->split = true;
            return full_grid(1, true, K, &out->grid);
        }
        SpmmKey key{};
        if (int rc = spmm_key(g, KB, static_cast<int>(sizeof(T)), &key)) return rc;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end()) {
                *out = it->second;
                return FJ_OK;
            }
        }
        std::vector<SpmmChoice> cand;
        for (bool split : {true, false}) {
            for (int cpl : {1, 2, 4}) {
                if (KB % cpl != 0) continue;
                if (!split && KB / cpl < 8) continue;  // a row per group of < 8 lanes serialises long rows
                int full = 1;
                if (int rc = full_grid(cpl, split, K, &full)) return rc;
                cand.push_back({cpl, full, split, 1});
                if (full >= 2) cand.push_back({cpl, full / 2, split, 1});
            }
        }
        // wide blocks: column passes keep each pass's gathered rows small
        for (int passes : {2, 4}) {
            for (int cpl : {1, 2}) {
                if (!spmm_shape_ok(KB, cpl, false, passes)) continue;
                int full = 1;
                if (int rc = full_grid(cpl, false, K, &full, passes)) return rc;
                cand.push_back({cpl, full, false, passes});
                if (full >= 2) cand.push_back({cpl, full / 2, false, passes});
            }
        }
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        constexpr int REPS = 3;
        float best = INFINITY;
        SpmmChoice pick = cand.front();
        int rc = FJ_OK;
        for (const SpmmChoice& ch : cand) {
            // timed on every column (no control blocks: no early exit, no shift)
            if ((rc = launch(ch, st, G, desc, K, P, R, minv, Q, part, nullptr))) break;  // warm-up
            if (hipEventRecord(e0, st) != hipSuccess) { rc = FJ_ERR_HIP; break; }
            for (int r = 0; r < REPS && rc == FJ_OK; ++r) rc = launch(ch, st, G, desc, K, P, R, minv, Q, part, nullptr);
            if (rc) break;
            float ms = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = FJ_ERR_HIP;
                break;
            }
            if (ms < best) {
                best = ms;
                pick = ch;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        *out = g_tune.emplace(key, pick).first->second;
        return FJ_OK;
    }
};

// ---------------------------------------------------------------- k columns

template <typename T>
struct BState {
    T *X, *R, *P, *Q;
    Ctrl* ctrl;  // KB control blocks
    double* part;
    const double* s_est = nullptr;  // FP64 only: the opinions (stride s_lds, s_k columns) for index estimates
    int64_t s_lds = 0;
    int s_k = 0;
};

// The batched driver for KB columns (see fj_batched.hpp).
template <int KB>
struct Batched {
    Ctx& c;
    bool tune = true;
    int grid_vec = 1;
    SpmmChoice ch64{1, 0}, ch32{1, 0};  // grid 0: not chosen yet
    // FJ_BLOCK_CG (FP64, KB >= 16): the shared-Krylov iteration and its buffers
    bool block = false;
    double *Zb = nullptr, *gpart = nullptr, *Gm = nullptr, *Wm = nullptr, *Cm = nullptr, *zmean = nullptr;
    int grid_mul = 1;
    static constexpr uint64_t ALL = KB >= 64 ? ~0ull : ((1ull << KB) - 1ull);

    int setup() {
        const int64_t units = (static_cast<int64_t>(c.g->n) * KB + WG - 1) / WG;
        return grid_for(k_update_batched<double, KB, true>, units, &grid_vec);
    }

    // deflate: start modes 0 and 2 from the column means and run deflated CG
    // (k_init_batched mode 3); a restart (mode 1) keeps it on.
    template <typename T>
    int init(BState<T>& S, const double* src, int64_t lds, int k, int kcheck, int mode, uint64_t mask,
             const double* rtol, int max_iter, bool range_check, double eps_stop = 0.0, bool deflate = false) {
        ColumnTol tol{};
        for (int col = 0; col < KB; ++col) tol.rtol2[col] = rtol[col] * rtol[col];
        const int n = c.g->n;
        if (mode != 1) {
            k_ctrl_reset<<<1, WG, 0, c.st>>>(S.ctrl, KB);
            HIPCHK(hipGetLastError());
        }
        const int rc_flag = range_check ? 1 : 0;
        k_init_batched<T, KB><<<grid_vec, WG, 0, c.st>>>(n, k, src, lds, S.X, S.R, S.P, c.minv(), mode, mask, kcheck,
                                                        S.part, S.ctrl);
        HIPCHK(hipGetLastError());
        k_fin_init_batched<KB><<<KB, WG, 0, c.st>>>(grid_vec, n, k, S.part, mode, mask, tol, max_iter, rc_flag,
                                                   S.ctrl, 1, eps_stop, (deflate && mode == 1) ? 1 : 0);
        HIPCHK(hipGetLastError());
        if (deflate && mode != 1) {
            k_init_batched<T, KB><<<grid_vec, WG, 0, c.st>>>(n, k, nullptr, 0, S.X, S.R, S.P, c.minv(), 3, mask, 0,
                                                            S.part, S.ctrl);
            HIPCHK(hipGetLastError());
            k_fin_init_batched<KB><<<KB, WG, 0, c.st>>>(grid_vec, n, k, S.part, 3, mask, tol, max_iter, rc_flag,
                                                       S.ctrl, 1, eps_stop, 1);
            HIPCHK(hipGetLastError());
        }
        return FJ_OK;
    }

    // One step of block CG (see fj_blockcg.hpp): Q = A P; W = (P^T Q)^+ and
    // alpha = W P^T R; X += P alpha, R -= Q alpha; Z = Pi M^-1 R; beta =
    // -W Q^T Z; P = (Z + P beta) D.
    int block_iteration(BState<double>& S) {
        if constexpr (KB >= 16) {
            const int n = c.g->n;
            int rc = with_graph(c.g, [&](auto G) -> int {
                using Vc = typename decltype(G)::value_type;
                if (ch64.grid == 0)
                    if (int e = Spmm<Vc, double, KB>::choose(c.g, c.st, G, c.desc(), c.pl.K, S.P, S.R, c.minv(), S.Q,
                                                             S.part, tune, &ch64))
                        return e;
                if (c.profile) {
                    if (int e = profile_events(*c.hs, c.n_prof + 1)) return e;
                    HIPCHK(hipEventRecord(c.hs->prof[2 * c.n_prof], c.st));
                }
                if (int e = Spmm<Vc, double, KB>::launch(ch64, c.st, G, c.desc(), c.pl.K, S.P, S.R, c.minv(), S.Q,
                                                         S.part, S.ctrl))
                    return e;
                if (c.profile) {
                    HIPCHK(hipEventRecord(c.hs->prof[2 * c.n_prof + 1], c.st));
                    ++c.n_prof;
                }
                return FJ_OK;
            });
            if (rc) return rc;
            constexpr int KK = KB * KB;
            // [P^T Q, P^T R] in one pass over P, Q, R
            k_gram<KB, 2><<<GRAM_G, WG, 0, c.st>>>(n, S.P, S.Q, S.R, gpart, S.ctrl);
            HIPCHK(hipGetLastError());
            k_gram_fin<<<2 * KK / 16, WG, 0, c.st>>>(GRAM_G, 2 * KK, gpart, 1.0, Gm, S.ctrl);
            HIPCHK(hipGetLastError());
            k_bcg_chol<KB><<<1, WG, 0, c.st>>>(Gm, Wm, Cm, S.ctrl);  // W and alpha (in Cm)
            HIPCHK(hipGetLastError());
            k_block_mul<KB><<<grid_mul, WG, 0, c.st>>>(n, S.P, Cm, 1.0, S.X, 1.0, nullptr, nullptr, S.X, S.ctrl);
            HIPCHK(hipGetLastError());
            k_block_mul<KB><<<grid_mul, WG, 0, c.st>>>(n, S.Q, Cm, -1.0, S.R, 1.0, nullptr, nullptr, S.R, S.ctrl);
            HIPCHK(hipGetLastError());
            if (int e = precondition(S, 0)) return e;
            k_gram<KB, 1><<<GRAM_G, WG, 0, c.st>>>(n, S.Q, Zb, nullptr, gpart, S.ctrl);
            HIPCHK(hipGetLastError());
            k_gram_fin<<<KK / 16, WG, 0, c.st>>>(GRAM_G, KK, gpart, 1.0, Gm, S.ctrl);
            HIPCHK(hipGetLastError());
            k_small_mul<KB><<<1, WG, 0, c.st>>>(Wm, Gm, -1.0, Cm, S.ctrl);  // beta
            HIPCHK(hipGetLastError());
            k_block_mul<KB><<<grid_mul, WG, 0, c.st>>>(n, S.P, Cm, 1.0, Zb, 1.0, zmean, zmean + KB, S.P, S.ctrl);
            HIPCHK(hipGetLastError());
        }
        return FJ_OK;
    }

    // Z = M^-1 R, its column means and the residual norms; the block's
    // stopping test (first = 1: a start, the iteration count stays).
    int precondition(BState<double>& S, int first) {
        if constexpr (KB >= 16) {
            const int n = c.g->n;
            k_bcg_precond<KB><<<grid_vec, WG, 0, c.st>>>(n, S.R, c.minv(), Zb, S.part, S.ctrl);
            HIPCHK(hipGetLastError());
            k_bcg_colsum<KB><<<KB, WG, 0, c.st>>>(grid_vec, S.part, Cm + KB * KB, S.ctrl);
            HIPCHK(hipGetLastError());
            k_bcg_decide<KB><<<1, 64, 0, c.st>>>(n, Cm + KB * KB, first, zmean, S.ctrl);
            HIPCHK(hipGetLastError());
        }
        return FJ_OK;
    }

    // The first search block of a block CG pass: Z = Pi M^-1 R and P = Z D.
    int block_start(BState<double>& S) {
        if constexpr (KB >= 16) {
            k_bcg_start<KB><<<1, 64, 0, c.st>>>(S.ctrl);
            HIPCHK(hipGetLastError());
            if (int e = precondition(S, 1)) return e;
            k_block_mul<KB><<<grid_mul, WG, 0, c.st>>>(c.g->n, nullptr, Cm, 1.0, Zb, 1.0, zmean, zmean + KB, S.P,
                                                      S.ctrl);
            HIPCHK(hipGetLastError());
        }
        return FJ_OK;
    }

    template <typename T>
    int iteration(BState<T>& S) {
        if constexpr (std::is_same<T, double>::value)
            if (block) return block_iteration(S);
        int grid_win = 1;
        int rc = with_graph(c.g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            SpmmChoice& ch = sizeof(T) == sizeof(double) ? ch64 : ch32;
            if (ch.grid == 0)
                if (int e = Spmm<Vc, T, KB>::choose(c.g, c.st, G, c.desc(), c.pl.K, S.P, S.R, c.minv(), S.Q, S.part,
                                                    tune, &ch))
                    return e;
            grid_win = ch.grid;
            if (c.profile) {
                if (int e = profile_events(*c.hs, c.n_prof + 1)) return e;
                HIPCHK(hipEventRecord(c.hs->prof[2 * c.n_prof], c.st));
            }
            if (int e = Spmm<Vc, T, KB>::launch(ch, c.st, G, c.desc(), c.pl.K, S.P, S.R, c.minv(), S.Q, S.part,
                                                S.ctrl))
                return e;
            if (c.profile) {
                HIPCHK(hipEventRecord(c.hs->prof[2 * c.n_prof + 1], c.st));
                ++c.n_prof;
            }
            return FJ_OK;
        });
        if (rc) return rc;
        k_fin_spmm<KB><<<KB, WG, 0, c.st>>>(grid_win, S.part, S.ctrl);
        HIPCHK(hipGetLastError());
        bool est = false;
        if constexpr (std::is_same<T, double>::value) est = S.s_est != nullptr;
        if (est) {
            if constexpr (std::is_same<T, double>::value) {
                k_update_batched<T, KB, true><<<grid_vec, WG, 0, c.st>>>(c.g->n, S.X, S.R, S.P, S.Q, c.minv(), S.s_est,
                                                                       S.s_lds, S.s_k, S.part, S.ctrl);
                HIPCHK(hipGetLastError());
                k_fin_update_batched<KB, true><<<KB, WG, 0, c.st>>>(grid_vec, c.g->n, S.part, S.ctrl);
                HIPCHK(hipGetLastError());
            }
        } else {
            k_update_batched<T, KB, false><<<grid_vec, WG, 0, c.st>>>(c.g->n, S.X, S.R, S.P, S.Q, c.minv(), nullptr,
                                                                    0, 0, S.part, S.ctrl);
            HIPCHK(hipGetLastError());
            k_fin_update_batched<KB, false><<<KB, WG, 0, c.st>>>(grid_vec, c.g->n, S.part, S.ctrl);
            HIPCHK(hipGetLastError());
        }
        return FJ_OK;
    }

    // Iterate until every column is done; out receives the KB control blocks.
    template <typename T>
    int run(BState<T>& S, int k, Ctrl* out) {
        HIPCHK(hipMemcpyAsync(c.hs->slot(NSLOT), S.ctrl, sizeof(Ctrl) * KB, hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        int start[KMAX];
        int budget = 0;  // launches the iteration caps still allow
        bool any = false;
        for (int col = 0; col < k; ++col) {
            const Ctrl& cc = c.hs->slot(NSLOT)[col];
            start[col] = cc.iters;
            if (cc.done == RUNNING) {
                any = true;
                budget = std::max(budget, cc.max_iter - cc.iters);
            }
        }
        if (!any) {
            std::memcpy(out, c.hs->slot(NSLOT), sizeof(Ctrl) * KB);
            return FJ_OK;
        }
        int queued = 0, slot_next = 0;
        Pending pending;
        auto enqueue = [&](int cnt) -> int {
            for (int t = 0; t < cnt; ++t)
                if (int rc = iteration(S)) return rc;
            queued += cnt;
            const int sl = slot_next++ % NSLOT;
            HIPCHK(hipMemcpyAsync(c.hs->slot(sl), S.ctrl, sizeof(Ctrl) * KB, hipMemcpyDeviceToHost, c.st));
            HIPCHK(hipEventRecord(c.hs->ev[sl], c.st));
            if (!pending.push_back(sl)) return FJ_ERR_INTERNAL;
            return FJ_OK;
        };
        for (int t = 0; t < 2 && queued < budget; ++t)
            if (int rc = enqueue(std::min(FIRST_CHUNK, budget - queued))) return rc;
        while (!pending.empty()) {
            const int sl = pending.front();
            pending.pop_front();
            HIPCHK(hipEventSynchronize(c.hs->ev[sl]));
            const Ctrl* cs = c.hs->slot(sl);
            int need = 0;
            bool running = false;
            for (int col = 0; col < k; ++col) {
                if (cs[col].done == RUNNING && cs[col].iters < cs[col].max_iter) {
                    running = true;
                    need = std::max(need, std::min(predict(cs[col], start[col]), cs[col].max_iter) - start[col]);
                }
            }
            if (!running || queued >= budget) {
                HIPCHK(hipStreamSynchronize(c.st));
                std::memcpy(out, c.hs->slot(pending.empty() ? sl : pending.back()), sizeof(Ctrl) * KB);
                return FJ_OK;
            }
            need = std::min(need, budget);
            if (need > queued) {
                if (int rc = enqueue(need - queued)) return rc;
            } else if (pending.empty()) {
                if (int rc = enqueue(1)) return rc;
            }
        }
        HIPCHK(hipMemcpyAsync(out, S.ctrl, sizeof(Ctrl) * KB, hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        return FJ_OK;
    }

    int epilogue(BState<double>& S, const double* src, int64_t lds, int k, Ctrl* out) {
        int grid_win = 1;
        int rc = with_graph(c.g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            if (int e = grid_for(k_epilogue_batched<Vc, KB>, c.pl.K, &grid_win)) return e;
            k_epilogue_batched<Vc, KB><<<grid_win, WG, 0, c.st>>>(G, c.desc(), c.pl.K, k, ALL, S.X, src, lds, S.R,
                                                                  S.part, S.ctrl);
            HIPCHK(hipGetLastError());
            return FJ_OK;
        });
        if (rc) return rc;
        k_fin_epilogue_batched<KB><<<KB, WG, 0, c.st>>>(grid_win, c.g->n, ALL, S.part, S.ctrl);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(c.hs->slot(NSLOT), S.ctrl, sizeof(Ctrl) * KB, hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        std::memcpy(out, c.hs->slot(NSLOT), sizeof(Ctrl) * KB);
        return FJ_OK;
    }

    // Shared outer logic: after an epilogue, decide per column whether it is
    // finished (certified / converged, or stalled) and which columns restart.
    // Returns the columns to run again; status[col] is final for the others.
    uint64_t triage(const Ctrl* cs, int k, const fj_opts& o, bool want_indices, const unsigned* which,
                    double* rtol, const double* prev_rho, int* status, bool last) {
        uint64_t again = 0;
        for (int col = 0; col < k; ++col) {
            if (status[col] != FJ_ERR_NOT_CONVERGED) continue;  // already final
            const Ctrl& cc = cs[col];
            if (cc.done == BREAKDOWN) {
                status[col] = FJ_ERR_BREAKDOWN;
                continue;
            }
            const double snorm = cc.res[6], rho = cc.res[5];
            const bool ok = want_indices ? certified(cc, o.eps, which[col])
                                         : (snorm == 0.0 || rho <= rtol_target(o) * snorm);
            if (ok) {
                status[col] = FJ_OK;
            } else if (cc.done == ITER_CAP || cc.iters >= cc.max_iter) {
                status[col] = FJ_ERR_NOT_CONVERGED;
            } else if (last || !(rho < 0.5 * prev_rho[col])) {
                status[col] = stalled_status(cc, want_indices, which[col]);
            } else {
                again |= 1ull << col;
                double next = rtol[col] * 0.1;
                if (want_indices && snorm > 0.0)
                    next = std::min(next, 0.5 * needed_rho(cc, o.eps, which[col]) / snorm);
                rtol[col] = std::max(next, 1e-16);
            }
        }
        return again;
    }

    static double rtol_target(const fj_opts& o) { return o.rtol > 0.0 ? o.rtol : o.eps * 1e-2; }
    static bool deflate_ok(const fj_opts& o) { return !(o.flags & FJ_ZERO_START); }

    // FP64 for every column.
    int solve_fp64(BState<double>& S, const double* src, int64_t lds, int k, int kcheck, const fj_opts& o,
                   bool want_indices, const unsigned* which, Ctrl* cs, int* status, int* passes) {
        const int max_iter = o.max_iter > 0 ? o.max_iter : 2000;
        const bool range_check = !(o.flags & FJ_NO_RANGE_CHECK);
        double rtol[KMAX], prev_rho[KMAX];
        for (int col = 0; col < KMAX; ++col) {
            rtol[col] = rtol_target(o);
            prev_rho[col] = INFINITY;
            if (col < k) status[col] = FJ_ERR_NOT_CONVERGED;
        }
        // default target with indices: also stop a column once the estimates of
        // its five indices meet 0.8 eps (see k_fin_update_batched)
        const double eps_stop = (want_indices && o.rtol == 0.0 && !(o.flags & FJ_TWO_SOLVE)) ? 0.8 * o.eps : 0.0;
        if (eps_stop > 0.0) {
            S.s_est = src;
            S.s_lds = lds;
            S.s_k = k;
        }
        const bool deflate = deflate_ok(o);
        if (int rc = init(S, src, lds, k, kcheck, 0, ALL, rtol, max_iter, range_check, eps_stop, deflate)) return rc;
        *passes = 0;
        for (;;) {
            ++*passes;
            if (int rc = run(S, k, cs)) return rc;
            for (int col = 0; col < kcheck; ++col)
                if (cs[col].done == BAD_INPUT) return FJ_ERR_OPINION_RANGE;
            if (int rc = epilogue(S, src, lds, k, cs)) return rc;
            const uint64_t again = triage(cs, k, o, want_indices, which, rtol, prev_rho, status, *passes >= MAX_PASSES);
            if (!again) break;
            for (int col = 0; col < k; ++col) prev_rho[col] = cs[col].res[5];
            S.s_est = nullptr;  // a restart runs to its residual target
            if (int rc = init(S, src, lds, k, kcheck, 1, again, rtol, max_iter, range_check, 0.0, deflate)) return rc;
        }
        return FJ_OK;
    }

    // FJ_BLOCK_CG: the passes of solve_fp64 with block CG inside; every pass
    // runs to the residual target (no index-estimate stop), then the
    // epilogue certifies each column and uncertified columns restart from
    // their true residuals (the whole block iterates again).
    int solve_block_cg(BState<double>& S, const double* src, int64_t lds, int k, int kcheck, const fj_opts& o,
                       bool want_indices, const unsigned* which, Ctrl* cs, int* status, int* passes) {
        const int max_iter = o.max_iter > 0 ? o.max_iter : 2000;
        const bool range_check = !(o.flags & FJ_NO_RANGE_CHECK);
        double rtol[KMAX], prev_rho[KMAX];
        for (int col = 0; col < KMAX; ++col) {
            rtol[col] = rtol_target(o);
            prev_rho[col] = INFINITY;
            if (col < k) status[col] = FJ_ERR_NOT_CONVERGED;
        }
        if (int rc = init(S, src, lds, k, kcheck, 0, ALL, rtol, max_iter, range_check, 0.0, true)) return rc;
        HIPCHK(hipMemcpyAsync(c.hs->slot(NSLOT), S.ctrl, sizeof(Ctrl) * KB, hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        for (int col = 0; col < kcheck; ++col)
            if (c.hs->slot(NSLOT)[col].done == BAD_INPUT) return FJ_ERR_OPINION_RANGE;
        if (int rc = block_start(S)) return rc;
        *passes = 0;
        for (;;) {
            ++*passes;
            if (int rc = run(S, k, cs)) return rc;
            if (int rc = epilogue(S, src, lds, k, cs)) return rc;
            const uint64_t again = triage(cs, k, o, want_indices, which, rtol, prev_rho, status, *passes >= MAX_PASSES);
            if (!again) break;
            for (int col = 0; col < k; ++col) prev_rho[col] = cs[col].res[5];
            // the shared space restarts for every column from its true residual;
            // columns already final keep their targets (their residual stays small)
            if (int rc = init(S, src, lds, k, kcheck, 1, ALL, rtol, max_iter, range_check, 0.0, true)) return rc;
            if (int rc = block_start(S)) return rc;
        }
        return FJ_OK;
    }

    // FJ_MIXED for every column: FP32 inner CG, FP64 refinement per column.
    int solve_mixed(BState<double>& S, BState<float>& I, const double* src, int64_t lds, int k, int kcheck,
                    const fj_opts& o, bool want_indices, const unsigned* which, Ctrl* cs, int* status, int* outer) {
        const int max_iter = o.max_iter > 0 ? o.max_iter : 2000;
        const bool range_check = !(o.flags & FJ_NO_RANGE_CHECK);
        const int n = c.g->n;
        double prev_rho[KMAX];
        Ctrl ci[KMAX];
        double tau[KMAX], ones[KMAX];
        for (int col = 0; col < KMAX; ++col) {
            tau[col] = 1e-4;
            ones[col] = 1.0;
            if (col < k) status[col] = FJ_ERR_NOT_CONVERGED;
        }
        if (int rc = init(S, src, lds, k, kcheck, 0, ALL, ones, max_iter, range_check)) return rc;
        HIPCHK(hipMemcpyAsync(c.hs->slot(NSLOT), S.ctrl, sizeof(Ctrl) * KB, hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        std::memcpy(cs, c.hs->slot(NSLOT), sizeof(Ctrl) * KB);
        for (int col = 0; col < kcheck; ++col)
            if (cs[col].done == BAD_INPUT) return FJ_ERR_OPINION_RANGE;
        for (int col = 0; col < k; ++col) prev_rho[col] = std::sqrt(cs[col].ss);
        uint64_t active = 0;
        for (int col = 0; col < k; ++col) {
            if (cs[col].ss > 0.0) active |= 1ull << col;
            else status[col] = FJ_OK;  // s = 0: z = 0 exactly
        }
        int inner_total = 0;
        *outer = 0;
        while (active && *outer < 8 && inner_total < max_iter) {
            ++*outer;
            const int mode = *outer == 1 ? 0 : 1;
            k_mixed_cast_batched<KB><<<grid_vec, WG, 0, c.st>>>(n, S.R, I.R, mode, active, S.ctrl, 1);
            HIPCHK(hipGetLastError());
            if (int rc = init(I, nullptr, 0, k, 0, 2, active, tau, max_iter - inner_total, false, 0.0, deflate_ok(o)))
                return rc;
            if (int rc = run(I, k, ci)) return rc;
            int most = 0;
            for (int col = 0; col < k; ++col) most = std::max(most, ci[col].iters);
            inner_total += most;
            k_mixed_refine_batched<KB><<<grid_vec, WG, 0, c.st>>>(n, S.X, I.X, mode, active, S.ctrl);
            HIPCHK(hipGetLastError());
            if (int rc = epilogue(S, src, lds, k, cs)) return rc;
            uint64_t again = 0;
            for (int col = 0; col < k; ++col) {
                if (!((active >> col) & 1ull)) continue;
                const Ctrl& cc = cs[col];
                if (ci[col].done == BREAKDOWN) {
                    status[col] = FJ_ERR_BREAKDOWN;
                    continue;
                }
                const double snorm = cc.res[6], rho = cc.res[5];
                const bool ok = want_indices ? certified(cc, o.eps, which[col])
                                             : (snorm == 0.0 || rho <= rtol_target(o) * snorm);
                if (ok) {
                    status[col] = FJ_OK;
                } else if (!(rho < 0.5 * prev_rho[col])) {
                    status[col] = stalled_status(cc, want_indices, which[col]);
                } else {
                    again |= 1ull << col;
                    const double goal = want_indices ? needed_rho(cc, o.eps, which[col]) : rtol_target(o) * snorm;
                    tau[col] = std::min(1e-2, std::max(1e-5, 0.5 * goal / rho));
                    prev_rho[col] = rho;
                }
            }
            active = again;
        }
        for (int col = 0; col < k; ++col) {
            cs[col].iters = inner_total;
            if ((active >> col) & 1ull) status[col] = FJ_ERR_NOT_CONVERGED;
        }
        return FJ_OK;
    }
};

// k columns (or Algorithm 1's two right-hand sides) through one Batched<KB>.
template <int KB>
int solve_block(Ctx& c, const WsLayout& wl, char* W, const double* S, int64_t lds, int k, double* Z, int64_t ldz,
                const fj_opts& o, bool want_indices, fj_indices_t* out, fj_info* info) {
    Batched<KB> B{c};
    B.tune = (o.flags & FJ_NO_TUNE) == 0;
    if (int rc = B.setup()) return rc;
    const bool mixed = o.precision == FJ_MIXED;
    const bool two = (o.flags & FJ_TWO_SOLVE) && k == 1;
    Ctrl* ctrls = reinterpret_cast<Ctrl*>(W + wl.ctrl);
    double* part = reinterpret_cast<double*>(W + wl.part);
    BState<double> S64{reinterpret_cast<double*>(W + wl.x), reinterpret_cast<double*>(W + wl.r),
                       mixed ? nullptr : reinterpret_cast<double*>(W + wl.p),
                       mixed ? nullptr : reinterpret_cast<double*>(W + wl.q), ctrls, part};
    const double* src = S;
    int64_t ld = lds;
    int kk = k, kcheck = k;
    unsigned which[KMAX];
    for (int col = 0; col < KMAX; ++col) which[col] = ALL_INDICES;
    if (two) {
        // statistics of s (mean, range) with the single-vector init, then the
        // block [s, s - mean(s)]; only s itself is range-checked.
        const int max_iter = o.max_iter > 0 ? o.max_iter : 2000;
        k_ctrl_reset<<<1, WG, 0, c.st>>>(ctrls, 1);
        HIPCHK(hipGetLastError());
        k_cg_init<double><<<c.grid_vec, WG, 0, c.st>>>(c.g->n, S, lds, S64.X, S64.R, nullptr, c.minv(), 0, part);
        HIPCHK(hipGetLastError());
        k_fin_init<<<1, WG, 0, c.st>>>(c.grid_vec, c.g->n, part, 0, 1.0, max_iter,
                                       (o.flags & FJ_NO_RANGE_CHECK) ? 0 : 1, ctrls, 0.0, 0);
        HIPCHK(hipGetLastError());
        Ctrl st0{};
        HIPCHK(hipMemcpyAsync(&st0, ctrls, sizeof(Ctrl), hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        if (st0.done == BAD_INPUT) return FJ_ERR_OPINION_RANGE;
        double* blk = reinterpret_cast<double*>(W + wl.sblk);
        k_two_solve_rhs<<<c.grid_vec, WG, 0, c.st>>>(c.g->n, S, lds, ctrls, blk);
        HIPCHK(hipGetLastError());
        src = blk;
        ld = 2;
        kk = 2;
        kcheck = 0;
        which[0] = 1u | 8u;  // z = Solve(s): internal conflict ||L z||^2 and controversy ||z||^2
        which[1] = 2u | 8u;  // q = Solve(s - mean s): disagreement and polarization ||q||^2
    }
    Ctrl cs[KMAX];
    int status[KMAX];
    int passes = 0, outer = 0;
    int rc;
    if (mixed) {
        BState<float> S32{reinterpret_cast<float*>(W + wl.x32), reinterpret_cast<float*>(W + wl.r32),
                          reinterpret_cast<float*>(W + wl.p32), reinterpret_cast<float*>(W + wl.q32), ctrls + KB, part};
        rc = B.solve_mixed(S64, S32, src, ld, kk, kcheck, o, want_indices, which, cs, status, &outer);
    } else if (o.flags & FJ_BLOCK_CG) {
        if constexpr (KB >= 16) {
            B.block = true;
            B.Zb = reinterpret_cast<double*>(W + wl.zb);
            B.gpart = reinterpret_cast<double*>(W + wl.gpart);
            B.Gm = reinterpret_cast<double*>(W + wl.gm);
            B.Wm = reinterpret_cast<double*>(W + wl.wm);
            B.Cm = reinterpret_cast<double*>(W + wl.cm);
            B.zmean = reinterpret_cast<double*>(W + wl.zmean);
            if (int e = grid_for(k_block_mul<KB>, (static_cast<int64_t>(c.g->n) + 16 * NWAVE - 1) / (16 * NWAVE),
                                 &B.grid_mul))
                return e;
            rc = B.solve_block_cg(S64, src, ld, kk, kcheck, o, want_indices, which, cs, status, &passes);
        } else {
            return FJ_ERR_INVALID_ARG;  // block_columns gives at least 16
        }
    } else {
        rc = B.solve_fp64(S64, src, ld, kk, kcheck, o, want_indices, which, cs, status, &passes);
    }
    if (rc) return rc;
    int worst = FJ_OK;
    if (two) {
        const Ctrl &a = cs[0], &b = cs[1];  // a: z = Solve(s), b: q = Solve(s - mean s)
        const int st = status[0] != FJ_OK ? status[0] : status[1];
        if (out) {
            out[0].internal_conflict = a.res[0];
            out[0].disagreement = b.res[1];
            out[0].polarization = b.res[3];
            out[0].controversy = a.res[3];
            out[0].dc_index = b.res[1] + a.res[3];  // Algorithm 1: D~ + C~
        }
        if (info) {
            info[0].status = st;
            info[0].iters = std::max(a.iters, b.iters);
            info[0].passes = mixed ? outer : passes;
            info[0].outer_iters = mixed ? outer : 0;
            info[0].rel_residual = a.res[6] > 0.0 ? a.res[5] / a.res[6] : 0.0;
            info[0].bound[0] = a.bound[0];
            info[0].bound[1] = b.bound[1];
            info[0].bound[2] = b.bound[3];
            info[0].bound[3] = a.bound[3];
            info[0].bound[4] = std::max(b.bound[1], a.bound[3]);  // a sum of eps-approximations
            info[0].residual_norm = std::max(a.res[5], b.res[5]);
            double aa[5], ab[5];
            abs_bounds(a, aa);
            abs_bounds(b, ab);
            info[0].abs_bound[0] = aa[0];
            info[0].abs_bound[1] = ab[1];
            info[0].abs_bound[2] = ab[3];
            info[0].abs_bound[3] = aa[3];
            info[0].abs_bound[4] = ab[1] + aa[3];
        }
        worst = st;
        if (Z) {
            HIPCHK(hipMemcpy2DAsync(Z, sizeof(double) * ldz, S64.X, sizeof(double) * 2, sizeof(double), c.g->n,
                                    hipMemcpyDeviceToDevice, c.st));
        }
    } else {
        for (int col = 0; col < k; ++col) {
            fill_outputs(cs[col], status[col], mixed ? outer : passes, mixed ? outer : 0, out ? out + col : nullptr,
                         info ? info + col : nullptr);
            if (worst == FJ_OK && status[col] != FJ_OK) worst = status[col];
        }
        if (Z) {
            HIPCHK(hipMemcpy2DAsync(Z, sizeof(double) * ldz, S64.X, sizeof(double) * KB, sizeof(double) * k, c.g->n,
                                    hipMemcpyDeviceToDevice, c.st));
        }
    }
    if (info) {
        for (int col = 0; col < (two ? 1 : k); ++col)
            if (int e = c.profile_total(info + col)) return e;
    }
    HIPCHK(hipStreamSynchronize(c.st));
    return worst;
}

// Any number of columns: blocks of up to KMAX columns.
int solve_many(const fj_csr* g, const void* plan, int k, const double* S, int64_t lds, double* Z, int64_t ldz,
               const fj_opts& o, void* ws, size_t ws_bytes, void* stream, bool want_indices, fj_indices_t* out,
               fj_info* info, HostSlots* slots = nullptr) {
    Ctx c{};
    WsLayout wl{};
    if (int rc = make_ctx(g, plan, ws, ws_bytes, k, stream, &o, &c, &wl, slots)) return rc;
    char* W = static_cast<char*>(ws);
    int worst = FJ_OK;
    for (int c0 = 0; c0 < k; c0 += KMAX) {
        const int kc = std::min(KMAX, k - c0);
        const int kp = block_columns(kc, o.flags);
        const double* Sc = S + c0;
        double* Zc = Z ? Z + c0 : nullptr;
        fj_indices_t* oc = out ? out + c0 : nullptr;
        fj_info* ic = info ? info + c0 : nullptr;
        int rc;
        switch (kp) {
            case 2: rc = solve_block<2>(c, wl, W, Sc, lds, kc, Zc, ldz, o, want_indices, oc, ic); break;
            case 4: rc = solve_block<4>(c, wl, W, Sc, lds, kc, Zc, ldz, o, want_indices, oc, ic); break;
            case 8: rc = solve_block<8>(c, wl, W, Sc, lds, kc, Zc, ldz, o, want_indices, oc, ic); break;
            case 16: rc = solve_block<16>(c, wl, W, Sc, lds, kc, Zc, ldz, o, want_indices, oc, ic); break;
            case 32: rc = solve_block<32>(c, wl, W, Sc, lds, kc, Zc, ldz, o, want_indices, oc, ic); break;
            default: rc = solve_block<64>(c, wl, W, Sc, lds, kc, Zc, ldz, o, want_indices, oc, ic); break;
        }
        if (rc == FJ_ERR_HIP || rc == FJ_ERR_OPINION_RANGE || rc == FJ_ERR_WORKSPACE) return rc;
        if (worst == FJ_OK && rc != FJ_OK) worst = rc;
    }
    return worst;
}

#include "fj_server.hpp"

}  // namespace

// ---------------------------------------------------------------- no-allocation entry point
//
// fj_indices_noalloc keeps its workspace in this array: one copy per GPU the
// library runs on, alive until the process ends. In host code `scratch` is a
// host-side stand-in, never a device address: the device address of each
// GPU's copy comes from hipGetSymbolAddress (once per device, with that
// device current) and only that pointer is handed to kernels.
static __device__ __align__(256) unsigned char scratch[FJ_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;

struct NoAllocDevice {
    std::once_flag once;
    int rc = FJ_OK;
    void* ptr = nullptr;    // this device's copy of `scratch`
    HostSlots slots;        // pinned control-block slots and events for calls on this device
    std::mutex mu;          // calls on one device share the array: one at a time
};
NoAllocDevice g_noalloc[NOALLOC_MAX_DEVICES];

// Set-up on the first call on a device (the device is current): the array's
// address on this device, and the pinned slots the CG driver polls.
int noalloc_setup(int dev, NoAllocDevice& d) {
    std::call_once(d.once, [&]() {
        d.rc = [&]() -> int {
            HIPCHK(hipGetSymbolAddress(&d.ptr, HIP_SYMBOL(scratch)));
            HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&d.slots.h), sizeof(Ctrl) * KMAX * (NSLOT + 1),
                                 hipHostMallocDefault));
            for (auto& e : d.slots.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            return FJ_OK;
        }();
        (void)dev;
    });
    return d.rc;
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
        case FJ_ERR_CANCELLED: return "request cancelled";
        case FJ_ERR_HOST_MEMORY: return "host memory allocation failed";
        case FJ_ERR_INTERNAL: return "internal error (unexpected C++ exception)";
        default: return "unknown status";
    }
}

const char* fj_last_error(void) { return g_last_error; }

size_t fj_plan_bytes(const fj_csr* g) {
    if (check_graph_args(g)) return 0;
    return plan_layout(g).total;
}

size_t fj_workspace_bytes(const fj_csr* g, int32_t k, const fj_opts* opts) {
    if (check_graph_args(g) || k < 1) return 0;
    return ws_layout(g, k, opts ? opts->precision : FJ_FP64, opts ? opts->flags : 0u).total;
}

int fj_prepare(const fj_csr* g, const fj_opts* opts, void* plan, size_t plan_bytes, void* stream) {
    return guarded([&]() -> int {
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
            // heavy-edge matching for the 2x2 block preconditioner
            int* mate = reinterpret_cast<int*>(P + pl.mate);
            int* prop = reinterpret_cast<int*>(P + pl.prop);
            float* pw = reinterpret_cast<float*>(P + pl.pw);
            float2* pc = reinterpret_cast<float2*>(P + pl.pc);
            const int gv = static_cast<int>(std::min<int64_t>((static_cast<int64_t>(g->n) + WG - 1) / WG, 8192));
            k_pair_init<<<gv, WG, 0, st>>>(g->n, mate);
            HIPCHK(hipGetLastError());
            const int gw = static_cast<int>(std::min<int64_t>((static_cast<int64_t>(g->n) + NWAVE - 1) / NWAVE, 65536));
            for (int round = 0; round < PAIR_ROUNDS; ++round) {
                k_pair_propose<Vc><<<gw, WG, 0, st>>>(G, mate, prop, pw);
                HIPCHK(hipGetLastError());
                k_pair_accept<<<gv, WG, 0, st>>>(g->n, prop, mate);
                HIPCHK(hipGetLastError());
            }
            k_pair_coef<<<gv, WG, 0, st>>>(g->n, mate, pw, minv, pc);
            HIPCHK(hipGetLastError());
            // the time-phased layout (synchronises the stream)
            if (!pl.ph.s.ok) return FJ_OK;
            const int64_t waves = (pl.ph.s.W + NWAVE - 1) / NWAVE;
            int gc = 1, gp = 1, gf = 1;
            if (int e = grid_for(k_ph_count<Vc>, waves, &gc)) return e;
            if (int e = grid_for(k_ph_place<Vc>, waves, &gp)) return e;
            if (int e = grid_for(k_ph_fill<Vc>, (pl.ph.s.nnzp + WG - 1) / WG, &gf)) return e;
            return build_phased<Vc>(g, G, P, pl.ph, st, gc, gp, gf);
        });
    });
}

int fj_apply(const fj_csr* g, const void* plan, const double* x, double* y, void* stream) {
    return guarded([&]() -> int {
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
    });
}

int fj_apply_phased(const fj_csr* g, const void* plan, const double* x, double* y, void* stream) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (!plan || !aligned(plan)) return FJ_ERR_WORKSPACE;
        if (g->n == 0) return FJ_OK;
        if (!x || !y || x == y) return FJ_ERR_INVALID_ARG;
        const PlanLayout pl = plan_layout(g);
        if (!pl.ph.s.ok) {
            std::snprintf(g_last_error, sizeof g_last_error, "no time-phased layout for this graph");
            return FJ_ERR_INVALID_ARG;
        }
        hipStream_t st = static_cast<hipStream_t>(stream);
        return with_graph(g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            int grid = 1;
            const int64_t chunk_waves = (pl.ph.s.W + NWAVE - 1) / NWAVE;
            const PhasedCsr<Vc> phg = phased_view<Vc>(static_cast<const char*>(plan), pl.ph);
            if (pl.ph.s.rmax == PH_RMAX_LONG) {
                if (int rc = grid_for(k_apply_ph<Vc, PH_RMAX_LONG>, chunk_waves, &grid)) return rc;
                k_apply_ph<Vc, PH_RMAX_LONG><<<grid, WG, 0, st>>>(phg, x, y);
            } else {
                if (int rc = grid_for(k_apply_ph<Vc, PH_RMAX_SHORT>, chunk_waves, &grid)) return rc;
                k_apply_ph<Vc, PH_RMAX_SHORT><<<grid, WG, 0, st>>>(phg, x, y);
            }
            HIPCHK(hipGetLastError());
            return FJ_OK;
        });
    });
}

double fj_apriori_delta(int64_t n, double w_min, double w_max, double sbar_norm, double eps) {
    if (n < 1 || !(w_min > 0.0) || !(w_max >= w_min) || !(sbar_norm >= 0.0) || !(eps > 0.0 && eps < 0.5))
        return NAN;
    const double nd = static_cast<double>(n);
    return eps * w_min * sbar_norm / (3.0 * w_max * nd * nd * nd * (nd * w_max + 1.0) * std::sqrt(nd));
}

int fj_spmm_choice(const fj_csr* g, int32_t kb, int32_t precision, int32_t* cpl, int32_t* grid,
                   int32_t* split, int32_t* passes) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (!cpl || !grid || !split || !passes || kb < 2 || kb > KMAX || (kb & (kb - 1)) != 0)
            return FJ_ERR_INVALID_ARG;
        if (precision != FJ_FP64 && precision != FJ_MIXED) return FJ_ERR_INVALID_ARG;
        SpmmKey key{};
        if (int rc = spmm_key(g, kb, precision == FJ_FP64 ? 8 : 4, &key)) return rc;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune.find(key);
        if (it == g_tune.end()) return FJ_ERR_INVALID_ARG;
        *cpl = it->second.cpl;
        *grid = it->second.grid;
        *split = it->second.split ? 1 : 0;
        *passes = it->second.passes;
        return FJ_OK;
    });
}

int fj_spmm_set_choice(const fj_csr* g, int32_t kb, int32_t precision, int32_t cpl, int32_t grid, int32_t split,
                       int32_t passes) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (kb < 2 || kb > KMAX || (kb & (kb - 1)) != 0) return FJ_ERR_INVALID_ARG;
        if (precision != FJ_FP64 && precision != FJ_MIXED) return FJ_ERR_INVALID_ARG;
        if ((cpl != 1 && cpl != 2 && cpl != 4) || kb % cpl != 0 || grid < 1 || grid > GMAX) return FJ_ERR_INVALID_ARG;
        if (split != 0 && split != 1) return FJ_ERR_INVALID_ARG;
        if (!spmm_shape_ok(kb, cpl, split == 1, passes)) return FJ_ERR_INVALID_ARG;
        SpmmKey key{};
        if (int rc = spmm_key(g, kb, precision == FJ_FP64 ? 8 : 4, &key)) return rc;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[key] = SpmmChoice{cpl, grid, split == 1, passes};
        return FJ_OK;
    });
}

#include "fj_aids.hpp"

#include "fj_hierarchy.hpp"

#include "fj_reorder.hpp"

int fj_dynamics(const fj_csr* g, const void* plan, const double* s, const double* z0, double* z,
                int32_t steps, double tol, void* ws, size_t ws_bytes, void* stream, fj_info* info) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (!plan || !ws || !aligned(plan) || !aligned(ws)) return FJ_ERR_WORKSPACE;
        if (steps < 0 || !(tol == tol)) return FJ_ERR_INVALID_ARG;
        if (g->n > 0 && (!s || !z)) return FJ_ERR_INVALID_ARG;
        const WsLayout wl = ws_layout(g, 1, FJ_FP64, 0);
        if (ws_bytes < wl.total) return FJ_ERR_WORKSPACE;
        if (info) *info = fj_info{};
        hipStream_t st = static_cast<hipStream_t>(stream);
        const int n = g->n;
        if (!z0) z0 = s;
        if (n == 0) return FJ_OK;
        if (steps == 0) {
            if (z0 != z) HIPCHK(hipMemcpyAsync(z, z0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            return FJ_OK;
        }
        const PlanLayout pl = plan_layout(g);
        const WinDesc* desc = reinterpret_cast<const WinDesc*>(static_cast<const char*>(plan) + pl.desc);
        char* W = static_cast<char*>(ws);
        double* B = reinterpret_cast<double*>(W + wl.x);
        double* part = reinterpret_cast<double*>(W + wl.part);
        Ctrl* ctrl = reinterpret_cast<Ctrl*>(W + wl.ctrl);
        HostSlots* hs = nullptr;
        if (int rc = host_slots(&hs)) return rc;
        if (z0 == z) {  // the first step must not read and write the same vector
            HIPCHK(hipMemcpyAsync(B, z0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            z0 = B;
        }
        k_ctrl_reset<<<1, WG, 0, st>>>(ctrl, 1);
        HIPCHK(hipGetLastError());
        k_fj_ctrl_init<<<1, 64, 0, st>>>(ctrl, tol < 0.0 ? -1.0 : tol, steps);
        HIPCHK(hipGetLastError());
        // step t reads src(t) and writes dst(t): dst(t) = z for even t, B for odd t
        auto src = [&](int t) -> const double* { return t == 0 ? z0 : (t % 2 == 1 ? z : B); };
        auto dst = [&](int t) -> double* { return t % 2 == 0 ? z : B; };
        int queued = 0, slot_next = 0;
        Pending pending;
        Ctrl fin{};
        int rc = with_graph(g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            int grid = 1;
            // from PH_MIN_N nodes on the sweeps run on the time-phased layout
            const bool ph = pl.ph.s.ok && n >= PH_MIN_N;
            const bool lng = pl.ph.s.rmax == PH_RMAX_LONG;
            if (ph) {
                const int64_t chunk_waves = (pl.ph.s.W + NWAVE - 1) / NWAVE;
                if (int e = lng ? grid_for(k_fj_sweep_ph<Vc, PH_RMAX_LONG>, chunk_waves, &grid)
                                : grid_for(k_fj_sweep_ph<Vc, PH_RMAX_SHORT>, chunk_waves, &grid))
                    return e;
            } else {
                if (int e = grid_for(k_fj_sweep<Vc>, pl.K, &grid)) return e;
            }
            const PhasedCsr<Vc> phg = phased_view<Vc>(static_cast<const char*>(plan), pl.ph);
            auto enqueue = [&](int cnt) -> int {
                for (int c = 0; c < cnt; ++c, ++queued) {
                    if (ph && lng)
                        k_fj_sweep_ph<Vc, PH_RMAX_LONG><<<grid, WG, 0, st>>>(phg, src(queued), s, dst(queued), part,
                                                                             ctrl);
                    else if (ph)
                        k_fj_sweep_ph<Vc, PH_RMAX_SHORT><<<grid, WG, 0, st>>>(phg, src(queued), s, dst(queued), part,
                                                                              ctrl);
                    else
                        k_fj_sweep<Vc><<<grid, WG, 0, st>>>(G, desc, pl.K, src(queued), s, dst(queued), part, ctrl);
                    HIPCHK(hipGetLastError());
                    k_fin_fj<<<1, WG, 0, st>>>(grid, part, ctrl);
                    HIPCHK(hipGetLastError());
                }
                const int sl = slot_next++ % NSLOT;
                HIPCHK(hipMemcpyAsync(hs->slot(sl), ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
                HIPCHK(hipEventRecord(hs->ev[sl], st));
                if (!pending.push_back(sl)) return FJ_ERR_INTERNAL;
                return FJ_OK;
            };
            constexpr int CHUNK = 32;
            for (int k = 0; k < 2 && queued < steps; ++k)
                if (int e = enqueue(std::min(CHUNK, steps - queued))) return e;
            while (!pending.empty()) {
                const int sl = pending.front();
                pending.pop_front();
                HIPCHK(hipEventSynchronize(hs->ev[sl]));
                const Ctrl& cc = *hs->slot(sl);
                if (cc.done != RUNNING) break;
                if (queued < steps)
                    if (int e = enqueue(std::min(CHUNK, steps - queued))) return e;
            }
            return FJ_OK;
        });
        if (rc) return rc;
        // later chunks are empty launches once the control block says done
        HIPCHK(hipMemcpyAsync(hs->slot(NSLOT), ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::memcpy(&fin, hs->slot(NSLOT), sizeof(Ctrl));
        const int taken = fin.iters;
        if (taken > 0 && dst(taken - 1) != z) {
            HIPCHK(hipMemcpyAsync(z, B, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        int status = FJ_OK;
        if (fin.done == BREAKDOWN) status = FJ_ERR_BREAKDOWN;
        else if (fin.done != CONVERGED && tol >= 0.0) status = FJ_ERR_NOT_CONVERGED;
        if (info) {
            info->status = status;
            info->iters = taken;
            info->passes = 1;
            info->rel_residual = fin.res[0];
        }
        return status;
    });
}

int fj_solve(const fj_csr* g, const void* plan, int32_t k, const double* S, int64_t lds, double* Z,
             int64_t ldz, const fj_opts* opts, void* ws, size_t ws_bytes, void* stream, fj_info* info) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (int rc = check_opts(opts)) return rc;
        if (k < 1 || lds < k || ldz < k || !S || !Z) return FJ_ERR_INVALID_ARG;
        if ((opts->flags & FJ_BLOCK_CG) && k < 2) return FJ_ERR_INVALID_ARG;
        if (int rc = check_ml(g, k, opts)) return rc;
        if ((opts->flags & FJ_WARM_START) && (k != 1 || (opts->flags & FJ_TWO_SOLVE))) {
            std::snprintf(g_last_error, sizeof g_last_error, "FJ_WARM_START needs k = 1 without FJ_TWO_SOLVE");
            return FJ_ERR_INVALID_ARG;
        }
        if (g->n == 0) return FJ_OK;
        if (k == 1 && !(opts->flags & FJ_TWO_SOLVE))
            return solve_one(g, plan, S, lds, Z, ldz, *opts, ws, ws_bytes, stream, false, nullptr, info);
        return solve_many(g, plan, k, S, lds, Z, ldz, *opts, ws, ws_bytes, stream, false, nullptr, info);
    });
}

int fj_indices(const fj_csr* g, const void* plan, int32_t k, const double* S, int64_t lds,
               const fj_opts* opts, void* ws, size_t ws_bytes, void* stream, fj_indices_t* out,
               fj_info* info) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (int rc = check_opts(opts)) return rc;
        if (k < 1 || lds < k || !S || !out) return FJ_ERR_INVALID_ARG;
        if (g->n == 0) return FJ_ERR_INVALID_ARG;
        if ((opts->flags & FJ_BLOCK_CG) && k < 2) return FJ_ERR_INVALID_ARG;
        if (int rc = check_ml(g, k, opts)) return rc;
        if (k == 1 && !(opts->flags & FJ_TWO_SOLVE))
            return solve_one(g, plan, S, lds, nullptr, 0, *opts, ws, ws_bytes, stream, true, out, info);
        return solve_many(g, plan, k, S, lds, nullptr, 0, *opts, ws, ws_bytes, stream, true, out, info);
    });
}

int fj_indices_noalloc(const fj_csr* g, const void* plan, int32_t k, const double* S, int64_t lds,
                       const fj_opts* opts, void* stream, fj_indices_t* out, fj_info* info) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (int rc = check_opts(opts)) return rc;
        if (k < 1 || lds < k || !S || !out) return FJ_ERR_INVALID_ARG;
        if (g->n == 0) return FJ_ERR_INVALID_ARG;
        if (opts->flags & FJ_MULTILEVEL) {  // a hierarchy's work vectors are shared, not scratch
            std::snprintf(g_last_error, sizeof g_last_error, "fj_indices_noalloc: FJ_MULTILEVEL is not available");
            return FJ_ERR_INVALID_ARG;
        }
        if (opts->flags & FJ_PROFILE) {  // profiling creates events
            std::snprintf(g_last_error, sizeof g_last_error, "fj_indices_noalloc: FJ_PROFILE is not available");
            return FJ_ERR_INVALID_ARG;
        }
        fj_opts o = *opts;
        o.flags |= FJ_NO_TUNE;  // the SpMM autotuner times candidates with events of its own
        const size_t need = ws_layout(g, k, o.precision, o.flags).total;
        if (need > FJ_NOALLOC_SCRATCH_BYTES) {
            std::snprintf(g_last_error, sizeof g_last_error,
                          "fj_indices_noalloc: this solve needs %zu bytes of workspace, the static scratch holds %zu",
                          need, static_cast<size_t>(FJ_NOALLOC_SCRATCH_BYTES));
            return FJ_ERR_WORKSPACE;
        }
        int dev = 0;
        if (int rc = current_device(&dev)) return rc;
        if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return FJ_ERR_INVALID_ARG;
        NoAllocDevice& d = g_noalloc[dev];
        if (int rc = noalloc_setup(dev, d)) return rc;
        std::lock_guard<std::mutex> lock(d.mu);
        if (k == 1 && !(o.flags & FJ_TWO_SOLVE))
            return solve_one(g, plan, S, lds, nullptr, 0, o, d.ptr, FJ_NOALLOC_SCRATCH_BYTES, stream, true, out, info,
                             &d.slots);
        return solve_many(g, plan, k, S, lds, nullptr, 0, o, d.ptr, FJ_NOALLOC_SCRATCH_BYTES, stream, true, out,
                          info, &d.slots);
    });
}

size_t fj_server_block_bytes(int32_t n, int32_t block_columns, int32_t precision) {
    if (n < 1 || (block_columns != 16 && block_columns != 64)) return 0;
    if (precision != FJ_FP64 && precision != FJ_MIXED) return 0;
    return block_bytes(n, block_columns, precision == FJ_MIXED);
}

int fj_server_create(const fj_server_opts* opts, fj_server** out) {
    return guarded([&]() -> int {
        if (!opts || !out) return FJ_ERR_INVALID_ARG;
        if (opts->precision != FJ_FP64 && opts->precision != FJ_MIXED) return FJ_ERR_INVALID_ARG;
        if (opts->block_columns != 16 && opts->block_columns != 64) return FJ_ERR_INVALID_ARG;
        if (opts->iters_per_replay < 1 || opts->iters_per_replay > 256) return FJ_ERR_INVALID_ARG;
        if (!(opts->eps > 0.0 && opts->eps < 0.5) || opts->max_iter < 0) return FJ_ERR_INVALID_ARG;
        if (!opts->arena || !aligned(opts->arena) || opts->arena_bytes == 0) return FJ_ERR_WORKSPACE;
        if (opts->large_lanes < 0 || opts->large_lanes > 8 || opts->large_entries < 0) return FJ_ERR_INVALID_ARG;
        if (opts->large_iters_per_replay < 0 || opts->large_iters_per_replay > 256) return FJ_ERR_INVALID_ARG;
        if (opts->large_blocks < 0 || opts->large_blocks > 4) return FJ_ERR_INVALID_ARG;
        Server* s = new Server();
        s->o = *opts;
        if (s->o.large_blocks == 0) s->o.large_blocks = 1;
        if (s->o.large_lanes == 0) s->o.large_lanes = 2;
        if (s->o.large_entries == 0) s->o.large_entries = int64_t(1) << 22;
        if (s->o.large_iters_per_replay == 0) s->o.large_iters_per_replay = std::max(1, s->o.iters_per_replay / 4);
        s->arena = static_cast<char*>(opts->arena);
        s->free_list[0] = opts->arena_bytes / ALIGN * ALIGN;
        int rc = current_device(&s->device);
        // the lanes: large_lanes streams for large graphs, then one for the others
        for (int l = 0; rc == FJ_OK && l <= s->o.large_lanes; ++l) {
            hipStream_t ls = nullptr;
            const hipError_t e = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking);
            if (e != hipSuccess) {
                set_error("fj_server_create: hipStreamCreateWithFlags", e);
                rc = FJ_ERR_HIP;
                break;
            }
            s->lanes.push_back(ls);
        }
        if (rc) {
            for (hipStream_t ls : s->lanes) (void)hipStreamDestroy(ls);
            delete s;
            return rc;
        }
        *out = reinterpret_cast<fj_server*>(s);
        return FJ_OK;
    });
}

int fj_server_destroy(fj_server* srv) {
    return guarded([&]() -> int {
        if (!srv) return FJ_ERR_INVALID_ARG;
        Server* s = reinterpret_cast<Server*>(srv);
        int status = FJ_OK;
        for (auto& G : s->graphs) {
            if (G.blk)
                if (int rc = release_block(*s, G)) status = rc;
            if (G.dep) (void)hipEventDestroy(G.dep);
        }
        for (hipStream_t ls : s->lanes) {
            hipError_t e = hipStreamSynchronize(ls);
            if (e == hipSuccess) e = hipStreamDestroy(ls);
            if (e != hipSuccess && status == FJ_OK) {
                set_error("fj_server_destroy: lane stream", e);
                status = FJ_ERR_HIP;
            }
        }
        delete s;
        return status;
    });
}

int fj_server_add_graph(fj_server* srv, const fj_csr* g, const void* plan, int32_t* graph_id, void* stream) {
    return guarded([&]() -> int {
        if (!srv || !graph_id) return FJ_ERR_INVALID_ARG;
        if (int rc = check_graph_args(g)) return rc;
        if (g->n < 1) return FJ_ERR_INVALID_ARG;
        if (!plan || !aligned(plan)) return FJ_ERR_WORKSPACE;
        Server* s = reinterpret_cast<Server*>(srv);
        const bool large = static_cast<int64_t>(g->n) + g->nnz >= s->o.large_entries;
        const int nb = large ? s->o.large_blocks : 1;
        // may throw: nothing created yet
        s->graphs.reserve(s->graphs.size() + nb);
        s->entries.reserve(s->entries.size() + 1);
        std::vector<int> mine;
        mine.reserve(nb);
        std::vector<ServerGraph> made;
        made.reserve(nb);
        const int nl = s->o.large_lanes;
        for (int b = 0; b < nb; ++b) {
            ServerGraph G;
            G.g = *g;
            G.plan = plan;
            G.pl = plan_layout(g);
            // a large graph's blocks take the large lanes in turn, any other graph the last lane
            G.large = large;
            G.st = large ? s->lanes[(s->n_large + b) % nl] : s->lanes[nl];
            hipError_t e = hipEventCreateWithFlags(&G.dep, hipEventDisableTiming);
            // the block's work waits for the caller's work so far (fj_prepare of this plan)
            if (e == hipSuccess) e = hipEventRecord(G.dep, static_cast<hipStream_t>(stream));
            if (e == hipSuccess) e = hipStreamWaitEvent(G.st, G.dep, 0);
            if (e != hipSuccess) {
                set_error("fj_server_add_graph: event", e);
                if (G.dep) (void)hipEventDestroy(G.dep);
                for (ServerGraph& M : made) (void)hipEventDestroy(M.dep);
                return FJ_ERR_HIP;
            }
            made.push_back(std::move(G));  // capacity reserved: does not throw
        }
        if (large) s->n_large += nb;
        // capacities are reserved; moving a ServerGraph may still allocate (its deque), and a
        // failure here leaves unused entries behind but returns no graph id
        for (ServerGraph& G : made) {
            mine.push_back(static_cast<int>(s->graphs.size()));
            s->graphs.push_back(std::move(G));
        }
        s->entries.push_back(std::move(mine));
        *graph_id = static_cast<int32_t>(s->entries.size() - 1);
        return FJ_OK;
    });
}

int fj_server_submit(fj_server* srv, int32_t graph_id, int32_t k, const double* S, int64_t lds, fj_indices_t* out,
                     fj_info* info, uint64_t* request_id, void* stream) {
    return guarded([&]() -> int {
        if (!srv || !S || !out || !request_id) return FJ_ERR_INVALID_ARG;
        Server* s = reinterpret_cast<Server*>(srv);
        if (graph_id < 0 || graph_id >= static_cast<int32_t>(s->entries.size())) return FJ_ERR_INVALID_ARG;
        if (k < 1 || k > s->o.block_columns || lds < k) return FJ_ERR_INVALID_ARG;
        // the graph's block with the fewest columns waiting or running (the first on ties)
        int pick = -1;
        int64_t best = 0;
        for (int e : s->entries[graph_id]) {
            const ServerGraph& H = s->graphs[e];
            int64_t load = 0;
            for (uint64_t q : H.queue) {
                const auto it = s->requests.find(q);
                if (it != s->requests.end()) load += it->second.k - it->second.admitted;
            }
            if (H.blk)
                for (int c = 0; c < s->o.block_columns; ++c) load += H.blk->slot_req[c] >= 0;
            if (pick < 0 || load < best) {
                pick = e;
                best = load;
            }
        }
        ServerGraph& G = s->graphs[pick];
        if (block_bytes(G.g.n, s->o.block_columns, s->o.precision == FJ_MIXED) > s->o.arena_bytes)
            return FJ_ERR_WORKSPACE;  // could never run
        ServerRequest r;
        r.id = s->next_id;
        r.gid = pick;
        r.user_gid = graph_id;
        r.k = k;
        r.S = S;
        r.lds = lds;
        r.out = out;
        r.info = info;
        r.remaining = k;
        r.t_submit = std::chrono::steady_clock::now();
        // whatever reads S later on the graph's stream waits for the caller's
        // work queued so far (the producer of S)
        HIPCHK(hipEventRecord(G.dep, static_cast<hipStream_t>(stream)));
        HIPCHK(hipStreamWaitEvent(G.st, G.dep, 0));
        auto ins = s->requests.emplace(r.id, r);  // may throw: nothing changed yet
        try {
            G.queue.push_back(r.id);
        } catch (...) {
            s->requests.erase(ins.first);
            throw;
        }
        ++s->next_id;
        *request_id = r.id;
        return FJ_OK;
    });
}

int fj_server_step(fj_server* srv, int32_t* busy_blocks) {
    return guarded([&]() -> int {
        if (!srv) return FJ_ERR_INVALID_ARG;
        Server* s = reinterpret_cast<Server*>(srv);
        int busy = 0;
        const int rc = s->o.block_columns == 64 ? server_step_kb<64>(*s, &busy) : server_step_kb<16>(*s, &busy);
        if (busy_blocks) *busy_blocks = busy;
        return rc;
    });
}

int fj_server_poll(fj_server* srv, fj_server_done* done, int32_t max, int32_t* count) {
    return guarded([&]() -> int {
        if (!srv || !count || (max > 0 && !done)) return FJ_ERR_INVALID_ARG;
        Server* s = reinterpret_cast<Server*>(srv);
        int32_t n = 0;
        while (n < max && !s->completed.empty()) {
            const uint64_t rid = s->completed.front();
            s->completed.pop_front();
            auto it = s->requests.find(rid);
            if (it == s->requests.end()) continue;
            const ServerRequest& r = it->second;
            done[n].request_id = rid;
            done[n].graph_id = r.user_gid;
            done[n].status = r.status;
            done[n].latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
            s->requests.erase(it);
            ++n;
        }
        *count = n;
        return FJ_OK;
    });
}

int fj_server_cancel(fj_server* srv, uint64_t request_id) {
    return guarded([&]() -> int {
        if (!srv) return FJ_ERR_INVALID_ARG;
        Server* s = reinterpret_cast<Server*>(srv);
        auto it = s->requests.find(request_id);
        if (it == s->requests.end() || it->second.remaining == 0) return FJ_ERR_INVALID_ARG;
        ServerRequest& r = it->second;
        ServerGraph& G = s->graphs[r.gid];
        for (auto q = G.queue.begin(); q != G.queue.end(); ++q)
            if (*q == request_id) {
                G.queue.erase(q);
                break;
            }
        if (ServerBlock* b = G.blk) {
            uint64_t mask = 0;
            for (int c = 0; c < s->o.block_columns; ++c)
                if (b->slot_req[c] == static_cast<int64_t>(request_id)) {
                    mask |= 1ull << c;
                    b->slot_req[c] = -1;
                }
            if (mask) {  // stream-ordered after any replay or epilogue in flight
                for (Ctrl* cb : {b->ctrl, b->ictrl}) {
                    if (!cb) continue;
                    k_ctrl_set_done<<<1, WG, 0, G.st>>>(cb, s->o.block_columns, mask, static_cast<int>(CONVERGED));
                    HIPCHK(hipGetLastError());
                }
                b->running &= ~mask;
                b->finishing &= ~mask;
                // the caller may free the request's opinion vectors once it is
                // reported: let the scatter that read them finish first
                HIPCHK(hipStreamSynchronize(G.st));
            }
        }
        r.status = FJ_ERR_CANCELLED;
        r.remaining = 0;
        r.t_done = std::chrono::steady_clock::now();
        s->completed.push_back(request_id);
        return FJ_OK;
    });
}

}  // extern "C"
