// fj_server.hpp -- continuous-batching server for FJ index requests (host side).
// Included by fj_api.hip inside its anonymous namespace; the extern "C" entry
// points are defined there.
//
// Graphs stay resident (CSR and plan owned by the caller). A graph with work
// gets a block: the CG state of KB columns carved from a caller-provided HBM
// arena by a first-fit allocator (admission by HBM footprint). FP64 blocks
// hold X, R, P, Q, the opinion block S, partials and KB control blocks;
// FJ_MIXED blocks hold the FP64 solution, true residual and S, FP32 inner CG
// vectors, and outer plus inner control blocks. The columns of a request
// (graph, k opinion vectors) enter free columns of the block in arrival
// order, at an iteration boundary, while the other columns keep iterating.
// Each block replays a HIP graph of `iters` captured CG iterations (FP32
// inner iterations for FJ_MIXED) on its graph's lane: large graphs (n + nnz
// at least large_entries) share large_lanes streams in turn, all other
// graphs one more stream. A hardware queue runs its work in order, so with
// one stream per graph a small graph's short replay could wait behind a
// large graph's long one sharing its queue; the lanes keep short and long
// work on different queues, and blocks on different lanes overlap. Large
// graphs also replay fewer iterations at a time (large_iters_per_replay), so
// that requests join their blocks sooner, and may hold several blocks
// (large_blocks, each an entry of its own in `graphs`; a request goes whole
// to the block with the least work). After each replay the host reads the control
// blocks; columns whose CG stopped are finished by the batched epilogue
// (after the FP64 correction z += ||r|| d for FJ_MIXED), then retired
// (certified, or final) or restarted from their true residual with a
// tighter target. A column's arithmetic never depends on the other columns
// of its block, so a result is bitwise the same alone or in the mix.
#pragma once

#include <chrono>
#include <unordered_map>

struct ServerRequest {
    uint64_t id = 0;
    int gid = 0;        // the internal graph entry (block) serving it
    int user_gid = 0;   // the caller's graph id
    int k = 0;
    const double* S = nullptr;
    int64_t lds = 0;
    fj_indices_t* out = nullptr;  // host, k entries
    fj_info* info = nullptr;      // host, k entries (may be null)
    int admitted = 0;   // columns placed in the block so far (in column order)
    int remaining = 0;  // columns not finished yet
    int status = FJ_OK;
    std::chrono::steady_clock::time_point t_submit, t_done;
};

enum class Phase { IDLE, REPLAY, EPILOGUE };

struct ServerBlock {
    size_t offset = 0, bytes = 0;
    bool mixed = false;
    double *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr, *S = nullptr;  // P, Q: FP64 blocks only
    float *X32 = nullptr, *R32 = nullptr, *P32 = nullptr, *Q32 = nullptr;         // FJ_MIXED inner CG
    Ctrl* ctrl = nullptr;   // FP64 CG (FP64 blocks) or outer refinement (FJ_MIXED) control blocks
    Ctrl* ictrl = nullptr;  // FJ_MIXED: inner CG control blocks
    double* part = nullptr;
    Ctrl* host = nullptr;  // pinned copy of the control blocks (outer, then inner)
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t slot_req[KMAX];  // request whose column occupies the slot (-1: free)
    int slot_col[KMAX];      // which column of that request
    double rtol[KMAX];       // FP64: relative residual target of the current pass
    double tau[KMAX];        // FJ_MIXED: inner relative residual target
    double prev_rho[KMAX];
    int outer[KMAX];         // FJ_MIXED: refinement steps so far
    int inner_total[KMAX];   // FJ_MIXED: inner iterations so far
    uint64_t running = 0, finishing = 0;
    Phase phase = Phase::IDLE;
    int grid_win = 1, grid_vec = 1;
    uint64_t last_used = 0;  // scheduling step that last found work in the block
};

struct ServerGraph {
    fj_csr g{};
    const void* plan = nullptr;
    PlanLayout pl{};
    hipStream_t st = nullptr;  // the graph's lane (shared with other graphs of its size class)
    bool large = false;        // n + nnz >= large_entries: a large lane and shorter replays
    hipEvent_t dep = nullptr;  // orders the lane after the caller's producer of plan / S
    std::deque<uint64_t> queue;
    ServerBlock* blk = nullptr;
};

struct Server {
    fj_server_opts o{};
    char* arena = nullptr;
    std::map<size_t, size_t> free_list;  // offset -> bytes
    std::vector<ServerGraph> graphs;           // one entry per block: a large graph may have several
    std::vector<std::vector<int>> entries;     // caller's graph id -> its entries in graphs
    std::unordered_map<uint64_t, ServerRequest> requests;
    std::deque<uint64_t> completed;
    std::vector<hipStream_t> lanes;  // large_lanes streams for large graphs, then one for the others
    int n_large = 0;                 // large graphs so far (they take the large lanes in turn)
    uint64_t next_id = 1;
    uint64_t tick = 0;  // scheduling steps so far
    int device = 0;
};

// ------------------------------------------------------------ arena

bool arena_alloc(Server& s, size_t bytes, size_t* off) {
    for (auto it = s.free_list.begin(); it != s.free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            s.free_list.erase(it);
            if (rest) s.free_list[at] = rest;
            return true;
        }
    }
    return false;
}

void arena_free(Server& s, size_t off, size_t bytes) {
    auto it = s.free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != s.free_list.end() && it->first + it->second == nx->first) {  // merge with the next range
        it->second += nx->second;
        s.free_list.erase(nx);
    }
    if (it != s.free_list.begin()) {  // merge with the previous range
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s.free_list.erase(it);
        }
    }
}

size_t block_bytes(int n, int kb, bool mixed) {
    const size_t v = align_up(sizeof(double) * static_cast<size_t>(n) * kb);
    const size_t v32 = align_up(sizeof(float) * static_cast<size_t>(n) * kb);
    const size_t tail = align_up(sizeof(double) * GMAX * BPART * kb) + align_up(sizeof(Ctrl) * kb) * (mixed ? 2 : 1);
    return (mixed ? 3 * v + 4 * v32 : 5 * v) + tail;
}

// ------------------------------------------------------------ per-KB machinery

template <int KB>
struct ServerOps {
    static constexpr uint64_t ALL = KB >= 64 ? ~0ull : ((1ull << KB) - 1ull);

    static int create(Server& s, ServerGraph& G, ServerBlock* b) {
        const int n = G.g.n;
        const bool mixed = s.o.precision == FJ_MIXED;
        b->mixed = mixed;
        char* base = s.arena + b->offset;
        const size_t v = align_up(sizeof(double) * static_cast<size_t>(n) * KB);
        const size_t v32 = align_up(sizeof(float) * static_cast<size_t>(n) * KB);
        size_t at = 0;
        auto take = [&](size_t bytes) { char* p = base + at; at += bytes; return p; };
        b->X = reinterpret_cast<double*>(take(v));
        b->R = reinterpret_cast<double*>(take(v));
        b->S = reinterpret_cast<double*>(take(v));
        if (mixed) {
            b->X32 = reinterpret_cast<float*>(take(v32));
            b->R32 = reinterpret_cast<float*>(take(v32));
            b->P32 = reinterpret_cast<float*>(take(v32));
            b->Q32 = reinterpret_cast<float*>(take(v32));
        } else {
            b->P = reinterpret_cast<double*>(take(v));
            b->Q = reinterpret_cast<double*>(take(v));
        }
        const size_t vec_bytes = at;
        b->part = reinterpret_cast<double*>(take(align_up(sizeof(double) * GMAX * BPART * KB)));
        b->ctrl = reinterpret_cast<Ctrl*>(take(align_up(sizeof(Ctrl) * KB)));
        if (mixed) b->ictrl = reinterpret_cast<Ctrl*>(take(align_up(sizeof(Ctrl) * KB)));
        for (int c = 0; c < KMAX; ++c) {
            b->slot_req[c] = -1;
            b->rtol[c] = 0.0;
            b->tau[c] = 1e-4;
            b->prev_rho[c] = INFINITY;
            b->outer[c] = 0;
            b->inner_total[c] = 0;
        }
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&b->host), sizeof(Ctrl) * KB * 2, hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming));
        const int64_t units = (static_cast<int64_t>(n) * KB + WG - 1) / WG;
        if (int rc = grid_for(k_update_batched<double, KB, true>, units, &b->grid_vec)) return rc;
        // zero the vectors (kernels, not memsets), every column idle
        k_fill_zero<<<b->grid_vec, WG, 0, G.st>>>(b->X, static_cast<int64_t>(vec_bytes / sizeof(double)));
        HIPCHK(hipGetLastError());
        for (Ctrl* cb : {b->ctrl, b->ictrl}) {
            if (!cb) continue;
            k_ctrl_reset<<<1, WG, 0, G.st>>>(cb, KB);
            HIPCHK(hipGetLastError());
            k_ctrl_set_done<<<1, WG, 0, G.st>>>(cb, KB, ALL, static_cast<int>(CONVERGED));
            HIPCHK(hipGetLastError());
        }
        return mixed ? capture<float>(s, G, b, b->X32, b->R32, b->P32, b->Q32, b->ictrl)
                     : capture<double>(s, G, b, b->X, b->R, b->P, b->Q, b->ctrl);
    }

    // Capture `iters` CG iterations on the block's CG vectors.
    template <typename T>
    static int capture(Server& s, ServerGraph& G, ServerBlock* b, T* X, T* R, T* P, T* Q, Ctrl* cg) {
        const int n = G.g.n;
        return with_graph(&G.g, [&](auto Gc) -> int {
            using Vc = typename decltype(Gc)::value_type;
            const WinDesc* desc = reinterpret_cast<const WinDesc*>(static_cast<const char*>(G.plan) + G.pl.desc);
            const float* minv = reinterpret_cast<const float*>(static_cast<const char*>(G.plan) + G.pl.minv);
            // the same tuned launch shape as the eager batched path of this graph, width and precision
            SpmmChoice ch{};
            if (int e = Spmm<Vc, T, KB>::choose(&G.g, G.st, Gc, desc, G.pl.K, P, R, minv, Q, b->part, true, &ch))
                return e;
            b->grid_win = ch.grid;
            HIPCHK(hipStreamBeginCapture(G.st, hipStreamCaptureModeThreadLocal));
            const int iters = G.large ? s.o.large_iters_per_replay : s.o.iters_per_replay;
            for (int t = 0; t < iters; ++t) {
                if (int e = Spmm<Vc, T, KB>::launch(ch, G.st, Gc, desc, G.pl.K, P, R, minv, Q, b->part, cg)) {
                    hipGraph_t dropped = nullptr;
                    (void)hipStreamEndCapture(G.st, &dropped);
                    if (dropped) (void)hipGraphDestroy(dropped);
                    return e;
                }
                k_fin_spmm<KB><<<KB, WG, 0, G.st>>>(b->grid_win, b->part, cg);
                if constexpr (std::is_same<T, double>::value) {  // with the index estimates of the eager path
                    k_update_batched<T, KB, true><<<b->grid_vec, WG, 0, G.st>>>(n, X, R, P, Q, minv, b->S, KB, KB,
                                                                               b->part, cg);
                    k_fin_update_batched<KB, true><<<KB, WG, 0, G.st>>>(b->grid_vec, n, b->part, cg);
                } else {
                    k_update_batched<T, KB, false><<<b->grid_vec, WG, 0, G.st>>>(n, X, R, P, Q, minv, nullptr, 0, 0,
                                                                                b->part, cg);
                    k_fin_update_batched<KB, false><<<KB, WG, 0, G.st>>>(b->grid_vec, n, b->part, cg);
                }
            }
            HIPCHK(hipStreamEndCapture(G.st, &b->graph));
            HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            return FJ_OK;
        });
    }

    // Admit columns j0 .. j0 + m - 1 of request r into free slots of block b:
    // scatter them into S, start their CG (masked), leave the other columns
    // untouched. A request may enter in pieces as slots free up.
    static int admit(Server& s, ServerGraph& G, ServerBlock* b, ServerRequest& r, int j0, int m) {
        SlotMap map{};
        uint64_t mask = 0;
        int got = 0;
        for (int c = 0; c < KB && got < m; ++c) {
            if (b->slot_req[c] < 0) {
                map.slot[got] = c;
                b->slot_req[c] = static_cast<int64_t>(r.id);
                b->slot_col[c] = j0 + got;
                b->rtol[c] = s.o.eps * 1e-2;
                b->tau[c] = 1e-4;
                b->prev_rho[c] = INFINITY;
                b->outer[c] = 0;
                b->inner_total[c] = 0;
                mask |= 1ull << c;
                ++got;
            }
        }
        const int n = G.g.n;
        k_scatter_columns<<<b->grid_vec, WG, 0, G.st>>>(n, m, r.S + j0, r.lds, map, b->S, KB);
        HIPCHK(hipGetLastError());
        k_ctrl_reset_masked<<<1, WG, 0, G.st>>>(b->ctrl, KB, mask);
        HIPCHK(hipGetLastError());
        if (b->mixed) {
            k_ctrl_reset_masked<<<1, WG, 0, G.st>>>(b->ictrl, KB, mask);
            HIPCHK(hipGetLastError());
        }
        return start(s, G, b, mask, 0);
    }

    // Masked start (mode 0 fresh from S, mode 1 restart from the true
    // residual). FP64: a CG pass to relative residual rtol. FJ_MIXED: mode 0
    // also sets z = 0, r = s and the statistics of s (outer control blocks,
    // with ||r|| = ||s|| recorded for the scaling); then an inner FP32 CG on
    // r / ||r|| to tau. The CG passes start from the column means and are
    // deflated, as in the eager path.
    static int start(Server& s, ServerGraph& G, ServerBlock* b, uint64_t mask, int mode) {
        const int n = G.g.n;
        const float* minv = reinterpret_cast<const float*>(static_cast<const char*>(G.plan) + G.pl.minv);
        const int max_iter = s.o.max_iter > 0 ? s.o.max_iter : 2000;
        const bool deflate = true;
        ColumnTol tol{};
        if (!b->mixed) {
            for (int c = 0; c < KB; ++c) tol.rtol2[c] = b->rtol[c] * b->rtol[c];
            k_init_batched<double, KB><<<b->grid_vec, WG, 0, G.st>>>(n, KB, b->S, KB, b->X, b->R, b->P, minv, mode,
                                                                    mask, KB, b->part, b->ctrl);
            HIPCHK(hipGetLastError());
            // the first pass may stop on the index estimates, as the eager path does
            const double eps_stop = mode == 0 ? 0.8 * s.o.eps : 0.0;
            k_fin_init_batched<KB><<<KB, WG, 0, G.st>>>(b->grid_vec, n, KB, b->part, mode, mask, tol, max_iter, 1,
                                                        b->ctrl, 0, eps_stop, (deflate && mode == 1) ? 1 : 0);
            HIPCHK(hipGetLastError());
            if (deflate && mode == 0) {
                k_init_batched<double, KB><<<b->grid_vec, WG, 0, G.st>>>(n, KB, nullptr, 0, b->X, b->R, b->P, minv, 3,
                                                                        mask, 0, b->part, b->ctrl);
                HIPCHK(hipGetLastError());
                k_fin_init_batched<KB><<<KB, WG, 0, G.st>>>(b->grid_vec, n, KB, b->part, 3, mask, tol, max_iter, 1,
                                                            b->ctrl, 0, eps_stop, 1);
                HIPCHK(hipGetLastError());
            }
            b->running |= mask;
            return FJ_OK;
        }
        if (mode == 0) {
            for (int c = 0; c < KB; ++c) tol.rtol2[c] = 1.0;
            k_init_batched<double, KB><<<b->grid_vec, WG, 0, G.st>>>(n, KB, b->S, KB, b->X, b->R, nullptr, minv, 0,
                                                                    mask, KB, b->part, b->ctrl);
            HIPCHK(hipGetLastError());
            k_fin_init_batched<KB><<<KB, WG, 0, G.st>>>(b->grid_vec, n, KB, b->part, 0, mask, tol, max_iter, 1, b->ctrl,
                                                        0, 0.0, 0);
            HIPCHK(hipGetLastError());
            k_ctrl_rho_from_s<<<1, WG, 0, G.st>>>(b->ctrl, KB, mask);
            HIPCHK(hipGetLastError());
        }
        k_mixed_cast_batched<KB><<<b->grid_vec, WG, 0, G.st>>>(n, b->R, b->R32, 1, mask, b->ctrl, 0);
        HIPCHK(hipGetLastError());
        for (int c = 0; c < KB; ++c) tol.rtol2[c] = b->tau[c] * b->tau[c];
        k_init_batched<float, KB><<<b->grid_vec, WG, 0, G.st>>>(n, KB, nullptr, 0, b->X32, b->R32, b->P32, minv, 2,
                                                               mask, 0, b->part, b->ictrl);
        HIPCHK(hipGetLastError());
        k_fin_init_batched<KB><<<KB, WG, 0, G.st>>>(b->grid_vec, n, KB, b->part, 2, mask, tol, max_iter, 0, b->ictrl,
                                                    0, 0.0, 0);
        HIPCHK(hipGetLastError());
        if (deflate) {
            k_init_batched<float, KB><<<b->grid_vec, WG, 0, G.st>>>(n, KB, nullptr, 0, b->X32, b->R32, b->P32, minv,
                                                                   3, mask, 0, b->part, b->ictrl);
            HIPCHK(hipGetLastError());
            k_fin_init_batched<KB><<<KB, WG, 0, G.st>>>(b->grid_vec, n, KB, b->part, 3, mask, tol, max_iter, 0,
                                                        b->ictrl, 0, 0.0, 1);
            HIPCHK(hipGetLastError());
        }
        b->running |= mask;
        return FJ_OK;
    }

    static int epilogue(ServerGraph& G, ServerBlock* b) {
        if (b->mixed) {  // z += ||r|| d for the finishing columns
            k_mixed_refine_batched<KB><<<b->grid_vec, WG, 0, G.st>>>(G.g.n, b->X, b->X32, 1, b->finishing, b->ctrl);
            HIPCHK(hipGetLastError());
        }
        int rc = with_graph(&G.g, [&](auto Gc) -> int {
            using Vc = typename decltype(Gc)::value_type;
            int grid = 1;
            if (int e = grid_for(k_epilogue_batched<Vc, KB>, G.pl.K, &grid)) return e;
            const WinDesc* desc = reinterpret_cast<const WinDesc*>(static_cast<const char*>(G.plan) + G.pl.desc);
            k_epilogue_batched<Vc, KB><<<grid, WG, 0, G.st>>>(Gc, desc, G.pl.K, KB, b->finishing, b->X, b->S, KB, b->R,
                                                              b->part, b->ctrl);
            HIPCHK(hipGetLastError());
            k_fin_epilogue_batched<KB><<<KB, WG, 0, G.st>>>(grid, G.g.n, b->finishing, b->part, b->ctrl);
            HIPCHK(hipGetLastError());
            return FJ_OK;
        });
        return rc;
    }

    static int snapshot(ServerGraph& G, ServerBlock* b) {
        HIPCHK(hipMemcpyAsync(b->host, b->ctrl, sizeof(Ctrl) * KB, hipMemcpyDeviceToHost, G.st));
        if (b->mixed)
            HIPCHK(hipMemcpyAsync(b->host + KB, b->ictrl, sizeof(Ctrl) * KB, hipMemcpyDeviceToHost, G.st));
        HIPCHK(hipEventRecord(b->ev, G.st));
        return FJ_OK;
    }

    static void finish_column(Server& s, ServerBlock* b, int c, int status) {
        const uint64_t rid = static_cast<uint64_t>(b->slot_req[c]);
        auto it = s.requests.find(rid);
        b->slot_req[c] = -1;
        if (it == s.requests.end()) return;
        ServerRequest& r = it->second;
        const int j = b->slot_col[c];
        Ctrl cc = b->host[c];
        if (b->mixed) cc.iters = b->inner_total[c];
        fill_outputs(cc, status, 0, b->mixed ? b->outer[c] : 0, r.out ? r.out + j : nullptr,
                     r.info ? r.info + j : nullptr);
        if (status != FJ_OK && r.status == FJ_OK) r.status = status;
        if (--r.remaining == 0) {
            r.t_done = std::chrono::steady_clock::now();
            s.completed.push_back(rid);
        }
    }

    // One non-blocking scheduling step for graph G. Sets *busy when the
    // block still has GPU work in flight.
    static int step(Server& s, ServerGraph& G, bool* busy) {
        ServerBlock* b = G.blk;
        if (b->phase != Phase::IDLE) {
            const hipError_t q = hipEventQuery(b->ev);
            if (q == hipErrorNotReady) {
                *busy = true;
                return FJ_OK;
            }
            if (q != hipSuccess) {
                set_error("hipEventQuery", q);
                return FJ_ERR_HIP;
            }
            if (b->phase == Phase::REPLAY) {
                uint64_t bad = 0;
                for (int c = 0; c < KB; ++c) {
                    if (!((b->running >> c) & 1ull)) continue;
                    const Ctrl& cg = b->mixed ? b->host[KB + c] : b->host[c];
                    const int d = b->host[c].done == BAD_INPUT ? BAD_INPUT : cg.done;
                    if (d == RUNNING && cg.iters < cg.max_iter) continue;
                    b->running &= ~(1ull << c);
                    if (b->mixed) b->inner_total[c] += cg.iters;
                    if (d == BAD_INPUT) {
                        finish_column(s, b, c, FJ_ERR_OPINION_RANGE);
                        bad |= 1ull << c;
                    } else if (d == BREAKDOWN) {
                        finish_column(s, b, c, FJ_ERR_BREAKDOWN);
                    } else {
                        b->finishing |= 1ull << c;
                    }
                }
                if (bad && b->mixed) {  // stop the inner CG of rejected columns
                    k_ctrl_set_done<<<1, WG, 0, G.st>>>(b->ictrl, KB, bad, static_cast<int>(CONVERGED));
                    HIPCHK(hipGetLastError());
                }
            } else {  // EPILOGUE: certify, retire or restart the finishing columns
                const int max_iter = s.o.max_iter > 0 ? s.o.max_iter : 2000;
                uint64_t again = 0;
                for (int c = 0; c < KB; ++c) {
                    if (!((b->finishing >> c) & 1ull)) continue;
                    const Ctrl& cc = b->host[c];
                    const double rho = cc.res[5], snorm = cc.res[6];
                    if (b->mixed) ++b->outer[c];
                    const bool capped = b->mixed ? (b->inner_total[c] >= max_iter || b->outer[c] >= 8)
                                                 : (cc.done == ITER_CAP || cc.iters >= cc.max_iter);
                    if (certified(cc, s.o.eps)) {
                        finish_column(s, b, c, FJ_OK);
                    } else if (capped) {
                        finish_column(s, b, c, FJ_ERR_NOT_CONVERGED);
                    } else if (!(rho < 0.5 * (b->mixed && std::isinf(b->prev_rho[c]) ? snorm : b->prev_rho[c]))) {
                        finish_column(s, b, c, stalled_status(cc, true));
                    } else {
                        b->prev_rho[c] = rho;
                        if (b->mixed) {
                            b->tau[c] = std::min(1e-2, std::max(1e-5, 0.5 * needed_rho(cc, s.o.eps) / rho));
                        } else {
                            double next = b->rtol[c] * 0.1;
                            if (snorm > 0.0) next = std::min(next, 0.5 * needed_rho(cc, s.o.eps) / snorm);
                            b->rtol[c] = std::max(next, 1e-16);
                        }
                        again |= 1ull << c;
                    }
                }
                b->finishing = 0;
                if (again)
                    if (int rc = start(s, G, b, again, 1)) return rc;
            }
            b->phase = Phase::IDLE;
        }
        // admit waiting columns of this graph into free slots, in arrival order
        while (!G.queue.empty()) {
            ServerRequest& r = s.requests[G.queue.front()];
            int free_slots = 0;
            for (int c = 0; c < KB; ++c) free_slots += b->slot_req[c] < 0;
            const int m = std::min(free_slots, r.k - r.admitted);
            if (m <= 0) break;
            if (int rc = admit(s, G, b, r, r.admitted, m)) return rc;
            r.admitted += m;
            if (r.admitted < r.k) break;  // the block is full
            G.queue.pop_front();
        }
        if (b->finishing) {
            if (int rc = epilogue(G, b)) return rc;
            if (int rc = snapshot(G, b)) return rc;
            b->phase = Phase::EPILOGUE;
            *busy = true;
        } else if (b->running) {
            HIPCHK(hipGraphLaunch(b->exec, G.st));
            if (int rc = snapshot(G, b)) return rc;
            b->phase = Phase::REPLAY;
            *busy = true;
        }
        return FJ_OK;
    }

    static bool empty(const ServerBlock* b) {
        if (b->running || b->finishing || b->phase != Phase::IDLE) return false;
        for (int c = 0; c < KB; ++c)
            if (b->slot_req[c] >= 0) return false;
        return true;
    }
};

int release_block(Server& s, ServerGraph& G) {
    ServerBlock* b = G.blk;
    HIPCHK(hipStreamSynchronize(G.st));
    if (b->exec) HIPCHK(hipGraphExecDestroy(b->exec));
    if (b->graph) HIPCHK(hipGraphDestroy(b->graph));
    if (b->ev) HIPCHK(hipEventDestroy(b->ev));
    if (b->host) HIPCHK(hipHostFree(b->host));
    arena_free(s, b->offset, b->bytes);
    delete b;
    G.blk = nullptr;
    return FJ_OK;
}

// Blocks stay allocated (with their captured graph) while idle, so a graph
// that keeps receiving requests pays the block set-up once. A graph with
// waiting requests and no block first takes free arena space, then releases
// idle blocks of other graphs, least recently used first.
template <int KB>
int server_step_kb(Server& s, int* busy_out) {
    int busy_blocks = 0;
    ++s.tick;
    for (auto& G : s.graphs) {
        if (!G.blk) {
            if (G.queue.empty()) continue;
            const size_t bytes = block_bytes(G.g.n, KB, s.o.precision == FJ_MIXED);
            size_t off = 0;
            bool got = arena_alloc(s, bytes, &off);
            while (!got) {
                ServerGraph* victim = nullptr;
                for (auto& H : s.graphs)
                    if (H.blk && &H != &G && H.queue.empty() && ServerOps<KB>::empty(H.blk) &&
                        (!victim || H.blk->last_used < victim->blk->last_used))
                        victim = &H;
                if (!victim) break;  // waits for HBM
                if (int rc = release_block(s, *victim)) return rc;
                got = arena_alloc(s, bytes, &off);
            }
            if (!got) continue;
            G.blk = new ServerBlock();
            G.blk->offset = off;
            G.blk->bytes = bytes;
            if (int rc = ServerOps<KB>::create(s, G, G.blk)) return rc;
        }
        bool busy = false;
        if (int rc = ServerOps<KB>::step(s, G, &busy)) return rc;
        if (busy || !ServerOps<KB>::empty(G.blk)) G.blk->last_used = s.tick;
        if (busy) ++busy_blocks;
    }
    *busy_out = busy_blocks;
    return FJ_OK;
}
