// fj_server.hpp -- continuous-batching server for FJ index requests (host side).
// Included by fj_api.hip inside its anonymous namespace; the extern "C" entry
// points are defined there.
//
// Graphs stay resident (CSR and plan owned by the caller). A graph with work
// gets a block: the CG state of KB columns (X, R, P, Q, the opinion block S,
// partials, KB control blocks) carved from a caller-provided HBM arena by a
// first-fit allocator; a graph whose block does not fit waits until another
// block is released (admission by HBM footprint). A request (graph, k
// opinion vectors) is admitted when k columns of its graph's block are free,
// at an iteration boundary, while the other columns keep iterating. Each
// block replays a HIP graph of `iters` captured CG iterations on its own
// stream, so blocks of different graphs overlap on the device. After each
// replay the host reads the KB control blocks; columns that stopped are
// finished by the batched epilogue (indices, certificate), then either
// retired (certified, or final) or restarted from their true residual with a
// tighter target. A column's arithmetic never depends on the other columns
// of its block, so a result is bitwise the same alone or in the mix.
#pragma once

#include <chrono>
#include <unordered_map>

struct ServerRequest {
    uint64_t id = 0;
    int gid = 0;
    int k = 0;
    const double* S = nullptr;
    int64_t lds = 0;
    fj_indices_t* out = nullptr;  // host, k entries
    fj_info* info = nullptr;      // host, k entries (may be null)
    int slots[KMAX] = {};
    int remaining = 0;
    int status = FJ_OK;
    std::chrono::steady_clock::time_point t_submit, t_done;
};

enum class Phase { IDLE, REPLAY, EPILOGUE };

struct ServerBlock {
    size_t offset = 0, bytes = 0;
    double *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr, *S = nullptr;
    Ctrl* ctrl = nullptr;
    double* part = nullptr;
    Ctrl* host = nullptr;  // pinned copy of the control blocks
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t slot_req[KMAX];
    double rtol[KMAX];
    double prev_rho[KMAX];
    uint64_t running = 0, finishing = 0;
    Phase phase = Phase::IDLE;
    int grid_win = 1, grid_vec = 1;
};

struct ServerGraph {
    fj_csr g{};
    const void* plan = nullptr;
    PlanLayout pl{};
    hipStream_t st = nullptr;
    std::deque<uint64_t> queue;
    ServerBlock* blk = nullptr;
};

struct Server {
    fj_server_opts o{};
    char* arena = nullptr;
    std::map<size_t, size_t> free_list;  // offset -> bytes
    std::vector<ServerGraph> graphs;
    std::unordered_map<uint64_t, ServerRequest> requests;
    std::deque<uint64_t> completed;
    uint64_t next_id = 1;
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

size_t block_bytes(int n, int kb) {
    const size_t v = align_up(sizeof(double) * static_cast<size_t>(n) * kb);
    return 5 * v + align_up(sizeof(double) * GMAX * BPART * kb) + align_up(sizeof(Ctrl) * kb);
}

// ------------------------------------------------------------ per-KB machinery

template <int KB>
struct ServerOps {
    static constexpr uint64_t ALL = KB >= 64 ? ~0ull : ((1ull << KB) - 1ull);

    static int create(Server& s, ServerGraph& G, ServerBlock* b) {
        const int n = G.g.n;
        char* base = s.arena + b->offset;
        const size_t v = align_up(sizeof(double) * static_cast<size_t>(n) * KB);
        b->X = reinterpret_cast<double*>(base);
        b->R = reinterpret_cast<double*>(base + v);
        b->P = reinterpret_cast<double*>(base + 2 * v);
        b->Q = reinterpret_cast<double*>(base + 3 * v);
        b->S = reinterpret_cast<double*>(base + 4 * v);
        b->part = reinterpret_cast<double*>(base + 5 * v);
        b->ctrl = reinterpret_cast<Ctrl*>(base + 5 * v + align_up(sizeof(double) * GMAX * BPART * KB));
        for (int c = 0; c < KMAX; ++c) {
            b->slot_req[c] = -1;
            b->rtol[c] = 0.0;
            b->prev_rho[c] = INFINITY;
        }
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&b->host), sizeof(Ctrl) * KB, hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming));
        const int64_t units = (static_cast<int64_t>(n) * KB + WG - 1) / WG;
        if (int rc = grid_for(k_update_batched<double, KB>, units, &b->grid_vec)) return rc;
        // zero the block (kernels, not memsets), every column idle
        const int64_t words = static_cast<int64_t>(5 * v / sizeof(double));
        k_fill_zero<<<b->grid_vec, WG, 0, G.st>>>(b->X, words);
        HIPCHK(hipGetLastError());
        k_ctrl_reset<<<1, WG, 0, G.st>>>(b->ctrl, KB);
        HIPCHK(hipGetLastError());
        k_ctrl_set_done<<<1, WG, 0, G.st>>>(b->ctrl, KB, ALL, static_cast<int>(CONVERGED));
        HIPCHK(hipGetLastError());
        // capture `iters` CG iterations of the block
        int rc = with_graph(&G.g, [&](auto Gc) -> int {
            using Vc = typename decltype(Gc)::value_type;
            const WinDesc* desc = reinterpret_cast<const WinDesc*>(static_cast<const char*>(G.plan) + G.pl.desc);
            const float* minv = reinterpret_cast<const float*>(static_cast<const char*>(G.plan) + G.pl.minv);
            // the same tuned launch shape as the eager batched path of this graph and width
            SpmmChoice ch{};
            if (int e = Spmm<Vc, double, KB>::choose(&G.g, G.st, Gc, desc, G.pl.K, b->P, b->R, minv, b->Q, b->part,
                                                     true, &ch))
                return e;
            b->grid_win = ch.grid;
            HIPCHK(hipStreamBeginCapture(G.st, hipStreamCaptureModeThreadLocal));
            for (int t = 0; t < s.o.iters_per_replay; ++t) {
                if (int e = Spmm<Vc, double, KB>::launch(ch, G.st, Gc, desc, G.pl.K, b->P, b->R, minv, b->Q, b->part)) {
                    hipGraph_t dropped = nullptr;
                    (void)hipStreamEndCapture(G.st, &dropped);
                    if (dropped) (void)hipGraphDestroy(dropped);
                    return e;
                }
                k_fin_spmm<KB><<<KB, WG, 0, G.st>>>(b->grid_win, b->part, b->ctrl);
                k_update_batched<double, KB><<<b->grid_vec, WG, 0, G.st>>>(n, b->X, b->R, b->P, b->Q, minv, b->part,
                                                                          b->ctrl);
                k_fin_update_batched<KB><<<KB, WG, 0, G.st>>>(b->grid_vec, b->part, b->ctrl);
            }
            HIPCHK(hipStreamEndCapture(G.st, &b->graph));
            HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            return FJ_OK;
        });
        return rc;
    }

    // Admit request r into free slots of block b: scatter its columns into S,
    // start their CG (masked), leave the other columns untouched.
    static int admit(Server& s, ServerGraph& G, ServerBlock* b, ServerRequest& r) {
        SlotMap map{};
        uint64_t mask = 0;
        int got = 0;
        for (int c = 0; c < KB && got < r.k; ++c) {
            if (b->slot_req[c] < 0) {
                map.slot[got] = c;
                r.slots[got] = c;
                b->slot_req[c] = static_cast<int64_t>(r.id);
                b->rtol[c] = s.o.eps * 1e-2;
                b->prev_rho[c] = INFINITY;
                mask |= 1ull << c;
                ++got;
            }
        }
        r.remaining = r.k;
        const int n = G.g.n;
        k_scatter_columns<<<b->grid_vec, WG, 0, G.st>>>(n, r.k, r.S, r.lds, map, b->S, KB);
        HIPCHK(hipGetLastError());
        k_ctrl_reset_masked<<<1, WG, 0, G.st>>>(b->ctrl, KB, mask);
        HIPCHK(hipGetLastError());
        return start(s, G, b, mask, 0);
    }

    // Masked CG start (mode 0 fresh from S, mode 1 restart from the true residual).
    static int start(Server& s, ServerGraph& G, ServerBlock* b, uint64_t mask, int mode) {
        const int n = G.g.n;
        const float* minv = reinterpret_cast<const float*>(static_cast<const char*>(G.plan) + G.pl.minv);
        ColumnTol tol{};
        for (int c = 0; c < KB; ++c) tol.rtol2[c] = b->rtol[c] * b->rtol[c];
        k_init_batched<double, KB><<<b->grid_vec, WG, 0, G.st>>>(n, KB, b->S, KB, b->X, b->R, b->P, minv, mode, mask,
                                                                KB, b->part);
        HIPCHK(hipGetLastError());
        const int max_iter = s.o.max_iter > 0 ? s.o.max_iter : 2000;
        k_fin_init_batched<KB><<<KB, WG, 0, G.st>>>(b->grid_vec, n, KB, b->part, mode, mask, tol, max_iter, 1, b->ctrl);
        HIPCHK(hipGetLastError());
        b->running |= mask;
        return FJ_OK;
    }

    static int epilogue(ServerGraph& G, ServerBlock* b) {
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
        HIPCHK(hipEventRecord(b->ev, G.st));
        return FJ_OK;
    }

    static void finish_column(Server& s, ServerBlock* b, int c, int status) {
        const uint64_t rid = static_cast<uint64_t>(b->slot_req[c]);
        auto it = s.requests.find(rid);
        b->slot_req[c] = -1;
        if (it == s.requests.end()) return;
        ServerRequest& r = it->second;
        int j = 0;
        while (j < r.k && r.slots[j] != c) ++j;
        const Ctrl& cc = b->host[c];
        fill_outputs(cc, status, 0, 0, r.out ? r.out + j : nullptr, r.info ? r.info + j : nullptr);
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
                for (int c = 0; c < KB; ++c) {
                    if (!((b->running >> c) & 1ull)) continue;
                    const int d = b->host[c].done;
                    if (d == RUNNING && b->host[c].iters < b->host[c].max_iter) continue;
                    b->running &= ~(1ull << c);
                    if (d == BAD_INPUT) finish_column(s, b, c, FJ_ERR_OPINION_RANGE);
                    else if (d == BREAKDOWN) finish_column(s, b, c, FJ_ERR_BREAKDOWN);
                    else b->finishing |= 1ull << c;
                }
            } else {  // EPILOGUE: certify, retire or restart the finishing columns
                uint64_t again = 0;
                for (int c = 0; c < KB; ++c) {
                    if (!((b->finishing >> c) & 1ull)) continue;
                    const Ctrl& cc = b->host[c];
                    const double rho = cc.res[5], snorm = cc.res[6];
                    if (certified(cc, s.o.eps)) {
                        finish_column(s, b, c, FJ_OK);
                    } else if (cc.done == ITER_CAP || cc.iters >= cc.max_iter) {
                        finish_column(s, b, c, FJ_ERR_NOT_CONVERGED);
                    } else if (!(rho < 0.5 * b->prev_rho[c])) {
                        finish_column(s, b, c, stalled_status(cc, true));
                    } else {
                        b->prev_rho[c] = rho;
                        double next = b->rtol[c] * 0.1;
                        if (snorm > 0.0) next = std::min(next, 0.5 * needed_rho(cc, s.o.eps) / snorm);
                        b->rtol[c] = std::max(next, 1e-16);
                        again |= 1ull << c;
                    }
                }
                b->finishing = 0;
                if (again)
                    if (int rc = start(s, G, b, again, 1)) return rc;
            }
            b->phase = Phase::IDLE;
        }
        // admit waiting requests of this graph into free slots
        while (!G.queue.empty()) {
            ServerRequest& r = s.requests[G.queue.front()];
            int free_slots = 0;
            for (int c = 0; c < KB; ++c) free_slots += b->slot_req[c] < 0;
            if (free_slots < r.k) break;
            G.queue.pop_front();
            if (int rc = admit(s, G, b, r)) return rc;
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

template <int KB>
int server_step_kb(Server& s, int* busy_out) {
    int busy_blocks = 0;
    for (auto& G : s.graphs) {
        if (!G.blk) {
            if (G.queue.empty()) continue;
            const size_t bytes = block_bytes(G.g.n, KB);
            size_t off = 0;
            if (!arena_alloc(s, bytes, &off)) continue;  // waits for HBM
            G.blk = new ServerBlock();
            G.blk->offset = off;
            G.blk->bytes = bytes;
            if (int rc = ServerOps<KB>::create(s, G, G.blk)) return rc;
        }
        bool busy = false;
        if (int rc = ServerOps<KB>::step(s, G, &busy)) return rc;
        if (busy) ++busy_blocks;
        else if (ServerOps<KB>::empty(G.blk) && G.queue.empty())
            if (int rc = release_block(s, G)) return rc;
    }
    *busy_out = busy_blocks;
    return FJ_OK;
}
