// fj_phased.hpp -- the time-phased entry layout of I + L and its SpMV (HIP,
// gfx950). Part of fj_api.hip's translation unit (included once).
//
// On a graph without locality (Chung-Lu, expander-like) every CSR-order row
// gathers x_j from all over the vector, and a vector larger than one XCD's
// 4 MB L2 misses on about half of those gathers: the window pass runs at the
// rate of L2 line fills from the Infinity Cache, not at HBM bandwidth. This
// layout orders the gathers in time instead:
//
//   * The rows are dealt to W wave-chunks (longest-processing-time first over
//     16-row blocks, so that every chunk holds about nnz / W entries and at
//     most 1248 or 1600 rows). A chunk belongs to one wave, which keeps the
//     chunk's row sums in LDS.
//   * The columns are cut into P phases of PH_PHASE_NODES nodes (1 MB of an
//     FP64 vector). A chunk's entries are stored phase by phase, each phase's
//     entries by local row, and each (chunk, phase) group is padded to a
//     multiple of 8 entries (padding: column 0, weight 0, key PH_SENT).
//   * Every wave walks its chunk phase by phase. All chunks are resident at
//     once and hold about the same entries per phase, so the whole chip
//     moves through the phases together and each XCD's L2 holds the current
//     phase of x: the gathers hit L2.
//
// Within a phase a wave takes 512 entries at a time, 8 consecutive entries
// per lane. A lane sums the runs of equal local row in its 8 entries, adds
// the runs that start and end inside them to LDS, and keeps its first and
// last run; one segmented scan over the 64 lanes joins the runs that cross
// lanes, and every row's run is added to LDS exactly once, by one lane, in a
// fixed order. The result is deterministic. The row sum is the raw
// sum_j w_ij x_j; with the weighted degree d_i of the row,
// ((I + L) x)_i = x_i + d_i x_i - sum_j w_ij x_j.
#pragma once

#include <algorithm>
#include <queue>
#include <type_traits>
#include <vector>

#include "fj_guard.hpp"
#include "fj_kernels.hpp"

namespace fj {

#define PH_HIPCHK(call)                                                                           \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            std::snprintf(g_last_error, sizeof g_last_error, "%s: %s", #call, hipGetErrorString(e_)); \
            return FJ_ERR_HIP;                                                                    \
        }                                                                                         \
    } while (0)

// Two chunk geometries: rows per wave-chunk (their sums live in LDS) and the
// chunk count up to which every chunk is resident at once.
//   short: 1248 rows, four workgroups (16 waves) per CU, up to 4096 chunks.
//     For graphs whose chunks hold less than one 512-entry window per phase:
//     the walk waits on gather latency, and more waves hide more of it.
//   long: 1600 rows, three workgroups (12 waves) per CU, up to 3072 chunks.
//     For the others: the walk is bound by the gather rate, and fewer
//     outstanding misses per CU gather faster (4M-node Chung-Lu graph:
//     0.67 against 0.85 ms per SpMV).
constexpr int PH_RMAX_SHORT = 1248, PH_WMAX_SHORT = 4096;
constexpr int PH_RMAX_LONG = 1600, PH_WMAX_LONG = 3072;
static_assert(NWAVE * PH_RMAX_SHORT * sizeof(double) + NWAVE * 4 * sizeof(double) <= 160 * 1024 / 4,
              "short chunks: four workgroups per CU");
static_assert(NWAVE * PH_RMAX_LONG * sizeof(double) + NWAVE * 4 * sizeof(double) <= 160 * 1024 / 3,
              "long chunks: three workgroups per CU");
constexpr int PH_PHASE_NODES = 131072;   // columns per phase
// One-vector solves and FJ steps use the layout from this many nodes on (the
// 2x2-block CG's threshold): certified solves on graphs of 100K to 1M nodes
// (Chung-Lu, Barabasi-Albert, weights spread over 1e6) took 6-32 % less time
// than on the row windows; on a 10K-node graph the two were level.
constexpr int PH_MIN_N = 65536;
constexpr int PH_BLOCK = 16;             // rows dealt together
constexpr int PH_SINGLE_ABOVE = 2048;    // a 16-row block with more entries is dealt row by row
constexpr unsigned PH_SENT = 0xFFFFu;    // key of a padding entry
constexpr int PH_PMAX = 2048;            // most phases (the placement keeps a cursor per phase in LDS)

struct PhasedShape {
    int rmax = PH_RMAX_SHORT;  // rows per chunk at most (PH_RMAX_SHORT or PH_RMAX_LONG)
    int W = 0;          // wave-chunks (a multiple of 4)
    int P = 0;          // phases
    int width = 1;      // columns per phase
    int64_t nnzp = 0;   // entry slots reserved: nnz + 7 W P (the most padding can take)
    bool ok = false;    // the layout exists for this graph
};

inline PhasedShape phased_shape(int n, int64_t nnz) {
    PhasedShape s;
    if (n < 1) return s;
    s.P = static_cast<int>((static_cast<int64_t>(n) + PH_PHASE_NODES - 1) / PH_PHASE_NODES);
    s.width = static_cast<int>((static_cast<int64_t>(n) + s.P - 1) / s.P);
    // about 256 rows per chunk but up to 1024 chunks (at least 64 rows each)
    // so that mid-size graphs still give every CU a workgroup, at most wmax
    // chunks, unless that leaves chunks of more than rmax / 1.2 rows on
    // average (room for the deal)
    auto chunks = [&](int rmax, int wmax) {
        const int64_t nn = n;
        const int64_t by_rows = (nn * 6 + 5 * rmax - 1) / (5 * rmax);
        const int64_t spread = std::max<int64_t>((nn + 255) / 256, std::min<int64_t>(1024, (nn + 63) / 64));
        const int64_t W = std::max<int64_t>(by_rows, std::min<int64_t>(wmax, spread));
        return std::max<int64_t>(4, (W + 3) / 4 * 4);
    };
    int64_t W = chunks(PH_RMAX_SHORT, PH_WMAX_SHORT);
    if (nnz >= 512 * W * s.P) {  // a full window per chunk and phase: long chunks
        s.rmax = PH_RMAX_LONG;
        W = chunks(PH_RMAX_LONG, PH_WMAX_LONG);
    }
    s.W = static_cast<int>(W);
    s.nnzp = nnz + 7 * W * s.P;
    s.ok = s.nnzp < INT32_MAX && W * (s.P + 1) < INT32_MAX && s.P <= PH_PMAX;
    return s;
}

template <typename V>
struct PhasedCsr {
    int W, P;
    const int* __restrict__ ps;              // entry offset of (chunk c, phase k) at c (P + 1) + k
    const int* __restrict__ col;
    const V* __restrict__ val;
    const unsigned short* __restrict__ key;  // local row of each entry, PH_SENT for padding
    const int* __restrict__ rs;              // first local row slot of each chunk (W + 1)
    const int* __restrict__ row;             // node of each row slot
    const double* __restrict__ deg;          // weighted degree of each row slot
};

typedef int ph_iv4 __attribute__((ext_vector_type(4)));
typedef float ph_fv4 __attribute__((ext_vector_type(4)));
typedef double ph_dv2 __attribute__((ext_vector_type(2)));
typedef unsigned ph_uv4 __attribute__((ext_vector_type(4)));

template <typename V>
__device__ __forceinline__ void ph_weights(const V* __restrict__ val, int i0, double (&w)[8]);
template <>
__device__ __forceinline__ void ph_weights<Unit>(const Unit* __restrict__, int, double (&w)[8]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = 1.0;
}
template <>
__device__ __forceinline__ void ph_weights<float>(const float* __restrict__ val, int i0, double (&w)[8]) {
    const ph_fv4 a = __builtin_nontemporal_load(reinterpret_cast<const ph_fv4*>(val + i0));
    const ph_fv4 b = __builtin_nontemporal_load(reinterpret_cast<const ph_fv4*>(val + i0) + 1);
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
}
template <>
__device__ __forceinline__ void ph_weights<double>(const double* __restrict__ val, int i0, double (&w)[8]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const ph_dv2 a = __builtin_nontemporal_load(reinterpret_cast<const ph_dv2*>(val + i0) + m);
        w[2 * m] = a.x;
        w[2 * m + 1] = a.y;
    }
}

// Row sums sum_j w_ij x_j of chunk c into a[0 .. rows of c), by one wave.
template <typename V, typename T>
__device__ __forceinline__ void ph_chunk_sums(const PhasedCsr<V>& g, int c, const T* __restrict__ x,
                                              double* a, int lane) {
    const int r0 = g.rs[c], nr = g.rs[c + 1] - r0;
    for (int r = lane; r < nr; r += 64) a[r] = 0.0;
    const int* pc = g.ps + static_cast<int64_t>(c) * (g.P + 1);
    int s = pc[0];
    for (int k = 0; k < g.P; ++k) {
        const int e = pc[k + 1];
        for (int base = s; base < e; base += 512) {
            const int i0 = base + lane * 8;
            const bool act = i0 < e;
            int j[8];
            double w[8];
            unsigned kk[8];
            if (act) {
                const ph_iv4 c0 = __builtin_nontemporal_load(reinterpret_cast<const ph_iv4*>(g.col + i0));
                const ph_iv4 c1 = __builtin_nontemporal_load(reinterpret_cast<const ph_iv4*>(g.col + i0) + 1);
                const ph_uv4 kv = __builtin_nontemporal_load(reinterpret_cast<const ph_uv4*>(g.key + i0));
                ph_weights<V>(g.val, i0, w);
                j[0] = c0.x; j[1] = c0.y; j[2] = c0.z; j[3] = c0.w;
                j[4] = c1.x; j[5] = c1.y; j[6] = c1.z; j[7] = c1.w;
                kk[0] = kv.x & 0xFFFFu; kk[1] = kv.x >> 16; kk[2] = kv.y & 0xFFFFu; kk[3] = kv.y >> 16;
                kk[4] = kv.z & 0xFFFFu; kk[5] = kv.z >> 16; kk[6] = kv.w & 0xFFFFu; kk[7] = kv.w >> 16;
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    j[i] = 0;
                    w[i] = 0.0;
                    kk[i] = PH_SENT;
                }
            }
            double xv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) xv[i] = act ? static_cast<double>(x[j[i]]) : 0.0;
            // the lane's runs: the first (hv) is kept, inner runs go to LDS, the last is kept
            double run = w[0] * xv[0], hv = 0.0;
            unsigned cur = kk[0];
            bool multi = false;
#pragma unroll
            for (int i = 1; i < 8; ++i) {
                if (kk[i] != cur) {
                    if (!multi) {
                        hv = run;
                        multi = true;
                    } else if (cur != PH_SENT) {
                        a[cur] += run;
                    }
                    run = 0.0;
                    cur = kk[i];
                }
                run += w[i] * xv[i];
            }
            const unsigned hk = kk[0], tk = cur;
            if (!multi) hv = run;
            // lane l continues the last run of lane l - 1 when its first key is that run's key
            const unsigned tk_prev = __shfl_up(tk, 1, 64);
            const bool cont = lane > 0 && hk == tk_prev && hk != PH_SENT;
            // carry chain: a lane with one run that continues adds to the carry it receives
            double v = multi ? run : hv;
            bool f = multi || !cont;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const double vu = __shfl_up(v, d, 64);
                const int fu = __shfl_up(static_cast<int>(f), d, 64);
                if (lane >= d) {
                    if (!f) v = vu + v;
                    f = f || fu;
                }
            }
            const double carry_prev = __shfl_up(v, 1, 64);
            const double cin = cont ? carry_prev : 0.0;
            const int cn = __shfl_down(static_cast<int>(cont), 1, 64);
            const bool cont_next = lane < 63 && cn;
            if (multi && hk != PH_SENT) a[hk] += cin + hv;
            if (!cont_next) {
                if (multi) {
                    if (tk != PH_SENT) a[tk] += run;
                } else if (hk != PH_SENT) {
                    a[hk] += v;
                }
            }
        }
        s = e;
    }
}

// Every row of every chunk of this wave: op.row(i, x_i, lin, sq, op.load(i))
// as the window pass calls it, with lin = ((L x)_i) = d_i x_i - sum_j w_ij x_j
// (AccLin), or lin = sum_j w_ij x_j and sq = d_i (AccRaw).
template <typename V, typename T, typename Acc, typename Op>
__device__ __forceinline__ void ph_rows(const PhasedCsr<V>& g, const T* __restrict__ x, Op& op, double* a) {
    static_assert(!Acc::SQ && !Acc::DEG, "the phased pass forms linear row sums only");
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = blockIdx.x * NWAVE + wv; c < g.W; c += gridDim.x * NWAVE) {
        ph_chunk_sums<V, T>(g, c, x, a, lane);
        const int r0 = g.rs[c], nr = g.rs[c + 1] - r0;
        for (int r = lane; r < nr; r += 64) {
            const int i = g.row[r0 + r];
            const T xi = x[i];
            const double d = g.deg[r0 + r];
            if constexpr (Acc::RAW) op.row(i, xi, a[r], d, op.load(i));
            else op.row(i, xi, d * static_cast<double>(xi) - a[r], 0.0, op.load(i));
        }
    }
}

// q = (I + L) p - pbar and p^T q (partial slot 0), as k_cg_spmv_pq.
template <typename V, typename T, int RM>
__global__ void __launch_bounds__(WG) k_cg_spmv_pq_ph(PhasedCsr<V> g, const T* __restrict__ p, T* __restrict__ q,
                                                      double* __restrict__ part, const Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double acc[NWAVE][RM];
    __shared__ double red[NWAVE * 4];
    OpCgSpmvPq<T> op{q, ctrl->pbar};
    ph_rows<V, T, AccLin>(g, p, op, acc[threadIdx.x >> 6]);
    double v[1] = {op.pq};
    block_sum<1>(v, red);
    store_partials<1>(v, part);
}

// q = (I + L) p - pbar with p^T q, r^T M^{-1} q, q^T M^{-1} q (slots 0-2), as k_cg_spmv.
template <typename V, typename T, int RM>
__global__ void __launch_bounds__(WG) k_cg_spmv_ph(PhasedCsr<V> g, const T* __restrict__ p, const T* __restrict__ r,
                                                   const float* __restrict__ minv, T* __restrict__ q,
                                                   double* __restrict__ part, const Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double acc[NWAVE][RM];
    __shared__ double red[NWAVE * 4];
    OpCgSpmv<T> op{r, minv, q, ctrl->pbar};
    ph_rows<V, T, AccLin>(g, p, op, acc[threadIdx.x >> 6]);
    double v[3] = {op.pq, op.rmq, op.qmq};
    block_sum<3>(v, red);
    store_partials<3>(v, part);
}

// One FJ step and its largest change (slot 0), as k_fj_sweep.
template <typename V, int RM>
__global__ void __launch_bounds__(WG) k_fj_sweep_ph(PhasedCsr<V> g, const double* __restrict__ z,
                                                    const double* __restrict__ s, double* __restrict__ znext,
                                                    double* __restrict__ part, const Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double acc[NWAVE][RM];
    __shared__ double red[NWAVE];
    OpFj op{s, znext};
    ph_rows<V, double, AccRaw>(g, z, op, acc[threadIdx.x >> 6]);
    double m = wave_max(op.maxc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w) m = fmax(m, red[w]);
        part[blockIdx.x * NPART] = m;
    }
}

// y = (I + L) x
template <typename V, int RM>
__global__ void __launch_bounds__(WG) k_apply_ph(PhasedCsr<V> g, const double* __restrict__ x,
                                                 double* __restrict__ y) {
    __shared__ double acc[NWAVE][RM];
    OpApply op{y};
    ph_rows<V, double, AccLin>(g, x, op, acc[threadIdx.x >> 6]);
}

// ---------------------------------------------------------------- host build

// Where the layout lives in the plan (byte offsets).
struct PhasedPlan {
    PhasedShape s;
    size_t ps = 0, rs = 0, row = 0, deg = 0, key = 0, col = 0, val = 0;
};

template <typename V>
PhasedCsr<V> phased_view(const char* plan, const PhasedPlan& pp) {
    PhasedCsr<V> g;
    g.W = pp.s.W;
    g.P = pp.s.P;
    g.ps = reinterpret_cast<const int*>(plan + pp.ps);
    g.col = reinterpret_cast<const int*>(plan + pp.col);
    g.val = std::is_same<V, Unit>::value ? nullptr : reinterpret_cast<const V*>(plan + pp.val);
    g.key = reinterpret_cast<const unsigned short*>(plan + pp.key);
    g.rs = reinterpret_cast<const int*>(plan + pp.rs);
    g.row = reinterpret_cast<const int*>(plan + pp.row);
    g.deg = reinterpret_cast<const double*>(plan + pp.deg);
    return g;
}

// ------------------------------------------------------- the layout's kernels

// Entries per (chunk, phase) into cnt[c P + k] (zeroed before), and the
// weighted degree of every row slot, one wave per chunk; a row's weights are
// summed lane-strided and then by a fixed butterfly.
template <typename V>
__global__ void __launch_bounds__(WG) k_ph_count(int W, int P, int width, const int* __restrict__ rs,
                                                 const int* __restrict__ prow, const int* __restrict__ rp,
                                                 const int* __restrict__ col, const V* __restrict__ val,
                                                 int* __restrict__ cnt, double* __restrict__ deg) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = blockIdx.x * NWAVE + wv; c < W; c += gridDim.x * NWAVE) {
        int* cc = cnt + static_cast<int64_t>(c) * P;
        for (int a = rs[c]; a < rs[c + 1]; ++a) {
            const int i = prow[a];
            double d = 0.0;
            for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) {
                atomicAdd(&cc[col[e] / width], 1);
                d += weight_at<V>(val, e);
            }
            d = wave_sum(d);
            if (lane == 0) deg[a] = d;
        }
    }
}

// Every entry slot to padding: column 0, weight 0, key PH_SENT.
template <typename V>
__global__ void __launch_bounds__(WG) k_ph_fill(int64_t slots, int* __restrict__ col, V* __restrict__ val,
                                                unsigned short* __restrict__ key) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < slots;
         e += static_cast<int64_t>(gridDim.x) * WG) {
        col[e] = 0;
        if constexpr (!std::is_same<V, Unit>::value) val[e] = V(0);
        key[e] = static_cast<unsigned short>(PH_SENT);
    }
}

// Places every entry of chunk c, one wave per chunk: rows in slot order,
// a row's entries 64 at a time; the lanes that fall in one phase take
// consecutive slots in lane order (a ballot per distinct phase), so each
// (chunk, phase) group lists its entries by local row and, within a row, in
// CSR order, whatever the timing.
template <typename V>
__global__ void __launch_bounds__(WG) k_ph_place(int W, int P, int width, const int* __restrict__ ps,
                                                 const int* __restrict__ rs, const int* __restrict__ prow,
                                                 const int* __restrict__ rp, const int* __restrict__ col,
                                                 const V* __restrict__ val, int* __restrict__ pcol,
                                                 V* __restrict__ pval, unsigned short* __restrict__ pkey) {
    __shared__ int cur_all[NWAVE][PH_PMAX];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int* cur = cur_all[wv];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int c = blockIdx.x * NWAVE + wv; c < W; c += gridDim.x * NWAVE) {
        for (int k = lane; k < P; k += 64) cur[k] = ps[static_cast<int64_t>(c) * (P + 1) + k];
        const int r0 = rs[c];
        for (int a = r0; a < rs[c + 1]; ++a) {
            const int i = prow[a];
            const int e1 = rp[i + 1];
            const unsigned short lr = static_cast<unsigned short>(a - r0);
            for (int base = rp[i]; base < e1; base += 64) {
                const int e = base + lane;
                const bool act = e < e1;
                const int j = act ? col[e] : 0;
                const int k = act ? j / width : -1;
                uint64_t todo = __ballot(act);
                while (todo) {
                    const int first = __builtin_ctzll(todo);
                    const int k0 = __shfl(k, first, 64);
                    const uint64_t m = __ballot(k == k0);
                    const int slot0 = cur[k0];
                    if (k == k0) {
                        const int d = slot0 + __builtin_popcountll(m & below);
                        pcol[d] = j;
                        if constexpr (!std::is_same<V, Unit>::value) pval[d] = val[e];
                        pkey[d] = lr;
                    }
                    if (lane == first) cur[k0] = slot0 + __builtin_popcountll(m);
                    todo &= ~m;
                }
            }
        }
    }
}

// Builds the layout of g into the plan. The host deals the rows (a greedy,
// sequential by nature, over about n / 16 blocks, from row_ptr alone) and
// turns the counts into offsets; the GPU counts, sums the degrees and places
// the entries. Synchronises the stream.
template <typename V>
int build_phased(const fj_csr* g, const Csr<V>& G, char* plan, const PhasedPlan& pp, hipStream_t st,
                 int grid_count, int grid_place, int grid_fill) {
    const PhasedShape& S = pp.s;
    const int n = g->n, W = S.W, P = S.P;
    std::vector<int> rp(static_cast<size_t>(n) + 1);
    PH_HIPCHK(hipStreamSynchronize(st));
    PH_HIPCHK(hipMemcpy(rp.data(), g->row_ptr, rp.size() * sizeof(int), hipMemcpyDeviceToHost));
    // deal 16-row blocks (heavy ones row by row), most entries first, each to
    // the chunk with the fewest entries that has room (ties: lowest chunk)
    struct Block {
        int64_t ent;
        int b0, b1;
    };
    std::vector<Block> blocks;
    blocks.reserve(static_cast<size_t>(n) / PH_BLOCK + 1);
    for (int b0 = 0; b0 < n; b0 += PH_BLOCK) {
        const int b1 = std::min(n, b0 + PH_BLOCK);
        const int64_t ent = rp[b1] - rp[b0];
        if (ent > PH_SINGLE_ABOVE) {
            for (int r = b0; r < b1; ++r) blocks.push_back({rp[r + 1] - rp[r], r, r + 1});
        } else {
            blocks.push_back({ent, b0, b1});
        }
    }
    std::stable_sort(blocks.begin(), blocks.end(), [](const Block& x, const Block& y) { return x.ent > y.ent; });
    using Slot = std::pair<int64_t, int>;
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (int c = 0; c < W; ++c) heap.push({0, c});
    std::vector<int> nrows(static_cast<size_t>(W), 0), chunk_of(static_cast<size_t>(n)), lrow_of(static_cast<size_t>(n));
    std::vector<Slot> aside;
    for (const Block& b : blocks) {
        const int len = b.b1 - b.b0;
        Slot s{};
        aside.clear();
        for (;;) {
            if (heap.empty()) {
                std::snprintf(g_last_error, sizeof g_last_error, "phased layout: no chunk has room");
                return FJ_ERR_INTERNAL;
            }
            s = heap.top();
            heap.pop();
            if (nrows[s.second] + len <= S.rmax) break;
            aside.push_back(s);
        }
        for (int r = b.b0; r < b.b1; ++r) {
            chunk_of[r] = s.second;
            lrow_of[r] = nrows[s.second]++;
        }
        heap.push({s.first + b.ent, s.second});
        for (const Slot& t : aside) heap.push(t);
    }
    std::vector<int> rs(static_cast<size_t>(W) + 1, 0);
    for (int c = 0; c < W; ++c) rs[c + 1] = rs[c] + nrows[c];
    std::vector<int> prow(static_cast<size_t>(n));
    for (int r = 0; r < n; ++r) prow[rs[chunk_of[r]] + lrow_of[r]] = r;
    int* d_ps = reinterpret_cast<int*>(plan + pp.ps);
    int* d_rs = reinterpret_cast<int*>(plan + pp.rs);
    int* d_row = reinterpret_cast<int*>(plan + pp.row);
    double* d_deg = reinterpret_cast<double*>(plan + pp.deg);
    int* d_col = reinterpret_cast<int*>(plan + pp.col);
    V* d_val = reinterpret_cast<V*>(plan + pp.val);
    unsigned short* d_key = reinterpret_cast<unsigned short*>(plan + pp.key);
    PH_HIPCHK(hipMemcpy(d_rs, rs.data(), rs.size() * sizeof(int), hipMemcpyHostToDevice));
    PH_HIPCHK(hipMemcpy(d_row, prow.data(), prow.size() * sizeof(int), hipMemcpyHostToDevice));
    // counts (in the offsets' own space, W P <= W (P + 1) ints) and degrees
    const size_t ncnt = static_cast<size_t>(W) * P;
    PH_HIPCHK(hipMemsetAsync(d_ps, 0, ncnt * sizeof(int), st));
    k_ph_count<V><<<grid_count, WG, 0, st>>>(W, P, S.width, d_rs, d_row, G.row_ptr, G.col, G.val, d_ps, d_deg);
    PH_HIPCHK(hipGetLastError());
    std::vector<int> cnt(ncnt);
    PH_HIPCHK(hipMemcpyAsync(cnt.data(), d_ps, ncnt * sizeof(int), hipMemcpyDeviceToHost, st));
    PH_HIPCHK(hipStreamSynchronize(st));
    std::vector<int> ps(static_cast<size_t>(W) * (P + 1));
    int64_t off = 0;
    for (int c = 0; c < W; ++c) {
        for (int k = 0; k < P; ++k) {
            ps[static_cast<size_t>(c) * (P + 1) + k] = static_cast<int>(off);
            off += (static_cast<int64_t>(cnt[static_cast<size_t>(c) * P + k]) + 7) / 8 * 8;
        }
        ps[static_cast<size_t>(c) * (P + 1) + P] = static_cast<int>(off);
    }
    if (off > S.nnzp) {
        std::snprintf(g_last_error, sizeof g_last_error, "phased layout: %lld slots exceed %lld",
                      static_cast<long long>(off), static_cast<long long>(S.nnzp));
        return FJ_ERR_INTERNAL;
    }
    PH_HIPCHK(hipMemcpy(d_ps, ps.data(), ps.size() * sizeof(int), hipMemcpyHostToDevice));
    if (off > 0) {
        k_ph_fill<V><<<grid_fill, WG, 0, st>>>(off, d_col, d_val, d_key);
        PH_HIPCHK(hipGetLastError());
        k_ph_place<V><<<grid_place, WG, 0, st>>>(W, P, S.width, d_ps, d_rs, d_row, G.row_ptr, G.col, G.val, d_col,
                                                 d_val, d_key);
        PH_HIPCHK(hipGetLastError());
    }
    PH_HIPCHK(hipStreamSynchronize(st));
    return FJ_OK;
}

#undef PH_HIPCHK

}  // namespace fj
