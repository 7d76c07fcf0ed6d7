// fj_kernels.hpp -- HIP kernels for gfx950 (MI355X) behind libfjgpu.
//
// The operator is I + L with L = D - A (Section 2.1), applied row by row as
//   ((I + L) x)_i = x_i + sum_{j in N(i)} w_ij (x_i - x_j),
// never materialised. Everything that touches the CSR is a "window pass":
//
//   Rows are cut into windows by the key  row_ptr[i] + i  (rows plus stored
//   entries): window k holds the rows whose key lies in [k*WIN, (k+1)*WIN). A
//   window therefore has at most WIN rows, and all its rows except the last
//   hold fewer than WIN entries in total, whatever the degree distribution.
//   A workgroup stages the window's neighbour values x_j (and weights) into
//   LDS with coalesced loads of col/val, then reduces each row from LDS. A
//   last row longer than LONGROW (a hub of a power-law graph) is reduced by
//   the whole workgroup straight from HBM instead.
//
// Kernels run on a persistent grid (a few workgroups per CU) that strides
// over windows or elements, so every thread accumulates its share of each
// reduction in a fixed order. Each workgroup stores its sums; the last
// workgroup to arrive (arrival counter) adds them up in a fixed order and
// updates the control block. Results are therefore bitwise reproducible, and
// no scalar ever round-trips through the host inside the CG loop.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fj {

constexpr int WG = 256;               // threads per workgroup: four wave64
constexpr int NWAVE = WG / 64;
#ifndef FJ_WIN
#define FJ_WIN 1024
#endif
constexpr int WIN = FJ_WIN;           // window width in (rows + entries)
constexpr int LONGROW = WIN / 2;      // a longer last row takes the workgroup-wide path
constexpr int STAGE = WIN + LONGROW;  // LDS staging capacity in entries
constexpr int STAGE_PER_THREAD = STAGE / WG;
constexpr int ROWS_PER_THREAD = WIN / WG;
constexpr int LONG_UNROLL = 8;        // loads in flight per thread on a long row
constexpr int NPART = 16;             // sums per workgroup in the partials buffer
constexpr int GMAX = 4096;            // largest persistent grid
constexpr int HIST = 64;              // residual history slots

static_assert(STAGE % WG == 0 && WIN % WG == 0, "window sizes must be multiples of the workgroup");

// Control block in the workspace. Written only by the one-workgroup finalize
// kernels; read by later kernels (kernel boundaries order the accesses) and
// copied to the host between CG chunks.
struct Ctrl {
    double alpha, beta;   // CG step length and direction update of this iteration
    double rz, rr;        // r^T M^{-1} r and r^T r after the last update
    double tol2;          // stop when rr <= tol2
    double mu, ss;        // mean(s) and ||s||^2
    double smin, smax;    // range of s
    double res[16];       // epilogue: indices, residual and diagnostics (see k_epilogue)
    double bound[5];      // certified relative error bound of each index
    double eps_stop;      // > 0: also stop once the estimated bounds of all five indices are below it
    double pbar;          // deflated CG: mean of the current direction p (0 otherwise)
    double rmean;         // mean of r at the last CG start (k_fin_init), the shift of k_cg_shift
    double hist[HIST];    // rr after iteration t is in hist[t % HIST]
    int32_t done;         // 0 running, 1 converged, 2 iteration cap, 3 breakdown, 4 bad input
    int32_t iters;        // CG iterations so far (all passes)
    int32_t max_iter;
    int32_t bad;          // 2 when some s_i is NaN or outside [0,1]
    int32_t deflate;      // 1: CG deflated by the constant vector (see k_cg_shift)
    int32_t pad[3];
};

enum Done : int32_t { RUNNING = 0, CONVERGED = 1, ITER_CAP = 2, BREAKDOWN = 3, BAD_INPUT = 4 };

struct Unit {};  // weight type tag: every edge has weight 1

template <typename V>
struct Csr {
    using value_type = V;
    int n;
    int nnz;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col;
    const V* __restrict__ val;
};

template <typename V>
__device__ __forceinline__ double weight_at(const V* __restrict__ v, int64_t e) {
    return static_cast<double>(v[e]);
}
template <>
__device__ __forceinline__ double weight_at<Unit>(const Unit* __restrict__, int64_t) {
    return 1.0;
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Workgroup sums of N values; every thread receives the totals. The butterfly
// gives every lane the same value and the waves are added in a fixed order.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < N; ++c) red[wave * N + c] = v[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < N; ++c) {
        double t = red[c];
#pragma unroll
        for (int w = 1; w < NWAVE; ++w) t += red[w * N + c];
        v[c] = t;
    }
    __syncthreads();
}

// Workgroup partial sums go to part[blockIdx.x * NPART + c]; a one-workgroup
// finalize kernel adds them up in workgroup order. Publishing through a
// kernel boundary needs no cross-workgroup fence inside the kernel.
template <int N>
__device__ __forceinline__ void store_partials(const double (&v)[N], double* __restrict__ part) {
    static_assert(N <= NPART, "too many partial sums");
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < N; ++c) part[blockIdx.x * NPART + c] = v[c];
    }
}

// Totals of N partial sums over G workgroups, in workgroup order, for a
// finalize kernel (one workgroup). Every thread receives the totals.
template <int N>
__device__ __forceinline__ void total_partials(int G, const double* __restrict__ part, double (&v)[N],
                                               double* red) {
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = 0.0;
    for (int b = threadIdx.x; b < G; b += WG) {
#pragma unroll
        for (int c = 0; c < N; ++c) v[c] += part[b * NPART + c];
    }
    block_sum<N>(v, red);
}

// ------------------------------------------------------------ window pass

// What a row accumulates over its neighbours j (d = x_i - x_j):
struct AccLin   { static constexpr bool X = true,  SQ = false, DEG = false, RAW = false; };  // sum w d
struct AccLinSq { static constexpr bool X = true,  SQ = true,  DEG = false, RAW = false; };  // sum w d, sum w d^2
struct AccDeg   { static constexpr bool X = false, SQ = false, DEG = true,  RAW = false; };  // sum w
struct AccRaw   { static constexpr bool X = true,  SQ = false, DEG = false, RAW = true;  };  // sum w x_j, sum w

// Entry slot STAGE - 1 and row slot WIN are never read: a window stages at
// most STAGE - 1 entries and WIN rows. Lanes with nothing to stage write
// there, so that every lane executes the same stores (no load is ever moved
// into a predicated block, which would stall the pipeline below).
template <typename T, typename V, typename In>
struct Stage {
    T x[STAGE];          // x_j of every staged entry
    V w[STAGE];          // w_ij of every staged entry
    T xrow[WIN + 1];     // x_i of every row of the window
    int rend[WIN + 1];   // end of each row, relative to the window's first entry
    In rin[WIN + 1];     // the operation's per-row inputs
    double clin[WG];     // partial sums of the row a thread's item range ends inside of
    double csq[WG];
};
template <typename T, typename In>
struct Stage<T, Unit, In> {
    T x[STAGE];
    T xrow[WIN + 1];
    int rend[WIN + 1];
    In rin[WIN + 1];
    double clin[WG];
    double csq[WG];
};

// Row window k, precomputed by fj_prepare (k_window_desc). Window k holds the
// rows whose key row_ptr[i] + i lies in [k*WIN, (k+1)*WIN).
struct WinDesc {
    int r0, r1;     // rows [r0, r1)
    int e0;         // row_ptr[r0]
    int elast;      // row_ptr[r1 - 1] (e0 for an empty window)
    int eend;       // row_ptr[r1]
    int nrs;        // rows walked from LDS: r1 - r0, less a long last row
    int ns;         // entries of those rows (< STAGE)
    int long_last;  // 1 when the last row has more than LONGROW entries
};
static_assert(sizeof(WinDesc) == 32, "WinDesc is two 16-byte loads");

template <typename P>
__device__ __forceinline__ P stream_load(const P* p) {
    return __builtin_nontemporal_load(p);
}

template <typename V> struct WeightReg { using type = V; };
template <> struct WeightReg<Unit> { using type = float; };  // unused placeholder

// Registers holding one window's staged entries: column indices and weights.
template <typename V>
struct EntryRegs {
    int j[STAGE_PER_THREAD];
    typename WeightReg<V>::type w[STAGE_PER_THREAD];
};

// Streaming loads of a window's col (and val) into registers. Every lane
// issues the same loads, so the compiler can keep them in flight: a lane past
// the window's entries re-reads the window's last entry (a line already being
// fetched) and records column 0, so its gather below touches one hot line
// shared by all such lanes instead of a random one.
template <typename V>
__device__ __forceinline__ void load_entries(const Csr<V>& g, const WinDesc& d, int last_e, EntryRegs<V>& R) {
    const int elim = min(d.e0 + max(d.ns, 1) - 1, last_e);
#pragma unroll
    for (int u = 0; u < STAGE_PER_THREAD; ++u) {
        const int e = static_cast<int>(threadIdx.x) + u * WG;
        const int idx = min(d.e0 + e, elim);
        const int c = stream_load(&g.col[idx]);
        R.j[u] = e < d.ns ? c : 0;
        if constexpr (!std::is_same<V, Unit>::value) R.w[u] = stream_load(&g.val[idx]);
    }
}

// Reduce one window whose entries, row ends, own values and per-row inputs
// are staged in LDS: calls op.row(i, x_i, sum_j w_ij (x_i - x_j),
// sum_j w_ij (x_i - x_j)^2, in_i) (with AccRaw: op.row(i, x_i,
// sum_j w_ij x_j, sum_j w_ij, in_i)) exactly once for every row of the window,
// from a thread fixed by the data layout (so per-thread partial sums are
// reproducible).
//
// Rows other than a long last row are reduced by a merge-path walk: the
// window's row ends and entries form one ordered list of items (each row's
// entries, then its end marker), and thread t walks items
// [t*ipt, (t+1)*ipt). A row finished inside one thread is emitted at once; a
// row that began in earlier threads is emitted by the thread holding its end,
// after adding the partial sums those threads left behind, in thread order.
// Every thread therefore handles at most ceil(items / WG) items, whatever the
// row lengths. A long last row is reduced by the whole workgroup from HBM.
template <typename T, typename V, typename Acc, typename Op>
__device__ __forceinline__ void window_reduce(const Csr<V>& g, const WinDesc& d, const T* __restrict__ x,
                                              Op& op, Stage<T, V, typename Op::In>& st, double* red) {
    constexpr bool WEIGHTED = !std::is_same<V, Unit>::value;
    const int tid = threadIdx.x;
    const int nrs = d.nrs, ns = d.ns;
    const int total = nrs + ns;
    const int ipt = (total + WG - 1) / WG;
    const int d0 = min(tid * ipt, total);
    const int d1 = min(d0 + ipt, total);
    int lo = 0, hi = nrs;
    while (lo < hi) {  // a0 = number of row ends before item d0 (row a's end is item rend[a] + a)
        const int mid = (lo + hi) >> 1;
        if (st.rend[mid] + mid < d0) lo = mid + 1;
        else hi = mid;
    }
    const int a0 = lo;
    int a = a0;
    int j = d0 - a0;
    const bool continued = (d0 < d1) && (j > (a0 > 0 ? st.rend[a0 - 1] : 0));
    int row_end = (a < nrs) ? st.rend[a] : 0;
    double xa = (Acc::X && a < nrs) ? static_cast<double>(st.xrow[a]) : 0.0;
    double lin = 0.0, sq = 0.0, first_lin = 0.0, first_sq = 0.0;
    bool first_pending = false;
    for (int dd = d0; dd < d1; ++dd) {
        if (j < row_end) {  // entry j of row a
            double w = 1.0;
            if constexpr (WEIGHTED) w = static_cast<double>(st.w[j]);
            if constexpr (Acc::DEG) {
                lin += w;
            } else if constexpr (Acc::RAW) {
                lin += w * static_cast<double>(st.x[j]);
                sq += w;
            } else {
                const double diff = xa - static_cast<double>(st.x[j]);
                lin += w * diff;
                if constexpr (Acc::SQ) sq += w * diff * diff;
            }
            ++j;
        } else {  // end of row a
            if (a == a0 && continued) {
                first_pending = true;
                first_lin = lin;
                first_sq = sq;
            } else {
                op.row(d.r0 + a, static_cast<T>(xa), lin, sq, st.rin[a]);
            }
            lin = 0.0;
            sq = 0.0;
            ++a;
            if (a < nrs) {
                row_end = st.rend[a];
                if constexpr (Acc::X) xa = static_cast<double>(st.xrow[a]);
            }
        }
    }
    st.clin[tid] = lin;
    st.csq[tid] = sq;
    __syncthreads();
    if (first_pending) {
        // Row a0 began in thread t0 (the one holding its first item) and every
        // thread from t0 to tid - 1 left a partial sum of it. They are added
        // from tid - 1 down to t0, eight independent LDS loads at a time.
        const int item0 = a0 > 0 ? st.rend[a0 - 1] + a0 : 0;
        const int t0 = item0 / ipt;
        constexpr bool TWO = Acc::SQ || Acc::RAW;
        double L = first_lin, S = first_sq;
        int t = tid - 1;
        for (; t - 7 >= t0; t -= 8) {
            double cl[8], cs[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cl[u] = st.clin[t - u];
                cs[u] = TWO ? st.csq[t - u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                L += cl[u];
                S += cs[u];
            }
        }
        for (; t >= t0; --t) {
            L += st.clin[t];
            if constexpr (TWO) S += st.csq[t];
        }
        op.row(d.r0 + a0, st.xrow[a0], L, S, st.rin[a0]);
    }

    if (d.long_last) {
        const T xi_t = st.xrow[nrs];
        const double xi = Acc::X ? static_cast<double>(xi_t) : 0.0;
        double v[2] = {0.0, 0.0};
        for (int base = d.elast + tid; base < d.eend; base += WG * LONG_UNROLL) {
            int jj[LONG_UNROLL];
            double ww[LONG_UNROLL];
#pragma unroll
            for (int u = 0; u < LONG_UNROLL; ++u) {  // clamped, unconditional loads
                const int e = base + u * WG;
                const int ec = min(e, d.eend - 1);
                jj[u] = stream_load(&g.col[ec]);
                double w = 1.0;
                if constexpr (WEIGHTED) w = static_cast<double>(stream_load(&g.val[ec]));
                ww[u] = (e < d.eend) ? w : 0.0;
            }
            if constexpr (Acc::DEG) {
#pragma unroll
                for (int u = 0; u < LONG_UNROLL; ++u) v[0] += ww[u];
            } else if constexpr (Acc::RAW) {
                double xv[LONG_UNROLL];
#pragma unroll
                for (int u = 0; u < LONG_UNROLL; ++u) xv[u] = static_cast<double>(x[jj[u]]);
#pragma unroll
                for (int u = 0; u < LONG_UNROLL; ++u) {
                    v[0] += ww[u] * xv[u];
                    v[1] += ww[u];
                }
            } else {
                double xv[LONG_UNROLL];
#pragma unroll
                for (int u = 0; u < LONG_UNROLL; ++u) xv[u] = static_cast<double>(x[jj[u]]);
#pragma unroll
                for (int u = 0; u < LONG_UNROLL; ++u) {
                    const double diff = xi - xv[u];
                    v[0] += ww[u] * diff;
                    if constexpr (Acc::SQ) v[1] += ww[u] * diff * diff;
                }
            }
        }
        block_sum<2>(v, red);
        if (tid == 0) op.row(d.r1 - 1, xi_t, v[0], v[1], st.rin[nrs]);
    }
}

// Window descriptors are loaded into vector registers and moved to scalar
// registers (the window index is uniform across the workgroup) only when the
// window comes up, so no load has to complete early.
struct RawDesc {
    int4 lo, hi;
};
__device__ __forceinline__ RawDesc load_raw_desc(const WinDesc* __restrict__ p) {
    return RawDesc{reinterpret_cast<const int4*>(p)[0], reinterpret_cast<const int4*>(p)[1]};
}
__device__ __forceinline__ WinDesc to_scalar(const RawDesc& r) {
    WinDesc d;
    d.r0 = __builtin_amdgcn_readfirstlane(r.lo.x);
    d.r1 = __builtin_amdgcn_readfirstlane(r.lo.y);
    d.e0 = __builtin_amdgcn_readfirstlane(r.lo.z);
    d.elast = __builtin_amdgcn_readfirstlane(r.lo.w);
    d.eend = __builtin_amdgcn_readfirstlane(r.hi.x);
    d.nrs = __builtin_amdgcn_readfirstlane(r.hi.y);
    d.ns = __builtin_amdgcn_readfirstlane(r.hi.z);
    d.long_last = __builtin_amdgcn_readfirstlane(r.hi.w);
    return d;
}

// Loads of one window that the reduction needs in registers: the gathered
// x_j and the weights of its staged entries, and the row ends, own values and
// per-row inputs of its rows (row a of a window is loaded by thread a % WG).
template <typename T, typename V, typename In>
struct WindowRegs {
    T xv[STAGE_PER_THREAD];
    typename WeightReg<V>::type w[STAGE_PER_THREAD];
    int re[ROWS_PER_THREAD];
    T xr[ROWS_PER_THREAD];
    In in[ROWS_PER_THREAD];
};

// The windows k0, k0 + G, k0 + 2G, ... (k0 = blockIdx.x, G = gridDim.x) of one
// workgroup, software-pipelined three deep: while window t is staged and
// reduced, the gathers and row loads of window t+1, the col/val loads of
// window t+2 and the descriptor of window t+3 are in flight, so the reduction
// never waits on memory it did not ask for a whole window earlier. Striding
// by G spreads the costly windows (hub rows) evenly over the workgroups.
// All loads and LDS stores are unconditional (clamped to valid addresses and
// dummy slots) so that the loads stay in flight across the loop body.
// ENTRIES is false only for a graph without edges, whose col/val may be null.
template <typename T, typename V, typename Acc, bool ENTRIES, typename Op>
__device__ __forceinline__ void window_range(const Csr<V>& g, const WinDesc* __restrict__ desc, int K,
                                             const T* __restrict__ x, Op& op,
                                             Stage<T, V, typename Op::In>& st, double* red) {
    constexpr bool WEIGHTED = !std::is_same<V, Unit>::value;
    constexpr bool LOADS = ENTRIES && (Acc::X || WEIGHTED);
    using In = typename Op::In;
    const int G = gridDim.x;
    const int k0 = blockIdx.x;
    if (k0 >= K) return;
    const int tid = threadIdx.x;
    const int last_e = g.nnz > 0 ? g.nnz - 1 : 0;
    const int klast = k0 + (K - 1 - k0) / G * G;  // this workgroup's last window

    auto issue_window = [&](const WinDesc& d, const EntryRegs<V>& E, WindowRegs<T, V, In>& W) {
        if constexpr (Acc::X) {
#pragma unroll
            for (int u = 0; u < STAGE_PER_THREAD; ++u) W.xv[u] = x[E.j[u]];
        }
        if constexpr (WEIGHTED) {
#pragma unroll
            for (int u = 0; u < STAGE_PER_THREAD; ++u) W.w[u] = E.w[u];
        }
        const int ilim = min(max(d.r1 - 1, d.r0), g.n - 1);  // lanes past the rows re-read the last one
#pragma unroll
        for (int u = 0; u < ROWS_PER_THREAD; ++u) {
            const int i = min(d.r0 + tid + u * WG, ilim);
            W.re[u] = g.row_ptr[i + 1];
            if constexpr (Acc::X) W.xr[u] = x[i];
            W.in[u] = op.load(i);
        }
    };

    WinDesc d_cur = to_scalar(load_raw_desc(desc + k0));
    WinDesc d_nxt = to_scalar(load_raw_desc(desc + min(k0 + G, klast)));
    WinDesc d_nn = to_scalar(load_raw_desc(desc + min(k0 + 2 * G, klast)));
    EntryRegs<V> E{};
    if constexpr (LOADS) load_entries(g, d_cur, last_e, E);
    WindowRegs<T, V, In> Wc;
    issue_window(d_cur, E, Wc);
    EntryRegs<V> En = E;
    if constexpr (LOADS) load_entries(g, d_nxt, last_e, En);

    for (int k = k0; k < K; k += G) {
        const RawDesc a3 = load_raw_desc(desc + min(k + 3 * G, klast));
        // window t+1: gathers and row loads; window t+2: col/val loads
        WindowRegs<T, V, In> Wn;
        issue_window(d_nxt, En, Wn);
        EntryRegs<V> Enn = En;
        if constexpr (LOADS) load_entries(g, d_nn, last_e, Enn);
        // stage window t
        const int nrows = d_cur.r1 - d_cur.r0;
#pragma unroll
        for (int u = 0; u < STAGE_PER_THREAD; ++u) {
            const int e = tid + u * WG;
            const int slot = e < d_cur.ns ? e : STAGE - 1;
            if constexpr (Acc::X) st.x[slot] = Wc.xv[u];
            if constexpr (WEIGHTED) st.w[slot] = Wc.w[u];
        }
#pragma unroll
        for (int u = 0; u < ROWS_PER_THREAD; ++u) {
            const int a = tid + u * WG;
            const int slot = a < nrows ? a : WIN;
            st.rend[slot] = Wc.re[u] - d_cur.e0;
            if constexpr (Acc::X) st.xrow[slot] = Wc.xr[u];
            st.rin[slot] = Wc.in[u];
        }
        __syncthreads();
        if (nrows > 0) window_reduce<T, V, Acc>(g, d_cur, x, op, st, red);
        __syncthreads();  // LDS is reused by the next window
        d_cur = d_nxt;
        d_nxt = d_nn;
        d_nn = to_scalar(a3);
        Wc = Wn;
        En = Enn;
    }
}

template <typename T, typename V, typename Acc, typename Op>
__device__ __forceinline__ void my_windows(const Csr<V>& g, const WinDesc* __restrict__ desc, int K,
                                           const T* __restrict__ x, Op& op,
                                           Stage<T, V, typename Op::In>& st, double* red) {
    if (g.nnz > 0) window_range<T, V, Acc, true>(g, desc, K, x, op, st, red);
    else window_range<T, V, Acc, false>(g, desc, K, x, op, st, red);
}

// ------------------------------------------------------------ row operations
// Each operation names the per-row inputs it needs (In, fetched by load(i)
// with the window's other loads) and finishes row i in row(i, x_i, lin, sq, in)
// with lin = ((L x)_i) and sq = sum_j w_ij (x_i - x_j)^2.

struct NoIn {
    char unused;
};

struct OpDiag {  // Jacobi preconditioner M^{-1} = diag(1 + d_i)^{-1}
    using In = NoIn;
    float* __restrict__ minv;
    __device__ In load(int) const { return {}; }
    template <typename T>
    __device__ void row(int i, T, double deg, double, const In&) { minv[i] = static_cast<float>(1.0 / (1.0 + deg)); }
};

struct OpApply {  // y = (I + L) x
    using In = NoIn;
    double* __restrict__ y;
    __device__ In load(int) const { return {}; }
    __device__ void row(int i, double xi, double lin, double, const In&) { y[i] = xi + lin; }
};

// q = (I + L) p and the three dot products the CG scalars need. T is the
// vector precision (double, or float for the inner solve of FJ_MIXED); the
// row sums and the dot products are accumulated in double, and the dots use q
// as stored.
template <typename T>
struct OpCgSpmv {
    struct In {
        T r;
        float m;
    };
    const T* __restrict__ r;
    const float* __restrict__ minv;
    T* __restrict__ q;
    double shift;  // deflated CG: q = (I+L) p - mean(p) 1, the projection of (I+L) p
    double pq = 0.0, rmq = 0.0, qmq = 0.0;
    __device__ In load(int i) const { return {r[i], minv[i]}; }
    __device__ void row(int i, T pi, double lin, double, const In& in) {
        const T qt = static_cast<T>(static_cast<double>(pi) + lin - shift);
        q[i] = qt;
        const double qi = static_cast<double>(qt);
        const double mq = static_cast<double>(in.m) * qi;
        pq += static_cast<double>(pi) * qi;
        rmq += static_cast<double>(in.r) * mq;
        qmq += qi * mq;
    }
};

// q = (I + L) p - shift and p^T q only: with the 2x2 block preconditioner the
// other two dot products need the partner's q and are formed by k_pair_dots.
template <typename T>
struct OpCgSpmvPq {
    using In = NoIn;
    T* __restrict__ q;
    double shift;
    double pq = 0.0;
    __device__ In load(int) const { return {}; }
    __device__ void row(int i, T pi, double lin, double, const In&) {
        const T qt = static_cast<T>(static_cast<double>(pi) + lin - shift);
        q[i] = qt;
        pq += static_cast<double>(pi) * static_cast<double>(qt);
    }
};

struct OpEpilogue {  // one pass over z: every index, the true residual and diagnostics
    struct In {
        double s;
    };
    const double* __restrict__ s;
    int64_t lds;
    double mu;
    double* __restrict__ rbuf;
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    __device__ In load(int i) const { return {s[static_cast<int64_t>(i) * lds]}; }
    __device__ void row(int i, double zi, double t, double dsq, const In& in) {
        const double si = in.s;
        const double ri = si - zi - t;  // t = (L z)_i, so r = s - (I + L) z
        rbuf[i] = ri;
        const double dm = zi - mu;
        const double dz = zi - si;
        v[0] += t * t;    // ||L z||^2                     (Lemma 4.1, C_I)
        v[1] += dsq;      // 2 * sum_E w (z_i - z_j)^2     (Section 3.2, D)
        v[2] += dm * dm;  // sum (z_i - mu)^2, mu = mean(s)
        v[3] += zi * zi;  // ||z||^2                       (C)
        v[4] += zi;       // sum z
        v[5] += si * zi;  // s^T z                         (I_dc)
        v[6] += ri * ri;  // ||r||^2
        v[7] += zi * ri;  // z^T r
        v[8] += dz * dz;  // sum (z_i - s_i)^2             (definition of C_I)
    }
};

// ------------------------------------------------------------ kernels

// blk_row[k] = first row i with row_ptr[i] + i >= k * WIN (n if none), k = 0..K.
__global__ void __launch_bounds__(WG) k_windows(int n, const int* __restrict__ row_ptr, int K,
                                                int* __restrict__ blk_row) {
    for (int k = blockIdx.x * WG + threadIdx.x; k <= K; k += gridDim.x * WG) {
        const int64_t target = static_cast<int64_t>(k) * WIN;
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (static_cast<int64_t>(row_ptr[mid]) + mid >= target) hi = mid;
            else lo = mid + 1;
        }
        blk_row[k] = lo;
    }
}

__global__ void __launch_bounds__(WG) k_window_desc(int n, const int* __restrict__ row_ptr, int K,
                                                    const int* __restrict__ blk_row, WinDesc* __restrict__ desc) {
    for (int k = blockIdx.x * WG + threadIdx.x; k < K; k += gridDim.x * WG) {
        WinDesc d;
        d.r0 = blk_row[k];
        d.r1 = blk_row[k + 1];
        d.e0 = row_ptr[d.r0];
        d.eend = row_ptr[d.r1];
        d.elast = d.r1 > d.r0 ? row_ptr[d.r1 - 1] : d.e0;
        d.long_last = (d.r1 > d.r0) && (d.eend - d.elast > LONGROW);
        d.nrs = d.r1 - d.r0 - d.long_last;
        d.ns = (d.long_last ? d.elast : d.eend) - d.e0;
        desc[k] = d;
    }
}

template <typename V>
__global__ void __launch_bounds__(WG) k_diag(Csr<V> g, const WinDesc* __restrict__ desc, int K,
                                             float* __restrict__ minv) {
    __shared__ Stage<double, V, OpDiag::In> st;
    __shared__ double red[NWAVE * 2];
    OpDiag op{minv};
    my_windows<double, V, AccDeg>(g, desc, K, static_cast<const double*>(nullptr), op, st, red);
}

template <typename V>
__global__ void __launch_bounds__(WG) k_apply(Csr<V> g, const WinDesc* __restrict__ desc, int K,
                                              const double* __restrict__ x, double* __restrict__ y) {
    __shared__ Stage<double, V, OpApply::In> st;
    __shared__ double red[NWAVE * 2];
    OpApply op{y};
    my_windows<double, V, AccLin>(g, desc, K, x, op, st, red);
}

// Measurement aid, not part of the solve: the bare gather of an SpMV in CSR
// order. Thread t reads entries 8t .. 8t+7 (col and val, streamed) and
// writes y[t] = sum w_e x_col(e), ignoring row boundaries, with eight gathers
// in flight. Its time is the floor for any pass that reads the CSR once and
// gathers x_j per entry in this order.
template <typename V>
__global__ void __launch_bounds__(WG) k_gather_bound(Csr<V> g, const double* __restrict__ x, double* __restrict__ y) {
    const int64_t groups = (static_cast<int64_t>(g.nnz) + 7) / 8;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; t < groups;
         t += static_cast<int64_t>(gridDim.x) * WG) {
        int j[8];
        double w[8], v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t e = t * 8 + u;
            const int64_t ec = e < g.nnz ? e : g.nnz - 1;
            j[u] = stream_load(&g.col[ec]);
            double wv = 1.0;
            if constexpr (!std::is_same<V, Unit>::value) wv = static_cast<double>(stream_load(&g.val[ec]));
            w[u] = e < g.nnz ? wv : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = x[j[u]];
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += w[u] * v[u];
        y[t] = acc;
    }
}

// Measurement aid: the same bare gather over entries regrouped into S
// streams (the host builds them; see fj_gather_bound_sliced). Stream s holds
// entries [off[s], off[s] + cnt[s]) padded to a multiple of 8 from off[s]
// (8-aligned); padding slots point at column 0 with weight 0. Workgroup b
// works on stream b % S, so with S = 8 a stream stays on one XCD (workgroups
// are dealt to the XCDs round robin). check (optional, int[2]) counts the
// workgroups whose hardware XCD id equals b % 8, and all workgroups.
template <typename V, typename X, int S>
__global__ void __launch_bounds__(WG) k_gather_sliced(const int* __restrict__ col, const V* __restrict__ val,
                                                      const X* __restrict__ x, double* __restrict__ y,
                                                      const int64_t* __restrict__ off, const int64_t* __restrict__ cnt,
                                                      int* __restrict__ check) {
    const int s = blockIdx.x % S;
    const int wb = blockIdx.x / S;
    const int gs = gridDim.x / S;
    if (check && threadIdx.x == 0) {
        unsigned xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
        atomicAdd(&check[0], static_cast<int>((xcc & 0xfu) == static_cast<unsigned>(blockIdx.x % 8)));
        atomicAdd(&check[1], 1);
    }
    const int64_t e0 = off[s], real_end = e0 + cnt[s];
    const int64_t groups = (cnt[s] + 7) / 8;
    typedef int iv4 __attribute__((ext_vector_type(4)));
    for (int64_t t = static_cast<int64_t>(wb) * WG + threadIdx.x; t < groups; t += static_cast<int64_t>(gs) * WG) {
        const int64_t b = e0 + t * 8;
        const iv4 ja = __builtin_nontemporal_load(reinterpret_cast<const iv4*>(col + b));
        const iv4 jb = __builtin_nontemporal_load(reinterpret_cast<const iv4*>(col + b + 4));
        const int j[8] = {ja.x, ja.y, ja.z, ja.w, jb.x, jb.y, jb.z, jb.w};
        double w[8], v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            double wv = 1.0;
            if constexpr (!std::is_same<V, Unit>::value) wv = static_cast<double>(stream_load(&val[b + u]));
            w[u] = b + u < real_end ? wv : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = static_cast<double>(x[j[u]]);
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += w[u] * v[u];
        y[e0 / 8 + t] = acc;
    }
}

// One synchronous step of the FJ update rule (Section 3.1, Eq. FJmodel):
// z'_i = (s_i + sum_j w_ij z_j) / (1 + sum_j w_ij), with the largest change
// |z'_i - z_i| of the step.
struct OpFj {
    struct In {
        double s;
    };
    const double* __restrict__ s;
    double* __restrict__ znext;
    double maxc = 0.0;
    __device__ In load(int i) const { return {s[i]}; }
    __device__ void row(int i, double zi, double wz, double wsum, const In& in) {
        const double zn = (in.s + wz) / (1.0 + wsum);
        znext[i] = zn;
        maxc = fmax(maxc, fabs(zn - zi));
    }
};

template <typename V>
__global__ void __launch_bounds__(WG) k_fj_sweep(Csr<V> g, const WinDesc* __restrict__ desc, int K,
                                                 const double* __restrict__ z, const double* __restrict__ s,
                                                 double* __restrict__ znext, double* __restrict__ part,
                                                 const Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ Stage<double, V, OpFj::In> st;
    __shared__ double red[NWAVE * 2];
    OpFj op{s, znext};
    my_windows<double, V, AccRaw>(g, desc, K, z, op, st, red);
    double m = wave_max(op.maxc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w) m = fmax(m, red[w]);
        red[0] = m;
    }
    __syncthreads();
    double v[1] = {red[0]};
    store_partials<1>(v, part);
}

// Largest change of the step; stops when it is at most tol (held in tol2), or
// at the step limit.
__global__ void __launch_bounds__(WG) k_fin_fj(int G, const double* __restrict__ part, Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double red[NWAVE];
    double m = 0.0;
    for (int b = threadIdx.x; b < G; b += WG) m = fmax(m, part[b * NPART]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w) m = fmax(m, red[w]);
        const int t = ctrl->iters;
        ctrl->res[0] = m;
        ctrl->hist[t % HIST] = m;
        ctrl->iters = t + 1;
        if (!isfinite(m)) ctrl->done = BREAKDOWN;
        else if (m <= ctrl->tol2) ctrl->done = CONVERGED;
        else if (t + 1 >= ctrl->max_iter) ctrl->done = ITER_CAP;
    }
}

__global__ void k_fj_ctrl_init(Ctrl* __restrict__ ctrl, double tol, int max_steps) {
    if (threadIdx.x == 0) {
        ctrl->tol2 = tol;
        ctrl->max_iter = max_steps;
        ctrl->iters = 0;
        ctrl->res[0] = 0.0;
        ctrl->done = max_steps > 0 ? RUNNING : ITER_CAP;
    }
}

// CG step, part 1: q = (I+L) p (minus mean(p) 1 when deflated) with the
// partial sums of p^T q, r^T M^{-1} q and q^T M^{-1} q.
template <typename V, typename T>
__global__ void __launch_bounds__(WG) k_cg_spmv(Csr<V> g, const WinDesc* __restrict__ desc, int K,
                                                const T* __restrict__ p, const T* __restrict__ r,
                                                const float* __restrict__ minv, T* __restrict__ q,
                                                double* __restrict__ part, const Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ Stage<T, V, typename OpCgSpmv<T>::In> st;
    __shared__ double red[NWAVE * 4];
    OpCgSpmv<T> op{r, minv, q, ctrl->pbar};
    my_windows<T, V, AccLin>(g, desc, K, p, op, st, red);
    double v[3] = {op.pq, op.rmq, op.qmq};
    block_sum<3>(v, red);
    store_partials<3>(v, part);
}

// alpha = rz / p^T q; from the recurrence r' = r - alpha q,
// rz' = rz - 2 alpha r^T M^{-1} q + alpha^2 q^T M^{-1} q and beta = rz' / rz,
// so that the update kernel can also move the direction in the same pass.
__global__ void __launch_bounds__(WG) k_fin_spmv(int G, const double* __restrict__ part,
                                                 Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double red[NWAVE * 3];
    double v[3];
    total_partials<3>(G, part, v, red);
    if (threadIdx.x == 0) {
        const double rz = ctrl->rz;
        const double pq = v[0];
        if (rz == 0.0) {
            ctrl->done = CONVERGED;
        } else if (!(pq > 0.0) || !isfinite(pq)) {
            ctrl->done = BREAKDOWN;
        } else {
            const double alpha = rz / pq;
            const double rz_next = rz - 2.0 * alpha * v[1] + alpha * alpha * v[2];
            ctrl->alpha = alpha;
            ctrl->beta = rz_next / rz;
        }
    }
}

// CG step, part 2: x += alpha (p - pbar), r -= alpha q, z = M^{-1} r,
// p = z + beta p, and the partial sums of the exact r^T M^{-1} r (next alpha),
// r^T r (stopping test) and sum p (next pbar). Each thread moves 16-byte packs
// of every vector (2 doubles or 4 floats); arithmetic is in double, rounded
// once when stored.
template <typename T> struct Pack;
template <> struct Pack<double> { using type = double2; using mtype = float2; static constexpr int N = 2; };
template <> struct Pack<float> { using type = float4; using mtype = float4; static constexpr int N = 4; };

template <typename T>
__device__ __forceinline__ void cg_update_elem(double alpha, double beta, double pbar, T& x, T& r, T& p, T q,
                                               float m, double (&v)[3]) {
    x = static_cast<T>(static_cast<double>(x) + alpha * (static_cast<double>(p) - pbar));
    r = static_cast<T>(static_cast<double>(r) - alpha * static_cast<double>(q));
    const double rd = static_cast<double>(r);
    const double z = static_cast<double>(m) * rd;
    p = static_cast<T>(z + beta * static_cast<double>(p));
    v[0] += rd * z;
    v[1] += rd * rd;
    v[2] += static_cast<double>(p);
}

template <typename T>
__device__ __forceinline__ void cg_update_pack(int t, double alpha, double beta, double pbar, T* __restrict__ x,
                                               T* __restrict__ r, T* __restrict__ p,
                                               const T* __restrict__ q, const float* __restrict__ minv,
                                               double (&v)[3]) {
    using P = typename Pack<T>::type;
    using M = typename Pack<T>::mtype;
    constexpr int N = Pack<T>::N;
    P xv = reinterpret_cast<P*>(x)[t];
    P rv = reinterpret_cast<P*>(r)[t];
    P pv = reinterpret_cast<P*>(p)[t];
    const P qv = reinterpret_cast<const P*>(q)[t];
    const M mv = reinterpret_cast<const M*>(minv)[t];
    T* xs = reinterpret_cast<T*>(&xv);
    T* rs = reinterpret_cast<T*>(&rv);
    T* ps = reinterpret_cast<T*>(&pv);
    const T* qs = reinterpret_cast<const T*>(&qv);
    const float* ms = reinterpret_cast<const float*>(&mv);
#pragma unroll
    for (int e = 0; e < N; ++e) cg_update_elem(alpha, beta, pbar, xs[e], rs[e], ps[e], qs[e], ms[e], v);
    reinterpret_cast<P*>(x)[t] = xv;
    reinterpret_cast<P*>(r)[t] = rv;
    reinterpret_cast<P*>(p)[t] = pv;
}

// EST (single vector, FP64, s contiguous): also the sums that estimate the
// five indices at the new x (Section 3.2 via Proposition 1: C = x^T x,
// sum x for P, I_dc = s^T x, C_I ~ ||s - x||^2 since s - z = L z), for the
// early stop in k_fin_update.
template <bool EST>
__device__ __forceinline__ void est_pack(int t, const double* __restrict__ x, const double* __restrict__ s,
                                         double (&e)[4]) {
    if constexpr (EST) {
        const double2 xv = reinterpret_cast<const double2*>(x)[t];
        const double2 sv = reinterpret_cast<const double2*>(s)[t];
        e[0] += xv.x * xv.x + xv.y * xv.y;
        e[1] += xv.x + xv.y;
        e[2] += sv.x * xv.x + sv.y * xv.y;
        const double d0 = sv.x - xv.x, d1 = sv.y - xv.y;
        e[3] += d0 * d0 + d1 * d1;
    }
}

template <typename T, bool EST>
__global__ void __launch_bounds__(WG) k_cg_update(int n, T* __restrict__ x, T* __restrict__ r,
                                                  T* __restrict__ p, const T* __restrict__ q,
                                                  const float* __restrict__ minv, const double* __restrict__ s,
                                                  double* __restrict__ part, const Ctrl* __restrict__ ctrl) {
    static_assert(!EST || std::is_same<T, double>::value, "estimates are for FP64 vectors");
    if (ctrl->done != RUNNING) return;
    __shared__ double red[NWAVE * 7];
    constexpr int N = Pack<T>::N;
    const double alpha = ctrl->alpha, beta = ctrl->beta, pbar = ctrl->pbar;
    double v[3] = {0.0, 0.0, 0.0};
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    const int npack = n / N;
    const int stride = gridDim.x * WG;
    int t = blockIdx.x * WG + threadIdx.x;
    for (; t + stride < npack; t += 2 * stride) {  // two packs per thread in flight
        cg_update_pack(t, alpha, beta, pbar, x, r, p, q, minv, v);
        cg_update_pack(t + stride, alpha, beta, pbar, x, r, p, q, minv, v);
        if constexpr (EST) {
            est_pack<EST>(t, reinterpret_cast<const double*>(x), s, e);
            est_pack<EST>(t + stride, reinterpret_cast<const double*>(x), s, e);
        }
    }
    if (t < npack) {
        cg_update_pack(t, alpha, beta, pbar, x, r, p, q, minv, v);
        if constexpr (EST) est_pack<EST>(t, reinterpret_cast<const double*>(x), s, e);
    }
    if (blockIdx.x == 0 && threadIdx.x < n - npack * N) {
        const int i = npack * N + threadIdx.x;
        cg_update_elem(alpha, beta, pbar, x[i], r[i], p[i], q[i], minv[i], v);
        if constexpr (EST) {
            const double xi = static_cast<double>(x[i]), si = s[i];
            e[0] += xi * xi;
            e[1] += xi;
            e[2] += si * xi;
            e[3] += (si - xi) * (si - xi);
        }
    }
    if constexpr (EST) {
        double w[7] = {v[0], v[1], v[2], e[0], e[1], e[2], e[3]};
        block_sum<7>(w, red);
        store_partials<7>(w, part);
    } else {
        block_sum<3>(v, red);
        store_partials<3>(v, part);
    }
}

// The relative error bound of an index from its value and the residual norm
// it sees (see k_fin_epilogue); infinite when no relative bound exists.
__device__ __forceinline__ double quad_bound(double X, double rh) {
    const double rx = sqrt(fmax(X, 0.0));
    return rx > rh ? rh * (2.0 * rx + rh) / ((rx - rh) * (rx - rh)) : INFINITY;
}

template <bool EST>
__global__ void __launch_bounds__(WG) k_fin_update(int G, int n, const double* __restrict__ part,
                                                   Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    constexpr int NV = EST ? 7 : 3;
    __shared__ double red[NWAVE * NV];
    double v[NV];
    total_partials<NV>(G, part, v, red);
    if (threadIdx.x == 0) {
        const int it = ctrl->iters + 1;
        ctrl->iters = it;
        ctrl->rz = v[0];
        ctrl->rr = v[1];
        ctrl->hist[it % HIST] = v[1];
        ctrl->pbar = ctrl->deflate ? v[2] / static_cast<double>(n) : 0.0;
        bool early = false;
        if constexpr (EST) {
            // estimated indices at the new x with the recursive residual norm;
            // the FP64 epilogue still certifies the result afterwards
            if (ctrl->eps_stop > 0.0 && v[1] >= 0.0) {
                const double rho = sqrt(v[1]);
                const double C = v[3], mean = v[4] / static_cast<double>(n), Idc = v[5];
                const double P = C - static_cast<double>(n) * mean * mean, D = Idc - C, CI = v[6];
                const double a = (sqrt(fmax(C, 0.0)) + rho) * rho;
                const double bdc = Idc > a ? a / (Idc - a) : INFINITY;
                early = fmax(fmax(quad_bound(CI, rho), quad_bound(D, 0.5 * rho)),
                             fmax(fmax(quad_bound(P, rho), quad_bound(C, rho)), bdc)) <= ctrl->eps_stop;
            }
        }
        if (!isfinite(v[1])) ctrl->done = BREAKDOWN;
        else if (v[1] <= ctrl->tol2 || early) ctrl->done = CONVERGED;
        else if (it >= ctrl->max_iter) ctrl->done = ITER_CAP;
    }
}

// ------------------------------------------------------------ 2x2 block preconditioner
// M = blockdiag of I + L restricted to the pairs of a heavy-edge matching
// (single nodes keep the Jacobi entry 1 + d_i). For a pair (i, j) with edge
// weight w the block is [[a_i, -w], [-w, a_j]], a = 1 + d, whose inverse gives
// z_i = c1_i r_i + c2_i r_j with c1_i = a_j / det, c2 = w / det,
// det = a_i a_j - w^2 > 0 (a_i >= 1 + w). Heavy edges are what Jacobi misses:
// on graphs with widely spread weights the pairs halve the CG iterations.
//
// Matching (fj_prepare): rounds of handshakes. Every unmatched node proposes
// its heaviest unmatched neighbour (ties: the larger index); mutual proposals
// become pairs. Deterministic, one pass over the CSR per round.

constexpr int PAIR_ROUNDS = 4;  // handshake rounds (1: the locally dominant edges; 4: about 70 % of nodes paired)
// One-vector FP64 solves of graphs from this many nodes on use the pairs
// (below, the extra launch per iteration costs more than the iterations it
// saves: 0.54 against 0.44 ms on a 10K-node Barabasi-Albert graph).
constexpr int PAIR_MIN_N = 65536;
// The FP32 inner solves of FJ_MIXED use them only when the SpMV's work per
// node (the mean degree) outweighs the pair pass's fixed work per node: on a
// 1M-node graph of mean degree 10 they cost more than they saved (2.88
// against 2.79 ms), on the 4M-node graph of mean degree 30 they save 14 %.
constexpr int PAIR_MIN_DEGREE_FP32 = 16;

__global__ void __launch_bounds__(WG) k_pair_init(int n, int* __restrict__ mate) {
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) mate[i] = -1;
}

// One wave per row (hub rows hold thousands of entries): lanes scan strided
// parts of the row, then a wave reduction keeps the heaviest (weight, index).
template <typename V>
__global__ void __launch_bounds__(WG) k_pair_propose(Csr<V> g, const int* __restrict__ mate, int* __restrict__ prop,
                                                     float* __restrict__ pw) {
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * NWAVE;
    for (int i = blockIdx.x * NWAVE + (threadIdx.x >> 6); i < g.n; i += waves) {
        if (mate[i] >= 0) {  // matched in an earlier round: keeps the weight of its pair's edge in pw
            if (lane == 0) prop[i] = -1;
            continue;
        }
        int best = -1;
        double bw = -1.0;
        const int e1 = g.row_ptr[i + 1];
        for (int e = g.row_ptr[i] + lane; e < e1; e += 64) {
            const int j = g.col[e];
            if (j == i || mate[j] >= 0) continue;
            const double w = weight_at<V>(g.val, e);
            if (w > bw || (w == bw && j > best)) {
                best = j;
                bw = w;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ow = __shfl_xor(bw, o, 64);
            const int oj = __shfl_xor(best, o, 64);
            if (ow > bw || (ow == bw && oj > best)) {
                best = oj;
                bw = ow;
            }
        }
        if (lane == 0) {
            prop[i] = best;
            pw[i] = static_cast<float>(bw);
        }
    }
}

__global__ void __launch_bounds__(WG) k_pair_accept(int n, const int* __restrict__ prop, int* __restrict__ mate) {
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const int j = prop[i];
        if (mate[i] < 0 && j >= 0 && prop[j] == i) mate[i] = j;
    }
}

// Both members of a pair take w from the lower index and the same det, so the
// preconditioner is symmetric whatever rounding the weights went through.
__global__ void __launch_bounds__(WG) k_pair_coef(int n, const int* __restrict__ mate, const float* __restrict__ pw,
                                                  const float* __restrict__ minv, float2* __restrict__ pc) {
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const int j = mate[i];
        if (j < 0) {
            pc[i] = make_float2(minv[i], 0.0f);
        } else {
            const double ai = 1.0 / static_cast<double>(minv[i]), aj = 1.0 / static_cast<double>(minv[j]);
            const double w = static_cast<double>(pw[i < j ? i : j]);
            const double det = ai * aj - w * w;
            pc[i] = make_float2(static_cast<float>(aj / det), static_cast<float>(w / det));
        }
    }
}

template <typename T>
__device__ __forceinline__ double pair_apply(int i, const T* __restrict__ v, const int* __restrict__ mate,
                                             const float2* __restrict__ pc) {
    const float2 c = pc[i];
    const int j = mate[i];
    double y = static_cast<double>(c.x) * static_cast<double>(v[i]);
    if (j >= 0) y += static_cast<double>(c.y) * static_cast<double>(v[j]);
    return y;
}

// CG start with the block preconditioner, after k_cg_init (and k_cg_shift):
// z = M^{-1} r, p = z, and the partial sums of rz, rr and sum p in the slots
// k_fin_init mode 1 reads. T: the vector precision (double, or float for the
// inner solves of FJ_MIXED); sums in double, each value rounded once.
template <typename T>
__global__ void __launch_bounds__(WG) k_pair_start(int n, const T* __restrict__ r, T* __restrict__ z,
                                                   T* __restrict__ p, const int* __restrict__ mate,
                                                   const float2* __restrict__ pc, double* __restrict__ part) {
    __shared__ double red[NWAVE * 3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const T zt = static_cast<T>(pair_apply(i, r, mate, pc));
        const double zi = static_cast<double>(zt);
        const double ri = static_cast<double>(r[i]);
        z[i] = zt;
        p[i] = zt;
        v[0] += ri * zi;
        v[1] += ri * ri;
        v[2] += zi;
    }
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
        double* out = part + blockIdx.x * NPART;
        out[0] = v[0];
        out[1] = v[1];
        out[2] = out[3] = out[4] = 0.0;
        out[5] = v[2];
        out[6] = INFINITY;
        out[7] = -INFINITY;
    }
}

// CG step with the block preconditioner, part 1: q = (I+L) p - pbar and p^T q
// (partial slot 0).
template <typename V, typename T>
__global__ void __launch_bounds__(WG) k_cg_spmv_pq(Csr<V> g, const WinDesc* __restrict__ desc, int K,
                                                   const T* __restrict__ p, T* __restrict__ q,
                                                   double* __restrict__ part, const Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ Stage<T, V, typename OpCgSpmvPq<T>::In> st;
    __shared__ double red[NWAVE * 4];
    OpCgSpmvPq<T> op{q, ctrl->pbar};
    my_windows<T, V, AccLin>(g, desc, K, p, op, st, red);
    double v[1] = {op.pq};
    block_sum<1>(v, red);
    store_partials<1>(v, part);
}

// Part 2: mq = M^{-1} q (the partner's q is final now), and the partial sums
// of r^T M^{-1} q = z^T q and q^T M^{-1} q (slots 1 and 2).
template <typename T>
__global__ void __launch_bounds__(WG) k_pair_dots(int n, const T* __restrict__ q, const T* __restrict__ z,
                                                  const int* __restrict__ mate, const float2* __restrict__ pc,
                                                  T* __restrict__ mq, double* __restrict__ part,
                                                  const Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double red[NWAVE * 2];
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const T mt = static_cast<T>(pair_apply(i, q, mate, pc));
        const double m = static_cast<double>(mt);
        const double qi = static_cast<double>(q[i]);
        mq[i] = mt;
        v[0] += static_cast<double>(z[i]) * qi;
        v[1] += qi * m;
    }
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x * NPART + 1] = v[0];
        part[blockIdx.x * NPART + 2] = v[1];
    }
}

// alpha and beta as k_fin_spmv, from p^T q over the SpMV's G1 workgroups and
// the two preconditioned products over k_pair_dots' G2 workgroups.
__global__ void __launch_bounds__(WG) k_fin_pair(int G1, int G2, const double* __restrict__ part,
                                                 Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double red[NWAVE * 3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < G1; b += WG) v[0] += part[b * NPART];
    for (int b = threadIdx.x; b < G2; b += WG) {
        v[1] += part[b * NPART + 1];
        v[2] += part[b * NPART + 2];
    }
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
        const double rz = ctrl->rz, pq = v[0];
        if (rz == 0.0) {
            ctrl->done = CONVERGED;
        } else if (!(pq > 0.0) || !isfinite(pq)) {
            ctrl->done = BREAKDOWN;
        } else {
            const double alpha = rz / pq;
            const double rz_next = rz - 2.0 * alpha * v[1] + alpha * alpha * v[2];
            ctrl->alpha = alpha;
            ctrl->beta = rz_next / rz;
        }
    }
}

// Part 3: x += alpha (p - pbar), r -= alpha q, z -= alpha M^{-1} q (z follows
// r by the same recurrence, so no thread reads a partner's r while it
// changes), p = z + beta p, with the partials of k_cg_update (exact r^T z,
// r^T r, sum p, and with EST the four index estimates) for k_fin_update.
template <typename T, bool EST>
__global__ void __launch_bounds__(WG) k_cg_update_pair(int n, T* __restrict__ x, T* __restrict__ r,
                                                       T* __restrict__ p, const T* __restrict__ q,
                                                       T* __restrict__ z, const T* __restrict__ mq,
                                                       const double* __restrict__ s, double* __restrict__ part,
                                                       const Ctrl* __restrict__ ctrl) {
    static_assert(!EST || std::is_same<T, double>::value, "estimates are for FP64 vectors");
    if (ctrl->done != RUNNING) return;
    __shared__ double red[NWAVE * 7];
    const double alpha = ctrl->alpha, beta = ctrl->beta, pbar = ctrl->pbar;
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const double pi = static_cast<double>(p[i]);
        const T xt = static_cast<T>(static_cast<double>(x[i]) + alpha * (pi - pbar));
        const T rt = static_cast<T>(static_cast<double>(r[i]) - alpha * static_cast<double>(q[i]));
        const T zt = static_cast<T>(static_cast<double>(z[i]) - alpha * static_cast<double>(mq[i]));
        const double zi = static_cast<double>(zt);
        const T pt = static_cast<T>(zi + beta * pi);
        x[i] = xt;
        r[i] = rt;
        z[i] = zt;
        p[i] = pt;
        const double xi = static_cast<double>(xt), ri = static_cast<double>(rt), pn = static_cast<double>(pt);
        (void)xi;
        v[0] += ri * zi;
        v[1] += ri * ri;
        v[2] += pn;
        if constexpr (EST) {
            const double si = s[i];
            v[3] += xi * xi;
            v[4] += xi;
            v[5] += si * xi;
            v[6] += (si - xi) * (si - xi);
        }
    }
    if constexpr (EST) {
        block_sum<7>(v, red);
        store_partials<7>(v, part);
    } else {
        double w[3] = {v[0], v[1], v[2]};
        block_sum<3>(w, red);
        store_partials<3>(w, part);
    }
}

// CG start. mode 0: x = 0, r = s, plus the statistics of s (mean, ||s||^2,
// range). mode 1: restart from the current x with r already holding the true
// residual (written by the epilogue). mode 2: x = 0 with r given (the inner
// solve of FJ_MIXED). All: p = M^{-1} r, the partial sums of rz and rr, and
// mean(r) for k_cg_shift.
// Partial slots: 0 rz, 1 rr, 2 ss, 3 sum s, 4 bad count, 5 sum p, 6 min s,
// 7 max s.
template <typename T>
__global__ void __launch_bounds__(WG) k_cg_init(int n, const double* __restrict__ s, int64_t lds,
                                                T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
                                                const float* __restrict__ minv, int mode,
                                                double* __restrict__ part) {
    __shared__ double red[NWAVE * 8];
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double smin = INFINITY, smax = -INFINITY;
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        double ri;
        if (mode == 0) {
            const double si = s[static_cast<int64_t>(i) * lds];
            x[i] = T(0);
            r[i] = static_cast<T>(si);
            ri = static_cast<double>(r[i]);
            v[2] += si * si;
            v[3] += si;
            if (!(si >= 0.0 && si <= 1.0)) v[4] += 1.0;
            smin = fmin(smin, si);
            smax = fmax(smax, si);
        } else {
            if (mode == 2) x[i] = T(0);
            ri = static_cast<double>(r[i]);
            v[3] += ri;
        }
        const T zt = static_cast<T>(static_cast<double>(minv[i]) * ri);
        if (p != nullptr) p[i] = zt;  // null: statistics only (FP64 side of FJ_MIXED)
        v[0] += ri * static_cast<double>(zt);
        v[1] += ri * ri;
        v[5] += static_cast<double>(zt);
    }
    block_sum<6>(v, red);
    smin = wave_min(smin);
    smax = wave_max(smax);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[NWAVE * 6 + wave] = smin;
        red[NWAVE * 7 + wave] = smax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = red[NWAVE * 6], b = red[NWAVE * 7];
        for (int w = 1; w < NWAVE; ++w) {
            a = fmin(a, red[NWAVE * 6 + w]);
            b = fmax(b, red[NWAVE * 7 + w]);
        }
        double* out = part + blockIdx.x * NPART;
        for (int c = 0; c < 6; ++c) out[c] = v[c];
        out[6] = a;
        out[7] = b;
    }
}

// Every CG solve runs deflated (below) unless FJ_ZERO_START asks for plain
// Jacobi-PCG from 0.
// Move the CG start by the mean of its residual: x += mean(r) 1, r -= mean(r) 1
// (the coarse-space correction of the deflation below). Since (I + L) 1 = 1
// (L 1 = 0, Section 2.1), the new r is exactly the residual of the new x. From
// x = 0 (k_cg_init modes 0 and 2) this starts from mean(s) 1, whose residual
// is the centred s, and the remaining error z - mean(s) 1 is the centred
// solution that Algorithm 1 solves for separately (Section 2.2: Omega 1 = 1),
// whose energy is far smaller than that of z. Runs after k_cg_init and
// k_fin_init (rmean known); k_fin_init mode 1 then takes rz, rr and sum p.
//
// Deflated CG (k_fin_init with deflate = 1) keeps that split for the whole
// solve: with coarse space span{1}, (I + L) 1 = 1 and 1^T (I + L) = 1^T turn
// the deflation projector into centring, P v = v - mean(v) 1. Each step then
// uses q = P (I + L) p, computed as (I + L) p - mean(p) 1 (the two means agree
// because 1^T (I + L) p = 1^T p), and moves x by alpha (p - mean(p) 1), so x
// keeps mean(x) = mean(s) = mean(z) and r stays its residual. The Jacobi-scaled
// operator's smallest eigenvalue, about 1 / (1 + mean degree), belongs to the
// near-constant direction that this removes; on power-law graphs the solve
// needs about a quarter fewer iterations.
template <typename T>
__global__ void __launch_bounds__(WG) k_cg_shift(int n, T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
                                                 const float* __restrict__ minv, const Ctrl* __restrict__ ctrl,
                                                 double* __restrict__ part) {
    __shared__ double red[NWAVE * 3];
    const double mu = ctrl->rmean;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        x[i] = static_cast<T>(static_cast<double>(x[i]) + mu);
        const T rt = static_cast<T>(static_cast<double>(r[i]) - mu);
        r[i] = rt;
        const double ri = static_cast<double>(rt);
        const T zt = static_cast<T>(static_cast<double>(minv[i]) * ri);
        p[i] = zt;
        v[0] += ri * static_cast<double>(zt);
        v[1] += ri * ri;
        v[2] += static_cast<double>(zt);
    }
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
        double* out = part + blockIdx.x * NPART;
        out[0] = v[0];
        out[1] = v[1];
        out[2] = out[3] = out[4] = 0.0;
        out[5] = v[2];
        out[6] = INFINITY;
        out[7] = -INFINITY;
    }
}

__global__ void __launch_bounds__(WG) k_fin_init(int G, int n, const double* __restrict__ part, int mode,
                                                 double rtol2, int max_iter, int range_check,
                                                 Ctrl* __restrict__ ctrl, double eps_stop, int deflate) {
    __shared__ double red[NWAVE * 6];
    __shared__ double mm[2 * NWAVE];
    double v[6];
    total_partials<6>(G, part, v, red);
    double a = INFINITY, b = -INFINITY;
    for (int k = threadIdx.x; k < G; k += WG) {
        a = fmin(a, part[k * NPART + 6]);
        b = fmax(b, part[k * NPART + 7]);
    }
    a = wave_min(a);
    b = wave_max(b);
    if ((threadIdx.x & 63) == 0) {
        mm[threadIdx.x >> 6] = a;
        mm[NWAVE + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (mode == 0) {
            for (int w = 1; w < NWAVE; ++w) {
                a = fmin(a, mm[w]);
                b = fmax(b, mm[NWAVE + w]);
            }
            ctrl->smin = a;
            ctrl->smax = b;
            ctrl->ss = v[2];
            ctrl->mu = v[3] / static_cast<double>(n);
            ctrl->bad = v[4] > 0.0 ? 2 : 0;
            ctrl->iters = 0;
            ctrl->max_iter = max_iter;
        }
        if (mode == 2) {  // the inner solve of FJ_MIXED: tolerance relative to its own right-hand side
            ctrl->ss = v[1];
            ctrl->iters = 0;
            ctrl->max_iter = max_iter;
            ctrl->bad = 0;
        }
        ctrl->tol2 = rtol2 * ctrl->ss;
        ctrl->eps_stop = eps_stop;
        ctrl->deflate = deflate;
        ctrl->pbar = deflate ? v[5] / static_cast<double>(n) : 0.0;
        ctrl->rmean = v[3] / static_cast<double>(n);
        ctrl->rz = v[0];
        ctrl->rr = v[1];
        ctrl->hist[ctrl->iters % HIST] = v[1];
        if (range_check && ctrl->bad) ctrl->done = BAD_INPUT;
        else if (!isfinite(v[1])) ctrl->done = BREAKDOWN;
        else if (v[1] <= ctrl->tol2) ctrl->done = CONVERGED;
        else if (ctrl->iters >= ctrl->max_iter) ctrl->done = ITER_CAP;
        else ctrl->done = RUNNING;
    }
}

// Epilogue: one pass over the CSR at z. Writes r = s - (I+L)z (for a restart)
// and the partial sums of OpEpilogue; k_fin_epilogue turns them into
//   res[0] C_I  = ||L z||^2           res[5] ||r||_2
//   res[1] D    = half the row sums    res[6] ||s||_2
//   res[2] P    = sum (z - mean z)^2   res[7] sum (z_i - s_i)^2
//   res[3] C    = ||z||^2              res[8] sum z
//   res[4] I_dc = s^T z                res[9] z^T r
// and bound[] (relative error bounds, see k_fin_epilogue).
template <typename V>
__global__ void __launch_bounds__(WG) k_epilogue(Csr<V> g, const WinDesc* __restrict__ desc, int K,
                                                 const double* __restrict__ z, const double* __restrict__ s,
                                                 int64_t lds, double* __restrict__ rbuf,
                                                 double* __restrict__ part, const Ctrl* __restrict__ ctrl) {
    __shared__ Stage<double, V, OpEpilogue::In> st;
    __shared__ double red[NWAVE * 9];
    OpEpilogue op{s, lds, ctrl->mu, rbuf};
    my_windows<double, V, AccLinSq>(g, desc, K, z, op, st, red);
    double v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = op.v[c];
    block_sum<9>(v, red);
    store_partials<9>(v, part);
}

__global__ void __launch_bounds__(WG) k_fin_epilogue(int G, int n_nodes, const double* __restrict__ part,
                                                     Ctrl* __restrict__ ctrl) {
    __shared__ double red[NWAVE * 9];
    double v[9];
    total_partials<9>(G, part, v, red);
    if (threadIdx.x == 0) {
        const double n = static_cast<double>(n_nodes);
        const double dev = v[4] - n * ctrl->mu;  // n (mean z - mu)
        double idx[5];
        idx[0] = v[0];
        idx[1] = 0.5 * v[1];
        idx[2] = fmax(v[2] - dev * dev / n, 0.0);
        idx[3] = v[3];
        idx[4] = v[5];
        const double rho = sqrt(v[6]);
        for (int c = 0; c < 5; ++c) ctrl->res[c] = idx[c];
        ctrl->res[5] = rho;
        ctrl->res[6] = sqrt(ctrl->ss);
        ctrl->res[7] = v[8];
        ctrl->res[8] = v[4];
        ctrl->res[9] = v[7];
        // With e = z_true - z = (I+L)^{-1} r and I <= I + L: ||e||, ||L e||,
        // ||e - mean(e) 1|| <= rho and ||W^{1/2} B e|| <= rho / 2, hence
        // |sqrt(X) - sqrt(X~)| <= rho_X and |X - X~| / X <= rho_X (2 sqrt(X~) + rho_X) / (sqrt(X~) - rho_X)^2.
        // For I_dc = s^T z: |s^T e| = |z_true^T r| <= (||z|| + rho) rho.
        // 1e-13 covers rounding in the FP64 sums themselves.
        const double rhos[4] = {rho, 0.5 * rho, rho, rho};
        for (int c = 0; c < 4; ++c) {
            const double rx = sqrt(idx[c]);
            const double rh = rhos[c];
            ctrl->bound[c] = (rx > rh) ? rh * (2.0 * rx + rh) / ((rx - rh) * (rx - rh)) + 1e-13 : INFINITY;
        }
        const double a = (sqrt(idx[3]) + rho) * rho;
        ctrl->bound[4] = (idx[4] > a) ? a / (idx[4] - a) + 1e-13 : INFINITY;
    }
}

// FJ_MIXED: the inner right-hand side r32 = f32(r / ||r||). mode 0 takes
// ||r|| = ||s|| (first step, z = 0 and r = s, from init), mode 1 the epilogue's
// true residual norm.
__global__ void __launch_bounds__(WG) k_mixed_cast(int n, const double* __restrict__ r64, float* __restrict__ r32,
                                                   int mode, const Ctrl* __restrict__ outer) {
    const double rho = mode == 0 ? sqrt(outer->ss) : outer->res[5];
    const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG)
        r32[i] = static_cast<float>(r64[i] * inv);
}

// FJ_MIXED: the FP64 correction z += ||r|| * f64(d), d the inner solution.
__global__ void __launch_bounds__(WG) k_mixed_refine(int n, double* __restrict__ z, const float* __restrict__ d,
                                                     int mode, const Ctrl* __restrict__ outer) {
    const double rho = mode == 0 ? sqrt(outer->ss) : outer->res[5];
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG)
        z[i] += rho * static_cast<double>(d[i]);
}

// Clear the control block before a solve (a kernel rather than a memset so
// that the sequence can be captured in a HIP graph).
__global__ void k_ctrl_reset(Ctrl* __restrict__ ctrl, int count) {
    const int words = static_cast<int>(sizeof(Ctrl) / sizeof(uint32_t)) * count;
    uint32_t* w = reinterpret_cast<uint32_t*>(ctrl);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) w[i] = 0u;
}

// CSR contract checks (fj_prepare with FJ_VALIDATE_GRAPH). Sets bits of *flags:
//   1 row_ptr[0] != 0 or row_ptr[n] != nnz   2 row_ptr decreasing or out of [0, nnz]
//   4 column out of range   8 self-loop   16 columns not strictly increasing in a row
//   32 weight not finite or <= 0   64 not symmetric (reverse entry missing or weight differs)
template <typename V>
__global__ void __launch_bounds__(WG) k_validate(Csr<V> g, int64_t nnz, int* __restrict__ flags) {
    const int n = g.n;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * WG;
    for (int64_t i = tid; i <= n; i += stride) {
        const int a = g.row_ptr[i];
        if (a < 0 || a > nnz) atomicOr(flags, 2);
        if (i == 0 && a != 0) atomicOr(flags, 1);
        if (i == n && a != nnz) atomicOr(flags, 1);
        if (i < n && g.row_ptr[i + 1] < a) atomicOr(flags, 2);
    }
    for (int64_t e = tid; e < nnz; e += stride) {
        // row of entry e: the last i in [0, n) with row_ptr[i] <= e
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (g.row_ptr[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int i = lo;
        const int j = g.col[e];
        if (j < 0 || j >= n) {
            atomicOr(flags, 4);
            continue;
        }
        if (j == i) atomicOr(flags, 8);
        const int rend = g.row_ptr[i + 1];
        if (e + 1 < rend && rend <= nnz && g.col[e + 1] <= j) atomicOr(flags, 16);
        const double w = weight_at<V>(g.val, e);
        if (!(w > 0.0) || !isfinite(w)) atomicOr(flags, 32);
        int a = g.row_ptr[j], b = g.row_ptr[j + 1];
        if (a < 0 || b > nnz || b < a) continue;  // reported by the row_ptr checks
        int found = -1;
        while (a < b) {  // binary search for i in row j
            const int mid = (a + b) >> 1;
            const int c = g.col[mid];
            if (c == i) { found = mid; break; }
            if (c < i) a = mid + 1;
            else b = mid;
        }
        if (found < 0 || weight_at<V>(g.val, found) != w) atomicOr(flags, 64);
    }
}

}  // namespace fj
