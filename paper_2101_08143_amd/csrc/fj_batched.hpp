// fj_batched.hpp -- k right-hand sides at once (HIP, gfx950).
//
// Vectors are node-major blocks: element (i, c) of X lives at X[i * KB + c],
// KB = the number of columns rounded up to a power of two (2..64); padding
// columns hold zeros and converge at once. The sparse pass gives each row a
// group of KB lanes, lane c owning column c: the group loads up to KB column
// indices and weights of the row with one coalesced load, broadcasts them
// lane to lane, and every neighbour j becomes one contiguous KB-wide read of
// X[j, :] (256 bytes for 64 FP32 columns). The CSR is thus read once per
// iteration for all k solves, and the gather reads whole rows instead of
// scattered elements.
//
// Every column runs its own CG (own alpha, beta, stopping test) on the shared
// operator pass. A column's arithmetic is the same whatever else is in the
// batch: its row sums run over the CSR in order on one lane, and its dot
// products are reduced over a fixed row-to-workgroup assignment in a fixed
// order. Results are therefore bitwise identical alone or batched, for the
// same KB.
#pragma once

#include "fj_kernels.hpp"

namespace fj {

constexpr int KMAX = 64;       // columns per block
constexpr int BPART = 16;      // partial sums per (workgroup, column)

// Per-column squared relative tolerances, passed by value to the batched
// start kernel so that no column's target depends on the others.
struct ColumnTol {
    double rtol2[KMAX];
};

__device__ __forceinline__ double shfl_d(double v, int src, int width) {
    return __shfl(v, src, width);
}

// CPL consecutive columns of one node as doubles: one vector load per 16 bytes.
template <typename T, int CPL>
__device__ __forceinline__ void load_cols(const T* __restrict__ p, double (&out)[CPL]) {
    if constexpr (std::is_same<T, double>::value && CPL >= 2) {
#pragma unroll
        for (int h = 0; h < CPL / 2; ++h) {
            const double2 v = reinterpret_cast<const double2*>(p)[h];
            out[2 * h] = v.x;
            out[2 * h + 1] = v.y;
        }
    } else if constexpr (std::is_same<T, float>::value && CPL == 4) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else if constexpr (std::is_same<T, float>::value && CPL == 2) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        out[0] = v.x; out[1] = v.y;
    } else {
#pragma unroll
        for (int q = 0; q < CPL; ++q) out[q] = static_cast<double>(p[q]);
    }
}

// LDS of the batched window pass: the window's column indices, weights and
// row ends (staged with coalesced loads), and per group the sums of the row
// its item range ends inside of (also reused to combine a long last row).
template <typename V, int KB, int CPL>
struct SpmmStage {
    static constexpr int NG = WG / (KB / CPL);
    int col[STAGE];
    typename WeightReg<V>::type w[std::is_same<V, Unit>::value ? 1 : STAGE];
    int rend[WIN + 1];
    double plin[NG * KB];
    double psq[NG * KB];
};

// The windows k0, k0 + G, ... of the workgroup (k0 = blockIdx.x). A group of
// GW = KB / CPL lanes works like one thread of the single-vector pass: lane l
// owns columns l*CPL .. l*CPL + CPL - 1, and group g walks the items
// (entries and row ends, in CSR order) [g*ipg, (g+1)*ipg) of the window, so
// every group gets the same share of the window whatever the row lengths.
// Each entry costs one CPL-wide gather per lane (the group reads the
// neighbour's KB values as one contiguous run). op.row(i, q, c, x_ic,
// sum_j w_ij (x_ic - x_jc), sum_j w_ij (x_ic - x_jc)^2) is called once per row
// and column, by the group holding the row's end; a row begun in earlier
// groups first adds their partial sums, in group order. Each column's row
// sum thus follows a fixed order set by the data alone. A long last row is
// split over all groups and combined in group order.
template <typename T, typename V, typename Acc, int KB, int CPL, typename Op>
__device__ __forceinline__ void spmm_windows(const Csr<V>& g, const WinDesc* __restrict__ desc, int K,
                                             const T* __restrict__ X, Op& op, SpmmStage<V, KB, CPL>& st) {
    static_assert(KB % CPL == 0, "CPL must divide KB");
    constexpr int GW = KB / CPL;
    constexpr int NG = WG / GW;
    constexpr bool WEIGHTED = !std::is_same<V, Unit>::value;
    const int tid = threadIdx.x;
    const int lane = tid % GW;
    const int grp = tid / GW;
    const int c0 = lane * CPL;

    for (int k = blockIdx.x; k < K; k += gridDim.x) {
        const WinDesc d = to_scalar(load_raw_desc(desc + k));
        const int nrs = d.nrs, ns = d.ns;
        for (int e = tid; e < ns; e += WG) {
            st.col[e] = stream_load(&g.col[d.e0 + e]);
            if constexpr (WEIGHTED) st.w[e] = stream_load(&g.val[d.e0 + e]);
        }
        for (int a = tid; a < nrs; a += WG) st.rend[a] = g.row_ptr[d.r0 + a + 1] - d.e0;
        __syncthreads();
        const int total = nrs + ns;
        const int ipg = (total + NG - 1) / NG;
        const int i0 = min(grp * ipg, total);
        const int i1 = min(i0 + ipg, total);
        int lo = 0, hi = nrs;
        while (lo < hi) {  // a0 = number of row ends before item i0 (row a's end is item rend[a] + a)
            const int mid = (lo + hi) >> 1;
            if (st.rend[mid] + mid < i0) lo = mid + 1;
            else hi = mid;
        }
        const int a0 = lo;
        int a = a0;
        int j = i0 - a0;
        const bool continued = (i0 < i1) && (j > (a0 > 0 ? st.rend[a0 - 1] : 0));
        int row_end = a < nrs ? st.rend[a] : 0;
        double xi[CPL], lin[CPL], sq[CPL], flin[CPL], fsq[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) lin[q] = sq[q] = flin[q] = fsq[q] = 0.0;
        if (a < nrs) load_cols<T, CPL>(X + static_cast<int64_t>(d.r0 + a) * KB + c0, xi);
        bool first_pending = false;
        int dd = i0;
        while (dd < i1) {
            if (j < row_end) {  // a run of entries of row a
                const int run = min(row_end - j, i1 - dd);
                int u = 0;
                for (; u + 4 <= run; u += 4) {  // four gathers in flight
                    int jj[4];
                    double w[4], xj[4][CPL];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        jj[v] = st.col[j + u + v];
                        w[v] = WEIGHTED ? static_cast<double>(st.w[j + u + v]) : 1.0;
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) load_cols<T, CPL>(X + static_cast<int64_t>(jj[v]) * KB + c0, xj[v]);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
#pragma unroll
                        for (int q = 0; q < CPL; ++q) {
                            const double df = xi[q] - xj[v][q];
                            lin[q] += w[v] * df;
                            if constexpr (Acc::SQ) sq[q] += w[v] * df * df;
                        }
                    }
                }
                if (u < run) {  // the last 1-3 entries of the run in one round (as in spmm_rows)
                    int jj[4];
                    double w[4], xj[4][CPL];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int at = j + min(u + v, run - 1);
                        jj[v] = st.col[at];
                        w[v] = WEIGHTED ? static_cast<double>(st.w[at]) : 1.0;
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) load_cols<T, CPL>(X + static_cast<int64_t>(jj[v]) * KB + c0, xj[v]);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (u + v >= run) break;  // uniform over the lane group
#pragma unroll
                        for (int q = 0; q < CPL; ++q) {
                            const double df = xi[q] - xj[v][q];
                            lin[q] += w[v] * df;
                            if constexpr (Acc::SQ) sq[q] += w[v] * df * df;
                        }
                    }
                }
                j += run;
                dd += run;
            } else {  // end of row a
                if (a == a0 && continued) {
                    first_pending = true;
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        flin[q] = lin[q];
                        fsq[q] = sq[q];
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < CPL; ++q) op.row(d.r0 + a, q, c0 + q, xi[q], lin[q], sq[q]);
                }
#pragma unroll
                for (int q = 0; q < CPL; ++q) lin[q] = sq[q] = 0.0;
                ++a;
                ++dd;
                if (a < nrs) {
                    row_end = st.rend[a];
                    load_cols<T, CPL>(X + static_cast<int64_t>(d.r0 + a) * KB + c0, xi);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < CPL; ++q) {  // the row still open at the end of the range
            st.plin[grp * KB + c0 + q] = lin[q];
            if constexpr (Acc::SQ) st.psq[grp * KB + c0 + q] = sq[q];
        }
        __syncthreads();
        if (first_pending) {  // groups t0 .. grp-1 hold the rest of row a0
            const int t0 = (a0 > 0 ? st.rend[a0 - 1] + a0 : 0) / ipg;
            double xr[CPL];
            load_cols<T, CPL>(X + static_cast<int64_t>(d.r0 + a0) * KB + c0, xr);
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                double L = flin[q], S = fsq[q];
                for (int t = grp - 1; t >= t0; --t) {
                    L += st.plin[t * KB + c0 + q];
                    if constexpr (Acc::SQ) S += st.psq[t * KB + c0 + q];
                }
                op.row(d.r0 + a0, q, c0 + q, xr[q], L, S);
            }
        }
        if (d.long_last) {  // workgroup-uniform
            __syncthreads();  // plin / psq are reused below
            const int i = d.r1 - 1;
            double xl[CPL], L[CPL], Sq[CPL];
            load_cols<T, CPL>(X + static_cast<int64_t>(i) * KB + c0, xl);
#pragma unroll
            for (int q = 0; q < CPL; ++q) L[q] = Sq[q] = 0.0;
            // group gr takes entry chunks elast + gr*GW, elast + (gr+NG)*GW, ...; lane l loads entry l of a chunk
            for (int e0 = d.elast + grp * GW; e0 < d.eend; e0 += NG * GW) {
                const int e = e0 + lane;
                int jl = 0;
                double wl = 0.0;
                if (e < d.eend) {
                    jl = g.col[e];
                    wl = weight_at<V>(g.val, e);
                }
                const int cnt = min(GW, d.eend - e0);
                for (int t = 0; t < cnt; ++t) {
                    const int jc = __shfl(jl, t, GW);
                    const double w = WEIGHTED ? shfl_d(wl, t, GW) : 1.0;
                    double xj[CPL];
                    load_cols<T, CPL>(X + static_cast<int64_t>(jc) * KB + c0, xj);
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        const double df = xl[q] - xj[q];
                        L[q] += w * df;
                        if constexpr (Acc::SQ) Sq[q] += w * df * df;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                st.plin[grp * KB + c0 + q] = L[q];
                st.psq[grp * KB + c0 + q] = Sq[q];
            }
            __syncthreads();
            if (grp == 0) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    double LL = 0.0, SS = 0.0;
#pragma unroll 4  // fully unrolled, the group loads of narrow blocks cost up to 100 registers
                    for (int gr = 0; gr < NG; ++gr) {
                        LL += st.plin[gr * KB + c0 + q];
                        SS += st.psq[gr * KB + c0 + q];
                    }
                    op.row(i, q, c0 + q, xl[q], LL, SS);
                }
            }
        }
        __syncthreads();  // LDS is reused by the next window
    }
}

// Row-per-group variant of the window pass (an autotuner candidate for wide
// blocks): the rows of the workgroup's windows (blockIdx.x, +gridDim.x, ...).
// A row is owned by a group of GW = KB / CPL lanes; lane l of the group owns columns
// l*CPL .. l*CPL + CPL - 1 and calls op.row(i, q, c, x_ic,
// sum_j w_ij (x_ic - x_jc), sum_j w_ij (x_ic - x_jc)^2) for each of them
// (q = c - l*CPL). Each column's row sum runs over the row's entries in CSR
// order whatever CPL is. A long last row is split over all groups of the
// workgroup and combined in LDS in group order. lred must hold
// 2 * WG * CPL doubles. The block's rows are LDX values apart: a pass may
// cover KB of LDX columns (X then points at the pass's first column).
template <typename T, typename V, typename Acc, int KB, int CPL, int LDX, typename Op>
__device__ __forceinline__ void spmm_rows(const Csr<V>& g, const WinDesc* __restrict__ desc, int K,
                                             const T* __restrict__ X, Op& op, double* lred) {
    static_assert(KB % CPL == 0, "CPL must divide KB");
    constexpr int GW = KB / CPL;
    constexpr int NG = WG / GW;
    constexpr bool WEIGHTED = !std::is_same<V, Unit>::value;
    const int lane = threadIdx.x % GW;
    const int grp = threadIdx.x / GW;
    const int c0 = lane * CPL;

    auto row_sum = [&](int e_begin, int e_end, const double (&xi)[CPL], double (&lin)[CPL], double (&sq)[CPL]) {
        for (int e0 = e_begin; e0 < e_end; e0 += GW) {
            const int e = e0 + lane;
            int jl = 0;
            double wl = 0.0;
            if (e < e_end) {
                jl = g.col[e];
                wl = weight_at<V>(g.val, e);
            }
            const int cnt = min(GW, e_end - e0);
            int t = 0;
            for (; t + 4 <= cnt; t += 4) {  // four gathers in flight
                int j[4];
                double w[4], xj[4][CPL];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    j[u] = __shfl(jl, t + u, GW);
                    w[u] = WEIGHTED ? shfl_d(wl, t + u, GW) : 1.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) load_cols<T, CPL>(X + static_cast<int64_t>(j[u]) * LDX + c0, xj[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        const double d = xi[q] - xj[u][q];
                        lin[q] += w[u] * d;
                        if constexpr (Acc::SQ) sq[q] += w[u] * d * d;
                    }
                }
            }
            if (t < cnt) {  // the last 1-3 entries in one round: slots past the end repeat the last
                int j[4];      // entry's address (a cached line) and are not summed
                double w[4], xj[4][CPL];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int tu = min(t + u, cnt - 1);
                    j[u] = __shfl(jl, tu, GW);
                    w[u] = WEIGHTED ? shfl_d(wl, tu, GW) : 1.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) load_cols<T, CPL>(X + static_cast<int64_t>(j[u]) * LDX + c0, xj[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (t + u >= cnt) break;  // uniform over the lane group
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        const double d = xi[q] - xj[u][q];
                        lin[q] += w[u] * d;
                        if constexpr (Acc::SQ) sq[q] += w[u] * d * d;
                    }
                }
            }
        }
    };

    for (int k = blockIdx.x; k < K; k += gridDim.x) {
        const WinDesc d = to_scalar(load_raw_desc(desc + k));
        for (int a = grp; a < d.nrs; a += NG) {
            const int i = d.r0 + a;
            double xi[CPL], lin[CPL], sq[CPL];
            load_cols<T, CPL>(X + static_cast<int64_t>(i) * LDX + c0, xi);
#pragma unroll
            for (int q = 0; q < CPL; ++q) lin[q] = sq[q] = 0.0;
            row_sum(g.row_ptr[i], g.row_ptr[i + 1], xi, lin, sq);
#pragma unroll
            for (int q = 0; q < CPL; ++q) op.row(i, q, c0 + q, xi[q], lin[q], sq[q]);
        }
        if (d.long_last) {  // workgroup-uniform
            const int i = d.r1 - 1;
            double xi[CPL], lin[CPL], sq[CPL];
            load_cols<T, CPL>(X + static_cast<int64_t>(i) * LDX + c0, xi);
#pragma unroll
            for (int q = 0; q < CPL; ++q) lin[q] = sq[q] = 0.0;
            // group gr takes entry chunks elast + gr*GW, elast + (gr+NG)*GW, ...
            for (int e0 = d.elast + grp * GW; e0 < d.eend; e0 += NG * GW)
                row_sum(e0, min(e0 + GW, d.eend), xi, lin, sq);
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                lred[grp * KB + c0 + q] = lin[q];
                lred[NG * KB + grp * KB + c0 + q] = sq[q];
            }
            __syncthreads();
            if (grp == 0) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    double L = 0.0, S = 0.0;
                    for (int gr = 0; gr < NG; ++gr) {
                        L += lred[gr * KB + c0 + q];
                        S += lred[NG * KB + gr * KB + c0 + q];
                    }
                    op.row(i, q, c0 + q, xi[q], L, S);
                }
            }
            __syncthreads();
        }
    }
}

// Per-column workgroup sums of N accumulators: lane l of every group holds
// the workgroup's share for columns l*CPL + q in v[a][q]; groups are added in
// order and the result goes to part[(blockIdx.x * LDP + coff + c) * BPART + a]
// (LDP columns per workgroup row; a column pass writes at its offset coff).
// C sums at a time (lred holds C * WG * CPL doubles), so that a kernel can
// reduce through LDS it already owns.
template <int N, int KB, int CPL, int C = N, int LDP = KB>
__device__ __forceinline__ void store_column_partials(const double (&v)[N][CPL], double* lred,
                                                      double* __restrict__ part, int coff = 0) {
    constexpr int GW = KB / CPL;
    constexpr int NG = WG / GW;
    static_assert(C * WG * CPL <= 12 * WG, "LDS buffer too small");
    const int lane = threadIdx.x % GW, grp = threadIdx.x / GW;
    for (int a0 = 0; a0 < N; a0 += C) {
        const int na = N - a0 < C ? N - a0 : C;
        for (int a = 0; a < na; ++a)
            for (int q = 0; q < CPL; ++q) lred[a * NG * KB + grp * KB + lane * CPL + q] = v[a0 + a][q];
        __syncthreads();
        if (threadIdx.x < KB) {
            for (int a = 0; a < na; ++a) {
                double t = 0.0;
                for (int gr = 0; gr < NG; ++gr) t += lred[a * NG * KB + gr * KB + threadIdx.x];
                part[(static_cast<int64_t>(blockIdx.x) * LDP + coff + threadIdx.x) * BPART + a0 + a] = t;
            }
        }
        __syncthreads();
    }
}

// Totals of N partials of column c = blockIdx.x over G workgroups, for a
// finalize kernel launched with one workgroup per column: thread t adds
// workgroups t, t + WG, ... in order, then the workgroup adds the threads'
// sums in a fixed order. Every thread receives the totals.
template <int N, int KB>
__device__ __forceinline__ void column_totals(int G, const double* __restrict__ part, double (&v)[N],
                                              double* red) {
    const int c = blockIdx.x;
#pragma unroll
    for (int a = 0; a < N; ++a) v[a] = 0.0;
    for (int b = threadIdx.x; b < G; b += WG) {
        const double* p = part + (static_cast<int64_t>(b) * KB + c) * BPART;
#pragma unroll
        for (int a = 0; a < N; ++a) v[a] += p[a];
    }
    block_sum<N>(v, red);
}

// ------------------------------------------------------------ row operations

template <typename T, int KB, int CPL, int LDX = KB>
struct OpSpmmCg {  // Q = (I + L) P and per-column p^T q, r^T M^{-1} q, q^T M^{-1} q
    const T* __restrict__ R;
    const float* __restrict__ minv;
    T* __restrict__ Q;
    double shift[CPL] = {};  // deflated columns: mean of P's column (see k_cg_shift)
    double v[3][CPL] = {};
    __device__ void row(int i, int q, int c, double pi, double lin, double) {
        const int64_t at = static_cast<int64_t>(i) * LDX + c;
        const T qt = static_cast<T>(pi + lin - shift[q]);
        // Q and R stream through once: non-temporal, so the L2 keeps the gathered rows of P
        __builtin_nontemporal_store(qt, Q + at);
        const double qd = static_cast<double>(qt);
        const double mq = static_cast<double>(minv[i]) * qd;
        v[0][q] += pi * qd;
        v[1][q] += static_cast<double>(__builtin_nontemporal_load(R + at)) * mq;
        v[2][q] += qd * mq;
    }
};

template <int KB>
struct OpSpmmEpilogue {  // per column: the sums of OpEpilogue; R is written for columns in mask only
    const double* __restrict__ S;
    int64_t lds;
    int k;
    uint64_t mask;
    const Ctrl* __restrict__ ctrl;
    double* __restrict__ R;
    double v[9][1] = {};
    __device__ void row(int i, int, int c, double zi, double t, double dsq) {
        const double si = c < k ? S[static_cast<int64_t>(i) * lds + c] : 0.0;
        const double ri = si - zi - t;
        if ((mask >> c) & 1ull) R[static_cast<int64_t>(i) * KB + c] = ri;
        const double dm = zi - ctrl[c].mu;
        const double dz = zi - si;
        v[0][0] += t * t;
        v[1][0] += dsq;
        v[2][0] += dm * dm;
        v[3][0] += zi * zi;
        v[4][0] += zi;
        v[5][0] += si * zi;
        v[6][0] += ri * ri;
        v[7][0] += zi * ri;
        v[8][0] += dz * dz;
    }
};

// ------------------------------------------------------------ kernels

// SPLIT: merge-path item split over lane groups (spmm_windows); otherwise one
// group per row (spmm_rows). LDX > KB: one column pass over columns
// [coff, coff + KB) of LDX-wide blocks (rows design only): every pass reads
// the CSR again, but gathers rows of KB instead of LDX values, which keeps a
// wide block's gathered part inside the Infinity Cache.
template <typename V, typename T, int KB, int CPL, bool SPLIT, int LDX = KB>
__global__ void __launch_bounds__(WG) k_spmm_cg(Csr<V> g, const WinDesc* __restrict__ desc, int K,
                                                const T* __restrict__ P, const T* __restrict__ R,
                                                const float* __restrict__ minv, T* __restrict__ Q,
                                                double* __restrict__ part, const Ctrl* __restrict__ ctrl,
                                                int coff = 0) {
    static_assert(LDX == KB || !SPLIT, "column passes use the rows design");
    P += coff;
    R += coff;
    Q += coff;
    if (ctrl != nullptr) ctrl += coff;
    // launches queued past the last column's stop return at once; ctrl null
    // (the autotuner's timing runs): every column, no shift
    __shared__ int live;
    if (threadIdx.x == 0) live = ctrl == nullptr ? 1 : 0;
    __syncthreads();
    if (ctrl != nullptr && threadIdx.x < KB && ctrl[threadIdx.x].done == RUNNING) live = 1;
    __syncthreads();
    if (!live) return;
    OpSpmmCg<T, KB, CPL, LDX> op{R, minv, Q};
    if (ctrl != nullptr) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) op.shift[q] = ctrl[(threadIdx.x % (KB / CPL)) * CPL + q].pbar;
    }
    if constexpr (SPLIT) {
        __shared__ SpmmStage<V, KB, CPL> st;
        static_assert(sizeof(st) >= 3 * WG * CPL * sizeof(double), "stage too small to reuse for the partials");
        spmm_windows<T, V, AccLin, KB, CPL>(g, desc, K, P, op, st);
        // the window pass ended with a barrier: its LDS now holds the partial sums
        store_column_partials<3, KB, CPL>(op.v, reinterpret_cast<double*>(&st), part);
    } else {
        __shared__ double lred[12 * WG];
        spmm_rows<T, V, AccLin, KB, CPL, LDX>(g, desc, K, P, op, lred);
        store_column_partials<3, KB, CPL, 3, LDX>(op.v, lred, part, coff);
    }
}

template <int KB>
__global__ void __launch_bounds__(WG) k_fin_spmm(int G, const double* __restrict__ part, Ctrl* __restrict__ ctrl) {
    Ctrl& c = ctrl[blockIdx.x];  // one workgroup per column
    if (c.done != RUNNING) return;
    __shared__ double red[NWAVE * 3];
    double tot[3];
    column_totals<3, KB>(G, part, tot, red);
    if (threadIdx.x == 0) {
        const double rz = c.rz, pq = tot[0];
        if (rz == 0.0) {
            c.done = CONVERGED;
        } else if (!(pq > 0.0) || !isfinite(pq)) {
            c.done = BREAKDOWN;
        } else {
            const double alpha = rz / pq;
            const double rz_next = rz - 2.0 * alpha * tot[1] + alpha * alpha * tot[2];
            c.alpha = alpha;
            c.beta = rz_next / rz;
        }
    }
}

// Element-wise CG update of every running column; thread t always handles
// column t % KB (the grid stride is a multiple of KB).
// EST (FP64): also, per column, the sums that estimate the five indices at the
// new x (see k_cg_update): x^T x, sum x, s^T x, ||s - x||^2, with s read from
// S (column c of node i at S[i * lds + c], zero for c >= k). Only columns
// whose residual is already within a factor 100 of their target pay for
// the extra read (est_window); the others cannot stop early yet.
__device__ __forceinline__ bool est_window(const Ctrl& c) { return c.eps_stop > 0.0 && c.rr <= 1e4 * c.tol2; }

template <typename T, int KB, bool EST>
__global__ void __launch_bounds__(WG) k_update_batched(int n, T* __restrict__ X, T* __restrict__ R,
                                                       T* __restrict__ P, const T* __restrict__ Q,
                                                       const float* __restrict__ minv,
                                                       const double* __restrict__ S, int64_t lds, int k,
                                                       double* __restrict__ part, const Ctrl* __restrict__ ctrl) {
    static_assert(!EST || std::is_same<T, double>::value, "estimates are for FP64 vectors");
    __shared__ double lred[12 * WG];
    const int c = threadIdx.x % KB;
    const bool run = ctrl[c].done == RUNNING;
    const bool est = EST && est_window(ctrl[c]);
    const double alpha = ctrl[c].alpha, beta = ctrl[c].beta, pbar = ctrl[c].pbar;
    double v[3] = {0.0, 0.0, 0.0};
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t total = static_cast<int64_t>(n) * KB;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * WG;
    auto est_add = [&](int i, T x) {
        const double xi = static_cast<double>(x);
        const double si = c < k ? S[static_cast<int64_t>(i) * lds + c] : 0.0;
        e[0] += xi * xi;
        e[1] += xi;
        e[2] += si * xi;
        e[3] += (si - xi) * (si - xi);
    };
    if (run) {
        int64_t e0 = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x;
        for (; e0 + stride < total; e0 += 2 * stride) {  // two elements' loads in flight
            const int64_t e1 = e0 + stride;
            const int i0 = static_cast<int>(e0 / KB), i1 = static_cast<int>(e1 / KB);
            T x0 = X[e0], r0 = R[e0], p0 = P[e0], q0 = Q[e0];
            T x1 = X[e1], r1 = R[e1], p1 = P[e1], q1 = Q[e1];
            const float m0 = minv[i0], m1 = minv[i1];
            cg_update_elem(alpha, beta, pbar, x0, r0, p0, q0, m0, v);
            cg_update_elem(alpha, beta, pbar, x1, r1, p1, q1, m1, v);
            X[e0] = x0;
            R[e0] = r0;
            P[e0] = p0;
            X[e1] = x1;
            R[e1] = r1;
            P[e1] = p1;
            if (EST && est) {
                est_add(i0, x0);
                est_add(i1, x1);
            }
        }
        if (e0 < total) {
            const int i = static_cast<int>(e0 / KB);
            T x = X[e0], r = R[e0], p = P[e0];
            cg_update_elem(alpha, beta, pbar, x, r, p, Q[e0], minv[i], v);
            X[e0] = x;
            R[e0] = r;
            P[e0] = p;
            if (EST && est) est_add(i, x);
        }
    }
    if constexpr (EST) {
        const double vv[7][1] = {{v[0]}, {v[1]}, {v[2]}, {e[0]}, {e[1]}, {e[2]}, {e[3]}};
        store_column_partials<7, KB, 1>(vv, lred, part);
    } else {
        const double vv[3][1] = {{v[0]}, {v[1]}, {v[2]}};
        store_column_partials<3, KB, 1>(vv, lred, part);
    }
}

template <int KB, bool EST>
__global__ void __launch_bounds__(WG) k_fin_update_batched(int G, int n, const double* __restrict__ part,
                                                           Ctrl* __restrict__ ctrl) {
    Ctrl& c = ctrl[blockIdx.x];  // one workgroup per column
    if (c.done != RUNNING) return;
    constexpr int NV = EST ? 7 : 3;
    __shared__ double red[NWAVE * NV];
    double tot[NV];
    column_totals<NV, KB>(G, part, tot, red);
    if (threadIdx.x == 0) {
        const bool est_on = EST && est_window(c);  // decided on the residual the update saw
        const double rz = tot[0], rr = tot[1];
        const int it = c.iters + 1;
        c.iters = it;
        c.rz = rz;
        c.rr = rr;
        c.hist[it % HIST] = rr;
        c.pbar = c.deflate ? tot[2] / static_cast<double>(n) : 0.0;
        bool early = false;
        if constexpr (EST) {  // as k_fin_update, for the columns the update summed
            if (est_on && rr >= 0.0) {
                const double rho = sqrt(rr);
                const double C = tot[3], mean = tot[4] / static_cast<double>(n), Idc = tot[5];
                const double P = C - static_cast<double>(n) * mean * mean, D = Idc - C, CI = tot[6];
                const double a = (sqrt(fmax(C, 0.0)) + rho) * rho;
                const double bdc = Idc > a ? a / (Idc - a) : INFINITY;
                early = fmax(fmax(quad_bound(CI, rho), quad_bound(D, 0.5 * rho)),
                             fmax(fmax(quad_bound(P, rho), quad_bound(C, rho)), bdc)) <= c.eps_stop;
            }
        }
        if (!isfinite(rr)) c.done = BREAKDOWN;
        else if (rr <= c.tol2 || early) c.done = CONVERGED;
        else if (it >= c.max_iter) c.done = ITER_CAP;
    }
}

// Batched CG start. mode 0: X = 0, R = S (zero in padding columns) and the
// statistics of each column of S; mode 1: restart from the current X with R
// holding the true residual; mode 2: X = 0, R given; mode 3, after mode 0 or
// 2: X += m 1, R -= m 1 with m the column's mean of R at that start (rmean),
// the start of deflated CG (see k_cg_shift). Only columns in `mask` are touched. Partial slots per
// column: 0 rz, 1 rr, 2 ss, 3 sum s (sum r in modes 1-3), 4 bad count
// (columns < kcheck only), 5 sum p, 6 max of -s, 7 max of s.
template <typename T, int KB>
__global__ void __launch_bounds__(WG) k_init_batched(int n, int k, const double* __restrict__ S, int64_t lds,
                                                     T* __restrict__ X, T* __restrict__ R, T* __restrict__ P,
                                                     const float* __restrict__ minv, int mode, uint64_t mask,
                                                     int kcheck, double* __restrict__ part,
                                                     const Ctrl* __restrict__ ctrl) {
    __shared__ double lred[12 * WG];
    const int c = threadIdx.x % KB;
    const bool on = (mask >> c) & 1ull;
    const double mu = mode == 3 ? ctrl[c].rmean : 0.0;
    double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY, -INFINITY};  // 6: max of -s, 7: max of s
    const int64_t total = static_cast<int64_t>(n) * KB;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * WG;
    if (on) {
        for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < total; e += stride) {
            const int i = static_cast<int>(e / KB);
            double ri;
            if (mode == 0) {
                const double si = c < k ? S[static_cast<int64_t>(i) * lds + c] : 0.0;
                X[e] = T(0);
                R[e] = static_cast<T>(si);
                ri = static_cast<double>(R[e]);
                v[2] += si * si;
                v[3] += si;
                if (c < kcheck && !(si >= 0.0 && si <= 1.0)) v[4] += 1.0;
                v[6] = fmax(v[6], -si);
                v[7] = fmax(v[7], si);
            } else {
                if (mode == 2) X[e] = T(0);
                if (mode == 3) {
                    X[e] = static_cast<T>(static_cast<double>(X[e]) + mu);
                    R[e] = static_cast<T>(static_cast<double>(R[e]) - mu);
                }
                ri = static_cast<double>(R[e]);
                v[3] += ri;
            }
            const T zt = static_cast<T>(static_cast<double>(minv[i]) * ri);
            if (P != nullptr) P[e] = zt;
            v[0] += ri * static_cast<double>(zt);
            v[1] += ri * ri;
            v[5] += static_cast<double>(zt);
        }
    }
    // per-column max of slots 6, 7 over the groups, sums of the others
    constexpr int NG = WG / KB;
    for (int a = 0; a < 8; ++a) lred[a * WG + threadIdx.x] = v[a];
    __syncthreads();
    if (threadIdx.x < KB) {
        for (int a = 0; a < 8; ++a) {
            double t = a < 6 ? 0.0 : -INFINITY;
            for (int gr = 0; gr < NG; ++gr) {
                const double u = lred[a * WG + gr * KB + threadIdx.x];
                t = a < 6 ? t + u : fmax(t, u);
            }
            part[(static_cast<int64_t>(blockIdx.x) * KB + threadIdx.x) * BPART + a] = t;
        }
    }
}

template <int KB>
__global__ void __launch_bounds__(WG) k_fin_init_batched(int G, int n, int k, const double* __restrict__ part,
                                                         int mode, uint64_t mask, ColumnTol tol, int max_iter,
                                                         int range_check, Ctrl* __restrict__ ctrl, int stop_others,
                                                         double eps_stop, int deflate) {
    const int c = blockIdx.x;  // one workgroup per column
    Ctrl& C = ctrl[c];
    if (!((mask >> c) & 1ull)) {
        // an inner solve of the eager path runs only the masked columns; the
        // server keeps the others running
        if (mode == 2 && stop_others && threadIdx.x == 0) C.done = CONVERGED;
        return;
    }
    __shared__ double red[NWAVE * 6];
    double tot[6];
    column_totals<6, KB>(G, part, tot, red);
    // max of slots 6 (-min s) and 7 (max s) over the workgroups
    double mx[2] = {-INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < G; b += WG) {
        const double* p = part + (static_cast<int64_t>(b) * KB + c) * BPART;
        mx[0] = fmax(mx[0], p[6]);
        mx[1] = fmax(mx[1], p[7]);
    }
    mx[0] = wave_max(mx[0]);
    mx[1] = wave_max(mx[1]);
    if ((threadIdx.x & 63) == 0) {
        red[(threadIdx.x >> 6) * 2] = mx[0];
        red[(threadIdx.x >> 6) * 2 + 1] = mx[1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w) {
            mx[0] = fmax(mx[0], red[w * 2]);
            mx[1] = fmax(mx[1], red[w * 2 + 1]);
        }
        const double rz = tot[0], rr = tot[1];
        if (mode == 0) {
            C.smin = -mx[0];
            C.smax = mx[1];
            C.ss = tot[2];
            C.mu = tot[3] / static_cast<double>(n);
            C.bad = tot[4] > 0.0 ? 2 : 0;
            C.iters = 0;
            C.max_iter = max_iter;
        } else if (mode == 2) {
            C.ss = rr;
            C.iters = 0;
            C.max_iter = max_iter;
            C.bad = 0;
        }
        C.tol2 = tol.rtol2[c] * C.ss;
        C.eps_stop = eps_stop;
        C.deflate = deflate;
        C.pbar = deflate ? tot[5] / static_cast<double>(n) : 0.0;
        C.rmean = tot[3] / static_cast<double>(n);
        C.rz = rz;
        C.rr = rr;
        C.hist[C.iters % HIST] = rr;
        if (c >= k) C.done = CONVERGED;  // padding column
        else if (range_check && C.bad) C.done = BAD_INPUT;
        else if (!isfinite(rr)) C.done = BREAKDOWN;
        else if (rr <= C.tol2) C.done = CONVERGED;
        else if (C.iters >= C.max_iter) C.done = ITER_CAP;
        else C.done = RUNNING;
    }
}

template <typename V, int KB>
__global__ void __launch_bounds__(WG) k_epilogue_batched(Csr<V> g, const WinDesc* __restrict__ desc, int K, int k,
                                                         uint64_t mask, const double* __restrict__ Z,
                                                         const double* __restrict__ S, int64_t lds,
                                                         double* __restrict__ R, double* __restrict__ part,
                                                         const Ctrl* __restrict__ ctrl) {
    __shared__ SpmmStage<V, KB, 1> st;
    OpSpmmEpilogue<KB> op{S, lds, k, mask, ctrl, R};
    spmm_windows<double, V, AccLinSq, KB, 1>(g, desc, K, Z, op, st);
    // the window pass ended with a barrier: its LDS takes the partial sums, three at a time
    static_assert(sizeof(st) >= 3 * WG * sizeof(double), "stage too small to reuse for the partials");
    store_column_partials<9, KB, 1, 3>(op.v, reinterpret_cast<double*>(&st), part);
}

template <int KB>
__global__ void __launch_bounds__(WG) k_fin_epilogue_batched(int G, int n_nodes, uint64_t mask,
                                                             const double* __restrict__ part, Ctrl* __restrict__ ctrl) {
    if (!((mask >> blockIdx.x) & 1ull)) return;  // one workgroup per column
    __shared__ double red[NWAVE * 9];
    double v[9];
    column_totals<9, KB>(G, part, v, red);
    if (threadIdx.x == 0) {
        Ctrl& C = ctrl[blockIdx.x];
        const double n = static_cast<double>(n_nodes);
        const double dev = v[4] - n * C.mu;
        double idx[5];
        idx[0] = v[0];
        idx[1] = 0.5 * v[1];
        idx[2] = fmax(v[2] - dev * dev / n, 0.0);
        idx[3] = v[3];
        idx[4] = v[5];
        const double rho = sqrt(v[6]);
        for (int c = 0; c < 5; ++c) C.res[c] = idx[c];
        C.res[5] = rho;
        C.res[6] = sqrt(C.ss);
        C.res[7] = v[8];
        C.res[8] = v[4];
        C.res[9] = v[7];
        const double rhos[4] = {rho, 0.5 * rho, rho, rho};  // see k_fin_epilogue
        for (int c = 0; c < 4; ++c) {
            const double rx = sqrt(idx[c]);
            const double rh = rhos[c];
            C.bound[c] = (rx > rh) ? rh * (2.0 * rx + rh) / ((rx - rh) * (rx - rh)) + 1e-13 : INFINITY;
        }
        const double a = (sqrt(idx[3]) + rho) * rho;
        C.bound[4] = (idx[4] > a) ? a / (idx[4] - a) + 1e-13 : INFINITY;
    }
}

// FJ_MIXED, batched: r32 = f32(r / ||r||) and z += ||r|| d per column (mode
// as in k_mixed_cast). Columns outside `mask` are left alone, except that the
// cast zeroes their r32 when zero_others is set.
template <int KB>
__global__ void __launch_bounds__(WG) k_mixed_cast_batched(int n, const double* __restrict__ R64,
                                                           float* __restrict__ R32, int mode, uint64_t mask,
                                                           const Ctrl* __restrict__ ctrl, int zero_others) {
    const int c = threadIdx.x % KB;
    if (!zero_others && !((mask >> c) & 1ull)) return;  // leave the other columns alone
    const double rho = mode == 0 ? sqrt(ctrl[c].ss) : ctrl[c].res[5];
    const double inv = (((mask >> c) & 1ull) && rho > 0.0) ? 1.0 / rho : 0.0;
    const int64_t total = static_cast<int64_t>(n) * KB;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < total; e += static_cast<int64_t>(gridDim.x) * WG)
        R32[e] = static_cast<float>(R64[e] * inv);
}

template <int KB>
__global__ void __launch_bounds__(WG) k_mixed_refine_batched(int n, double* __restrict__ Z, const float* __restrict__ D,
                                                             int mode, uint64_t mask, const Ctrl* __restrict__ ctrl) {
    const int c = threadIdx.x % KB;
    if (!((mask >> c) & 1ull)) return;
    const double rho = mode == 0 ? sqrt(ctrl[c].ss) : ctrl[c].res[5];
    const int64_t total = static_cast<int64_t>(n) * KB;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < total; e += static_cast<int64_t>(gridDim.x) * WG)
        Z[e] += rho * static_cast<double>(D[e]);
}

// Zero `words` doubles (a kernel rather than a memset, so it can be captured).
__global__ void __launch_bounds__(WG) k_fill_zero(double* __restrict__ p, int64_t words) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < words; e += static_cast<int64_t>(gridDim.x) * WG)
        p[e] = 0.0;
}

// Set the done state of the columns in mask.
__global__ void k_ctrl_set_done(Ctrl* __restrict__ ctrl, int count, uint64_t mask, int value) {
    const int c = threadIdx.x;
    if (c < count && ((mask >> c) & 1ull)) ctrl[c].done = value;
}

// res[5] = ||s|| for the columns in mask: the scale of the first inner solve
// of FJ_MIXED, so that every later cast and correction reads res[5].
__global__ void k_ctrl_rho_from_s(Ctrl* __restrict__ ctrl, int count, uint64_t mask) {
    const int c = threadIdx.x;
    if (c < count && ((mask >> c) & 1ull)) ctrl[c].res[5] = sqrt(ctrl[c].ss);
}

// Clear the control blocks of the columns in mask (the others keep running).
__global__ void k_ctrl_reset_masked(Ctrl* __restrict__ ctrl, int count, uint64_t mask) {
    constexpr int words = static_cast<int>(sizeof(Ctrl) / sizeof(uint32_t));
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words * count; i += gridDim.x * blockDim.x) {
        const int c = i / words;
        if ((mask >> c) & 1ull) reinterpret_cast<uint32_t*>(ctrl)[i] = 0u;
    }
}

// Scatter the k columns of a request into the slots slot[0..k) of a block.
struct SlotMap {
    int slot[KMAX];
};
__global__ void __launch_bounds__(WG) k_scatter_columns(int n, int k, const double* __restrict__ src, int64_t lds,
                                                        SlotMap map, double* __restrict__ dst, int kb) {
    const int64_t total = static_cast<int64_t>(n) * k;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < total; e += static_cast<int64_t>(gridDim.x) * WG) {
        const int64_t i = e / k;
        const int c = static_cast<int>(e % k);
        dst[i * kb + map.slot[c]] = src[i * lds + c];
    }
}

// Gather columns of a node-major block into another (different leading
// dimensions; padding columns of the destination are zeroed).
__global__ void __launch_bounds__(WG) k_copy_block(int n, int k, int kd, const double* __restrict__ src,
                                                   int64_t lds, double* __restrict__ dst, int64_t ldd) {
    const int64_t total = static_cast<int64_t>(n) * kd;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < total; e += static_cast<int64_t>(gridDim.x) * WG) {
        const int64_t i = e / kd;
        const int c = static_cast<int>(e % kd);
        dst[i * ldd + c] = c < k ? src[i * lds + c] : 0.0;
    }
}

// Algorithm 1 literally (FJ_TWO_SOLVE): column 1 of the block is the centred
// opinion vector s - mean(s) (Algorithm 1's second right-hand side), column 0 s.
__global__ void __launch_bounds__(WG) k_two_solve_rhs(int n, const double* __restrict__ s, int64_t lds,
                                                      const Ctrl* __restrict__ stats, double* __restrict__ dst) {
    const double mu = stats->mu;
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const double si = s[static_cast<int64_t>(i) * lds];
        dst[static_cast<int64_t>(i) * 2] = si;
        dst[static_cast<int64_t>(i) * 2 + 1] = si - mu;
    }
}

}  // namespace fj
