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
constexpr int WIN = 1024;             // window width in (rows + entries)
constexpr int LONGROW = 512;          // a longer last row takes the workgroup-wide path
constexpr int STAGE = WIN + LONGROW;  // LDS staging capacity in entries
constexpr int STAGE_PER_THREAD = STAGE / WG;
constexpr int ROWS_PER_THREAD = WIN / WG;
constexpr int NPART = 16;             // sums per workgroup in the partials buffer
constexpr int GMAX = 4096;            // largest persistent grid
constexpr int HIST = 64;              // residual history slots

static_assert(STAGE % WG == 0 && WIN % WG == 0, "window sizes must be multiples of the workgroup");

// Control block in the workspace. Written only by the last workgroup of a
// kernel; read by later kernels (kernel boundaries order the accesses) and
// copied to the host between CG chunks.
struct Ctrl {
    double alpha, beta;   // CG step length and direction update of this iteration
    double rz, rr;        // r^T M^{-1} r and r^T r after the last update
    double tol2;          // stop when rr <= tol2
    double mu, ss;        // mean(s) and ||s||^2
    double smin, smax;    // range of s
    double res[16];       // epilogue: indices, residual and diagnostics (see k_epilogue)
    double bound[5];      // certified relative error bound of each index
    double hist[HIST];    // rr after iteration t is in hist[t % HIST]
    int32_t done;         // 0 running, 1 converged, 2 iteration cap, 3 breakdown, 4 bad input
    int32_t iters;        // CG iterations so far (all passes)
    int32_t max_iter;
    int32_t bad;          // bit 0: NaN in s, bit 1: s outside [0,1]
    uint32_t ticket;      // arrival counter of the last-workgroup reduction
    int32_t pad[3];
};

enum Done : int32_t { RUNNING = 0, CONVERGED = 1, ITER_CAP = 2, BREAKDOWN = 3, BAD_INPUT = 4 };

struct Unit {};  // weight type tag: every edge has weight 1

template <typename V>
struct Csr {
    using value_type = V;
    int n;
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

__device__ __forceinline__ double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Each workgroup publishes its N sums; the last workgroup to arrive adds all
// of them in workgroup order and returns true with the grand totals in v.
// Every thread of every workgroup must call it (it synchronises).
template <int N>
__device__ bool last_block_total(double (&v)[N], double* __restrict__ part, Ctrl* ctrl,
                                 double* red, int* flag) {
    static_assert(N <= NPART, "too many partial sums");
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < N; ++c) part[blockIdx.x * NPART + c] = v[c];
        __threadfence();
        const uint32_t t = atomicAdd(&ctrl->ticket, 1u);
        *flag = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!*flag) return false;
    __threadfence();
    double acc[N];
#pragma unroll
    for (int c = 0; c < N; ++c) acc[c] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += WG) {
#pragma unroll
        for (int c = 0; c < N; ++c) acc[c] += load_coherent(&part[b * NPART + c]);
    }
    block_sum<N>(acc, red);
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = acc[c];
    if (threadIdx.x == 0) ctrl->ticket = 0u;
    return true;
}

// ------------------------------------------------------------ window pass

// What a row accumulates over its neighbours j (d = x_i - x_j):
struct AccLin   { static constexpr bool X = true,  SQ = false, DEG = false; };  // sum w d
struct AccLinSq { static constexpr bool X = true,  SQ = true,  DEG = false; };  // sum w d, sum w d^2
struct AccDeg   { static constexpr bool X = false, SQ = false, DEG = true;  };  // sum w

template <typename T, typename V>
struct Stage {
    T x[STAGE];
    V w[STAGE];
};
template <typename T>
struct Stage<T, Unit> {
    T x[STAGE];
};

template <typename T, typename V, typename Acc, typename Op>
__device__ __forceinline__ void window_pass(const Csr<V>& g, const int* __restrict__ blk_row, int k,
                                            const T* __restrict__ x, Op& op, Stage<T, V>& st,
                                            double* red) {
    const int tid = threadIdx.x;
    const int r0 = blk_row[k];
    const int r1 = blk_row[k + 1];
    if (r0 >= r1) return;  // workgroup-uniform: an empty window
    const int e0 = g.row_ptr[r0];
    const int elast = g.row_ptr[r1 - 1];
    const int eend = g.row_ptr[r1];
    const bool long_last = (eend - elast) > LONGROW;
    const int rs_end = long_last ? r1 - 1 : r1;
    const int ns = (long_last ? elast : eend) - e0;  // < STAGE by construction of the windows

    // Phase 1: coalesced loads of col (and val), gathers of x_j, into LDS.
    if constexpr (Acc::X || !std::is_same<V, Unit>::value) {
        int jj[STAGE_PER_THREAD];
#pragma unroll
        for (int u = 0; u < STAGE_PER_THREAD; ++u) {
            const int e = tid + u * WG;
            jj[u] = (e < ns) ? g.col[e0 + e] : 0;
        }
        if constexpr (Acc::X) {
            T xv[STAGE_PER_THREAD];
#pragma unroll
            for (int u = 0; u < STAGE_PER_THREAD; ++u) {
                const int e = tid + u * WG;
                if (e < ns) xv[u] = x[jj[u]];
            }
#pragma unroll
            for (int u = 0; u < STAGE_PER_THREAD; ++u) {
                const int e = tid + u * WG;
                if (e < ns) st.x[e] = xv[u];
            }
        }
        if constexpr (!std::is_same<V, Unit>::value) {
#pragma unroll
            for (int u = 0; u < STAGE_PER_THREAD; ++u) {
                const int e = tid + u * WG;
                if (e < ns) st.w[e] = g.val[e0 + e];
            }
        }
        __syncthreads();
    }

    // Phase 2: one thread per row, reduced from LDS.
#pragma unroll
    for (int u = 0; u < ROWS_PER_THREAD; ++u) {
        const int i = r0 + tid + u * WG;
        if (i < rs_end) {
            const int a = g.row_ptr[i] - e0;
            const int b = min(g.row_ptr[i + 1] - e0, STAGE);  // the min only guards malformed input
            const T xi = Acc::X ? x[i] : T(0);
            double lin = 0.0, sq = 0.0;
            if constexpr (Acc::DEG && std::is_same<V, Unit>::value) {
                lin = static_cast<double>(b - a);
            } else {
                for (int e = a; e < b; ++e) {
                    double w = 1.0;
                    if constexpr (!std::is_same<V, Unit>::value) w = static_cast<double>(st.w[e]);
                    if constexpr (Acc::DEG) {
                        lin += w;
                    } else {
                        const double d = static_cast<double>(xi) - static_cast<double>(st.x[e]);
                        lin += w * d;
                        if constexpr (Acc::SQ) sq += w * d * d;
                    }
                }
            }
            op.row(i, xi, lin, sq);
        }
    }

    // Phase 3: a long last row, reduced by the whole workgroup from HBM.
    if (long_last) {
        const int i = r1 - 1;
        const T xi = Acc::X ? x[i] : T(0);
        double v[2] = {0.0, 0.0};
        for (int e = elast + tid; e < eend; e += WG) {
            const double w = weight_at<V>(g.val, e);
            if constexpr (Acc::DEG) {
                v[0] += w;
            } else {
                const double d = static_cast<double>(xi) - static_cast<double>(x[g.col[e]]);
                v[0] += w * d;
                if constexpr (Acc::SQ) v[1] += w * d * d;
            }
        }
        block_sum<2>(v, red);
        if (tid == 0) op.row(i, xi, v[0], v[1]);
    }
    __syncthreads();  // LDS is reused by the next window
}

// ------------------------------------------------------------ row operations

struct OpDiag {  // Jacobi preconditioner M^{-1} = diag(1 + d_i)^{-1}
    float* __restrict__ minv;
    template <typename T>
    __device__ void row(int i, T, double deg, double) { minv[i] = static_cast<float>(1.0 / (1.0 + deg)); }
};

struct OpApply {  // y = (I + L) x
    double* __restrict__ y;
    __device__ void row(int i, double xi, double lin, double) { y[i] = xi + lin; }
};

struct OpCgSpmv {  // q = (I + L) p and the three dot products the CG scalars need
    const double* __restrict__ r;
    const float* __restrict__ minv;
    double* __restrict__ q;
    double pq = 0.0, rmq = 0.0, qmq = 0.0;
    __device__ void row(int i, double pi, double lin, double) {
        const double qi = pi + lin;
        q[i] = qi;
        const double mq = static_cast<double>(minv[i]) * qi;
        pq += pi * qi;
        rmq += r[i] * mq;
        qmq += qi * mq;
    }
};

struct OpEpilogue {  // one pass over z: every index, the true residual and diagnostics
    const double* __restrict__ s;
    int64_t lds;
    double mu;
    double* __restrict__ rbuf;
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    __device__ void row(int i, double zi, double t, double dsq) {
        const double si = s[static_cast<int64_t>(i) * lds];
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

template <typename V>
__global__ void __launch_bounds__(WG) k_diag(Csr<V> g, const int* __restrict__ blk_row, int K,
                                             float* __restrict__ minv) {
    __shared__ Stage<double, V> st;
    __shared__ double red[NWAVE * 2];
    OpDiag op{minv};
    for (int k = blockIdx.x; k < K; k += gridDim.x)
        window_pass<double, V, AccDeg>(g, blk_row, k, static_cast<const double*>(nullptr), op, st, red);
}

template <typename V>
__global__ void __launch_bounds__(WG) k_apply(Csr<V> g, const int* __restrict__ blk_row, int K,
                                              const double* __restrict__ x, double* __restrict__ y) {
    __shared__ Stage<double, V> st;
    __shared__ double red[NWAVE * 2];
    OpApply op{y};
    for (int k = blockIdx.x; k < K; k += gridDim.x)
        window_pass<double, V, AccLin>(g, blk_row, k, x, op, st, red);
}

// CG step, part 1: q = (I+L) p with p^T q, r^T M^{-1} q and q^T M^{-1} q.
// The last workgroup forms alpha = rz / p^T q and, from the recurrence
// r' = r - alpha q, rz' = rz - 2 alpha r^T M^{-1} q + alpha^2 q^T M^{-1} q and
// beta = rz' / rz, so that the update kernel can also move the direction.
template <typename V>
__global__ void __launch_bounds__(WG) k_cg_spmv(Csr<V> g, const int* __restrict__ blk_row, int K,
                                                const double* __restrict__ p,
                                                const double* __restrict__ r,
                                                const float* __restrict__ minv,
                                                double* __restrict__ q, double* __restrict__ part,
                                                Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ Stage<double, V> st;
    __shared__ double red[NWAVE * 4];
    __shared__ int flag;
    OpCgSpmv op{r, minv, q};
    for (int k = blockIdx.x; k < K; k += gridDim.x)
        window_pass<double, V, AccLin>(g, blk_row, k, p, op, st, red);
    double v[3] = {op.pq, op.rmq, op.qmq};
    block_sum<3>(v, red);
    if (last_block_total<3>(v, part, ctrl, red, &flag) && threadIdx.x == 0) {
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

// CG step, part 2: x += alpha p, r -= alpha q, z = M^{-1} r, p = z + beta p, and
// the exact r^T M^{-1} r (next alpha) and r^T r (stopping test).
__global__ void __launch_bounds__(WG) k_cg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ p, const double* __restrict__ q,
                                                  const float* __restrict__ minv,
                                                  double* __restrict__ part, Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double red[NWAVE * 2];
    __shared__ int flag;
    const double alpha = ctrl->alpha, beta = ctrl->beta;
    double v[2] = {0.0, 0.0};
    const int npair = n >> 1;
    for (int t = blockIdx.x * WG + threadIdx.x; t < npair; t += gridDim.x * WG) {
        double2 xv = reinterpret_cast<double2*>(x)[t];
        double2 rv = reinterpret_cast<double2*>(r)[t];
        double2 pv = reinterpret_cast<double2*>(p)[t];
        const double2 qv = reinterpret_cast<const double2*>(q)[t];
        const float2 mv = reinterpret_cast<const float2*>(minv)[t];
        xv.x += alpha * pv.x;
        xv.y += alpha * pv.y;
        rv.x -= alpha * qv.x;
        rv.y -= alpha * qv.y;
        const double zx = static_cast<double>(mv.x) * rv.x;
        const double zy = static_cast<double>(mv.y) * rv.y;
        pv.x = zx + beta * pv.x;
        pv.y = zy + beta * pv.y;
        v[0] += rv.x * zx + rv.y * zy;
        v[1] += rv.x * rv.x + rv.y * rv.y;
        reinterpret_cast<double2*>(x)[t] = xv;
        reinterpret_cast<double2*>(r)[t] = rv;
        reinterpret_cast<double2*>(p)[t] = pv;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int i = n - 1;
        x[i] += alpha * p[i];
        r[i] -= alpha * q[i];
        const double zi = static_cast<double>(minv[i]) * r[i];
        p[i] = zi + beta * p[i];
        v[0] += r[i] * zi;
        v[1] += r[i] * r[i];
    }
    block_sum<2>(v, red);
    if (last_block_total<2>(v, part, ctrl, red, &flag) && threadIdx.x == 0) {
        const int it = ctrl->iters + 1;
        ctrl->iters = it;
        ctrl->rz = v[0];
        ctrl->rr = v[1];
        ctrl->hist[it % HIST] = v[1];
        if (!isfinite(v[1])) ctrl->done = BREAKDOWN;
        else if (v[1] <= ctrl->tol2) ctrl->done = CONVERGED;
        else if (it >= ctrl->max_iter) ctrl->done = ITER_CAP;
    }
}

// CG start. mode 0: x = 0, r = s, plus the statistics of s (mean, ||s||^2,
// range). mode 1: restart from the current x with r already holding the true
// residual (written by the epilogue). Both: p = M^{-1} r, rz, rr, and the
// stopping threshold tol2 = rtol2 * ||s||^2.
__global__ void __launch_bounds__(WG) k_cg_init(int n, const double* __restrict__ s, int64_t lds,
                                                double* __restrict__ x, double* __restrict__ r,
                                                double* __restrict__ p, const float* __restrict__ minv,
                                                int mode, double rtol2, int max_iter, int range_check,
                                                double* __restrict__ part, Ctrl* __restrict__ ctrl) {
    __shared__ double red[NWAVE * 8];
    __shared__ int flag;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // rz, rr, ss, sum s, bad count
    double smin = INFINITY, smax = -INFINITY;
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        double ri;
        if (mode == 0) {
            const double si = s[static_cast<int64_t>(i) * lds];
            x[i] = 0.0;
            ri = si;
            r[i] = si;
            v[2] += si * si;
            v[3] += si;
            if (!(si >= 0.0 && si <= 1.0)) v[4] += 1.0;
            smin = fmin(smin, si);
            smax = fmax(smax, si);
        } else {
            ri = r[i];
        }
        const double zi = static_cast<double>(minv[i]) * ri;
        p[i] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
    }
    block_sum<5>(v, red);
    // workgroup min / max, published beside the sums
    smin = wave_min(smin);
    smax = wave_max(smax);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[NWAVE * 5 + wave] = smin;
        red[NWAVE * 6 + wave] = smax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = red[NWAVE * 5], b = red[NWAVE * 6];
        for (int w = 1; w < NWAVE; ++w) {
            a = fmin(a, red[NWAVE * 5 + w]);
            b = fmax(b, red[NWAVE * 6 + w]);
        }
        part[blockIdx.x * NPART + 5] = a;
        part[blockIdx.x * NPART + 6] = b;
    }
    __syncthreads();
    if (last_block_total<5>(v, part, ctrl, red, &flag) && threadIdx.x == 0) {
        if (mode == 0) {
            double a = INFINITY, b = -INFINITY;
            for (int k = 0; k < (int)gridDim.x; ++k) {
                a = fmin(a, load_coherent(&part[k * NPART + 5]));
                b = fmax(b, load_coherent(&part[k * NPART + 6]));
            }
            ctrl->smin = a;
            ctrl->smax = b;
            ctrl->ss = v[2];
            ctrl->mu = v[3] / static_cast<double>(n);
            ctrl->bad = v[4] > 0.0 ? 2 : 0;
            ctrl->iters = 0;
            ctrl->max_iter = max_iter;
        }
        ctrl->tol2 = rtol2 * ctrl->ss;
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
// and the control block's results:
//   res[0] C_I  = ||L z||^2           res[5] ||r||_2
//   res[1] D    = half the row sums    res[6] ||s||_2
//   res[2] P    = sum (z - mean z)^2   res[7] sum (z_i - s_i)^2
//   res[3] C    = ||z||^2              res[8] sum z
//   res[4] I_dc = s^T z                res[9] z^T r
// and bound[] (relative error bounds, see below).
template <typename V>
__global__ void __launch_bounds__(WG) k_epilogue(Csr<V> g, const int* __restrict__ blk_row, int K,
                                                 const double* __restrict__ z, const double* __restrict__ s,
                                                 int64_t lds, double* __restrict__ rbuf,
                                                 double* __restrict__ part, Ctrl* __restrict__ ctrl) {
    __shared__ Stage<double, V> st;
    __shared__ double red[NWAVE * 10];
    __shared__ int flag;
    OpEpilogue op{s, lds, ctrl->mu, rbuf};
    for (int k = blockIdx.x; k < K; k += gridDim.x)
        window_pass<double, V, AccLinSq>(g, blk_row, k, z, op, st, red);
    double v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = op.v[c];
    block_sum<9>(v, red);
    if (last_block_total<9>(v, part, ctrl, red, &flag) && threadIdx.x == 0) {
        const double n = static_cast<double>(g.n);
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
