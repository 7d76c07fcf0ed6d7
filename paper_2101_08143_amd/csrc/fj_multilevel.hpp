// fj_multilevel.hpp -- the aggregation V-cycle of FJ_MULTILEVEL (HIP, gfx950).
//
// The method needs a Laplacian solver (Lemma ST; the experiments use one
// built by approximate Gaussian elimination). The single-level preconditioners
// (Jacobi, 2x2 blocks) lose their grip when edge weights spread over many
// orders of magnitude: nodes joined by heavy edges move together, and the
// error that lives on such clusters is smooth along the heavy edges, where a
// local smoother barely touches it. This file applies one V-cycle of an
// aggregation hierarchy (built on the host, see fj_hierarchy_create) of
//   A_l = diag(a_l) - W_l,   A_{l+1} = P_l^T A_l P_l,
// P_l the 0/1 indicator of level l's aggregates (the nodes of level l + 1).
//
// One V-cycle on level l, right-hand side b (all FP64):
//   y = D^-1 b                        k_ml_scale on level 0, else with b by OpSum
//   u = w y                           pre-smoothing from 0 (Jacobi, weight w)
//   t = b - A u                       k_ml_rows<OpPre>: (1-w) b + w W y
//   b' = P^T t                        k_ml_rows<OpSum> over the member lists
//   x' = V-cycle on level l + 1 (the last level: exact dense solve or Jacobi)
//   u = w y + P x'                    k_ml_prolong
//   x = u + w D^-1 (b - A u)          k_ml_rows<OpPost>
// Each row of the sparse passes is summed by a group of 8 lanes (entries
// strided over the lanes, then a fixed shuffle tree); rows with more than 64
// entries are listed per level and take a whole wave. Sums therefore follow
// a fixed order and the V-cycle is deterministic.
#pragma once

#include "fj_kernels.hpp"

namespace fj {

constexpr int ML_GW = 8;       // lanes per row
constexpr int ML_LONG = 64;    // rows longer than this take a wave
constexpr int ML_MAXL = 16;    // levels
constexpr double ML_OMEGA = 0.9;

// Level l of the hierarchy as the kernels see it (device pointers).
struct MlLevel {
    int n = 0, nc = 0;            // nodes of this level and of the next
    int nlong = 0, nclong = 0;    // rows with > ML_LONG entries; aggregates with > ML_LONG members
    const int* rp = nullptr;      // W_l: CSR without the diagonal
    const int* col = nullptr;
    const double* w = nullptr;
    const int* longs = nullptr;   // the long rows
    const double* a = nullptr;    // diagonal a_l
    const double* ainv = nullptr; // 1 / a_l
    const int* agg = nullptr;     // aggregate of each node (a node of level l + 1)
    const int* mrp = nullptr;     // members of each aggregate (CSR over level l + 1)
    const int* mem = nullptr;
    const int* clongs = nullptr;  // the long aggregates
    double* t = nullptr;          // work: n (D^-1 b of every level lives in fj_hierarchy::ybuf)
};

// Row sums of a CSR (weights optional) against op.src, epilogue op.row.
template <typename Op>
__global__ void __launch_bounds__(WG) k_ml_rows(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                const double* __restrict__ w, const int* __restrict__ longs,
                                                int nlong, Op op, const Ctrl* __restrict__ ctrl) {
    if (ctrl && ctrl->done != RUNNING) return;
    const int gid = blockIdx.x * WG + threadIdx.x;
    const int lane = threadIdx.x % ML_GW;
    const int ngrp = gridDim.x * (WG / ML_GW);
    for (int i = gid / ML_GW; i < n; i += ngrp) {  // uniform over the group
        const int e0 = rp[i], e1 = rp[i + 1];
        if (e1 - e0 > ML_LONG) continue;
        double acc = 0.0;
        for (int e = e0 + lane; e < e1; e += ML_GW) acc += (w ? w[e] : 1.0) * op.src(col[e]);
        acc += __shfl_xor(acc, 4, ML_GW);
        acc += __shfl_xor(acc, 2, ML_GW);
        acc += __shfl_xor(acc, 1, ML_GW);
        if (lane == 0) op.row(i, acc);
    }
    const int wl = threadIdx.x & 63;
    const int nwave = gridDim.x * (WG / 64);
    for (int k = gid / 64; k < nlong; k += nwave) {  // uniform over the wave
        const int i = longs[k];
        const int e0 = rp[i], e1 = rp[i + 1];
        double acc = 0.0;
        for (int e = e0 + wl; e < e1; e += 64) acc += (w ? w[e] : 1.0) * op.src(col[e]);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        if (wl == 0) op.row(i, acc);
    }
}

// t = b - A (w D^-1 b) = (1 - w) b + w W y, y = D^-1 b
struct OpPre {
    const double* __restrict__ b;
    const double* __restrict__ y;
    double* __restrict__ t;
    __device__ double src(int j) const { return y[j]; }
    __device__ void row(int i, double acc) const { t[i] = (1.0 - ML_OMEGA) * b[i] + ML_OMEGA * acc; }
};

// restriction: b'[A] = sum over the members i of A of t[i], and y' = b' / a'
struct OpSum {
    const double* __restrict__ t;
    const double* __restrict__ ainv_next;
    double* __restrict__ out;
    double* __restrict__ y_next;
    __device__ double src(int j) const { return t[j]; }
    __device__ void row(int i, double acc) const {
        out[i] = acc;
        y_next[i] = acc * ainv_next[i];
    }
};

// y = D^-1 b on level 0 (the finer levels get it from OpSum)
__global__ void __launch_bounds__(WG) k_ml_scale(int n, const double* __restrict__ b,
                                                 const double* __restrict__ ainv, double* __restrict__ y,
                                                 const Ctrl* __restrict__ ctrl) {
    if (ctrl && ctrl->done != RUNNING) return;
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) y[i] = b[i] * ainv[i];
}

// x = u + w D^-1 (b - a u + W u)
struct OpPost {
    const double* __restrict__ b;
    const double* __restrict__ u;
    const double* __restrict__ a;
    const double* __restrict__ ainv;
    double* __restrict__ x;
    __device__ double src(int j) const { return u[j]; }
    __device__ void row(int i, double acc) const {
        const double ui = u[i];
        x[i] = ui + ML_OMEGA * ainv[i] * (b[i] - a[i] * ui + acc);
    }
};

// u = w D^-1 b + P x' = w y + P x'
__global__ void __launch_bounds__(WG) k_ml_prolong(int n, const double* __restrict__ y, const int* __restrict__ agg,
                                                   const double* __restrict__ xc, double* __restrict__ u,
                                                   const Ctrl* __restrict__ ctrl) {
    if (ctrl && ctrl->done != RUNNING) return;
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) u[i] = ML_OMEGA * y[i] + xc[agg[i]];
}

// The last level. dense: x = A^-1 b with the stored inverse (one wave per row,
// fixed reduction order); otherwise one Jacobi step x = D^-1 b.
__global__ void __launch_bounds__(WG) k_ml_coarse(int n, const double* __restrict__ inv,
                                                  const double* __restrict__ ainv, const double* __restrict__ b,
                                                  double* __restrict__ x, const Ctrl* __restrict__ ctrl) {
    if (ctrl && ctrl->done != RUNNING) return;
    if (!inv) {
        for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) x[i] = ainv[i] * b[i];
        return;
    }
    const int wl = threadIdx.x & 63;
    const int nwave = gridDim.x * (WG / 64);
    for (int i = (blockIdx.x * WG + threadIdx.x) / 64; i < n; i += nwave) {
        const double* __restrict__ row = inv + static_cast<int64_t>(i) * n;
        double acc = 0.0;
        for (int k = wl; k < n; k += 64) acc += row[k] * b[k];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        if (wl == 0) x[i] = acc;
    }
}

// CG start with the V-cycle (after k_cg_init / k_cg_shift and z = V r):
// p = z, and the partial sums k_fin_init mode 1 reads (0 rz, 1 rr, 5 sum p).
__global__ void __launch_bounds__(WG) k_ml_start(int n, const double* __restrict__ r, const double* __restrict__ z,
                                                 double* __restrict__ p, double* __restrict__ part) {
    __shared__ double red[NWAVE * 3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const double zi = z[i], ri = r[i];
        p[i] = zi;
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

// After mq = V q: the partial sums of z^T q and q^T V q (slots 1 and 2, as
// k_pair_dots writes them for k_fin_pair).
__global__ void __launch_bounds__(WG) k_ml_dots(int n, const double* __restrict__ q, const double* __restrict__ z,
                                                const double* __restrict__ mq, double* __restrict__ part,
                                                const Ctrl* __restrict__ ctrl) {
    if (ctrl->done != RUNNING) return;
    __shared__ double red[NWAVE * 2];
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        const double qi = q[i];
        v[0] += z[i] * qi;
        v[1] += qi * mq[i];
    }
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x * NPART + 1] = v[0];
        part[blockIdx.x * NPART + 2] = v[1];
    }
}

}  // namespace fj
