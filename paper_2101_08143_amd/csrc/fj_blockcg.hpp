// fj_blockcg.hpp -- O'Leary's block conjugate gradients for KB columns
// (HIP, gfx950): one Krylov space shared by all the columns of a block.
//
// The per-column batched CG of fj_batched.hpp runs k independent solves on
// one SpMM pass. Block CG instead searches, at every step, along a KB-wide
// block of directions P shared by all columns: X += P alpha with alpha a
// KB x KB matrix, so each column's update combines every direction of the
// block (O'Leary 1980), with A = I + L and M the Jacobi preconditioner:
//
//   Q = A P,  W = (P^T Q)^+,  alpha = W (P^T R),  X += P alpha,  R -= Q alpha
//   Z = Pi M^-1 R                  (Jacobi, then centred: deflation by 1)
//   beta = -W (Q^T Z),  P <- (Z + P beta) D
//
// W comes from a Cholesky factorisation L L^T = P^T Q, W = L^-T L^-1; a
// pivot that vanishes (the block lost rank, e.g. a column that has
// converged, or two equal columns) drops that direction for the step, which
// makes W the inverse on the remaining directions. D scales column c by
// 1 / ||r_c||: it leaves the search space unchanged and keeps columns whose
// residuals differ in scale from looking dependent. The n x KB by KB x KB
// products and the KB x KB Gram matrices are dense contractions over n and
// run on the matrix cores (v_mfma_f64_16x16x4f64): KB is 16, 32 or 64.
//
// Unlike the per-column path, a column's arithmetic depends on the other
// columns of the block (they share the search space).
#pragma once

#include "fj_batched.hpp"

namespace fj {

typedef double dv4 __attribute__((ext_vector_type(4)));

constexpr int GRAM_G = 1024;  // workgroups of a Gram pass (each writes a KB x KB partial)

// v_mfma_f64_16x16x4f64, D = A B + C with A 16 x 4, B 4 x 16: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 r + l / 16][l % 16]
// in element r of the result (measured on gfx950).
__device__ __forceinline__ dv4 mfma16(double a, double b, dv4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Partial Gram matrices A^T B_g (g < NG, the B_g sharing A) of node-major
// n x KB blocks. A workgroup walks its contiguous node range in chunks of
// GCH nodes: the chunk's rows are staged in LDS with coalesced loads, then
// wave w multiplies the 16 x 16 tiles t with t % NWAVE == w from LDS.
// Workgroup b writes its NG partials to part[(b * NG + g) * KB * KB ...]
// (row-major). The next chunk's loads are issued before the current chunk's
// products.
constexpr int GCH = 16;
template <int KB, int NG>
__global__ void __launch_bounds__(WG) k_gram(int n, const double* __restrict__ A, const double* __restrict__ B0,
                                             const double* __restrict__ B1, double* __restrict__ part,
                                             const Ctrl* __restrict__ ctrl) {
    if (ctrl[0].done != RUNNING) return;
    static_assert(KB % 16 == 0 && KB <= KMAX && (NG == 1 || NG == 2), "tiles of 16 columns, one or two Grams");
    constexpr int TT = KB / 16, NT = TT * TT, PER = (NT + NWAVE - 1) / NWAVE;
    constexpr int LD = KB + 1;              // padded LDS rows
    constexpr int PT = GCH * KB / WG;       // elements each thread stages per block and chunk
    __shared__ double As[GCH * LD];
    __shared__ double Bs[NG][GCH * LD];
    const double* __restrict__ Bp[2] = {B0, B1};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane & 15, kk = lane >> 4;
    const int64_t chunk = ((static_cast<int64_t>(n) + gridDim.x - 1) / gridDim.x + GCH - 1) / GCH * GCH;
    const int64_t i_begin = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t i_end = std::min<int64_t>(n, i_begin + chunk);
    dv4 acc[NG][PER];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int p = 0; p < PER; ++p) acc[g][p] = dv4{0.0, 0.0, 0.0, 0.0};
    double va[PT], vb[NG][PT];
    // the chunk at c0 into registers (element e of a chunk: node e / KB, column e % KB)
    auto fetch = [&](int64_t c0) {
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int e = threadIdx.x + u * WG;
            const bool ok = c0 + e / KB < i_end;
            va[u] = ok ? A[c0 * KB + e] : 0.0;
#pragma unroll
            for (int g = 0; g < NG; ++g) vb[g][u] = ok ? Bp[g][c0 * KB + e] : 0.0;
        }
    };
    if (i_begin < i_end) fetch(i_begin);
    for (int64_t c0 = i_begin; c0 < i_end; c0 += GCH) {
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int e = threadIdx.x + u * WG;
            As[(e / KB) * LD + e % KB] = va[u];
#pragma unroll
            for (int g = 0; g < NG; ++g) Bs[g][(e / KB) * LD + e % KB] = vb[g][u];
        }
        __syncthreads();
        if (c0 + GCH < i_end) fetch(c0 + GCH);  // the next chunk's loads fly during these products
#pragma unroll
        for (int s = 0; s < GCH / 4; ++s) {
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int t = wave + p * NWAVE;
                if (t < NT) {
                    const int tr = t / TT, tc = t % TT;
                    const double a = As[(4 * s + kk) * LD + 16 * tr + sub];
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        acc[g][p] = mfma16(a, Bs[g][(4 * s + kk) * LD + 16 * tc + sub], acc[g][p]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        double* out = part + (static_cast<int64_t>(blockIdx.x) * NG + g) * KB * KB;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int t = wave + p * NWAVE;
            if (t < NT) {
                const int tr = t / TT, tc = t % TT;
#pragma unroll
                for (int r = 0; r < 4; ++r) out[(16 * tr + 4 * r + kk) * KB + 16 * tc + sub] = acc[g][p][r];
            }
        }
    }
}

// out[e] = scale * (sum over the G partials of entry e), e < entries (the NG
// Grams of one pass, contiguous): 16 threads per entry each add every 16th
// partial, then the 16 sums are added in order (a fixed tree).
__global__ void __launch_bounds__(WG) k_gram_fin(int G, int entries, const double* __restrict__ part, double scale,
                                                 double* __restrict__ out, const Ctrl* __restrict__ ctrl) {
    if (ctrl[0].done != RUNNING) return;
    __shared__ double s16[16][17];
    const int q = threadIdx.x & 15, sl = threadIdx.x >> 4;
    const int e = blockIdx.x * 16 + q;
    double t = 0.0;
    if (e < entries)
        for (int b = sl; b < G; b += 16) t += part[static_cast<int64_t>(b) * entries + e];
    s16[sl][q] = t;
    __syncthreads();
    if (threadIdx.x < 16 && e < entries) {
        double v = 0.0;
        for (int j = 0; j < 16; ++j) v += s16[j][q];
        out[e] = scale * v;
    }
}

// From G = [P^T Q, P^T R] (two KB x KB matrices, one workgroup): the
// Cholesky factor L L^T = (P^T Q + Q^T P) / 2, C = L^-T, W = C C^T (written to
// Wm) and alpha = W P^T R (written to Am). A pivot below 1e-13 of the
// largest diagonal entry (or not finite) drops that direction: its row and
// column of C are zero, so W inverts P^T Q on the other directions only.
template <int KB>
__global__ void __launch_bounds__(WG) k_bcg_chol(const double* __restrict__ G2, double* __restrict__ Wm,
                                                 double* __restrict__ Am, const Ctrl* __restrict__ ctrl) {
    if (ctrl[0].done != RUNNING) return;
    __shared__ double L[KB][KB + 1];   // lower triangle: L; upper triangle: C (i < c); dc: C's diagonal
    __shared__ double Wl[KB][KB + 1];  // W
    __shared__ double dc[KB];
    __shared__ int drop[KB];
    __shared__ double dmax;
    const int tid = threadIdx.x;
    for (int e = tid; e < KB * KB; e += WG) {
        const int i = e / KB, j = e % KB;
        L[i][j] = 0.5 * (G2[i * KB + j] + G2[j * KB + i]);
    }
    __syncthreads();
    if (tid == 0) {
        double m = 0.0;
        for (int i = 0; i < KB; ++i) m = fmax(m, L[i][i]);
        dmax = m;
    }
    __syncthreads();
    // right-looking: pivot j, scale column j, update the trailing lower triangle
    for (int j = 0; j < KB; ++j) {
        if (tid == 0) {
            const double d = L[j][j];
            const bool bad = !(d > 1e-13 * dmax) || !isfinite(d);
            drop[j] = bad ? 1 : 0;
            L[j][j] = bad ? 0.0 : sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < KB; i += WG) L[i][j] = drop[j] ? 0.0 : L[i][j] / L[j][j];
        __syncthreads();
        const int m = KB - 1 - j;  // trailing (i, k), j < k <= i < KB
        for (int e = tid; e < m * m; e += WG) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k <= i) L[i][k] -= L[i][j] * L[k][j];
        }
        __syncthreads();
    }
    // C = L^-T, upper triangular: thread c solves L^T C[:, c] = e_c from the bottom
    if (tid < KB) {
        const int c = tid;
        for (int i = c; i >= 0; --i) {
            double v = 0.0;
            if (!drop[i] && !drop[c]) {
                v = i == c ? 1.0 : 0.0;
                for (int k = i + 1; k <= c; ++k) v -= L[k][i] * (k == c ? dc[c] : L[k][c]);
                v /= L[i][i];
            }
            if (i == c) dc[c] = v;
            else L[i][c] = v;
        }
    }
    __syncthreads();
    // W = C C^T: W[i][j] = sum_{k >= max(i, j)} C[i][k] C[j][k] (gfx950 gives a
    // workgroup up to 160 KB of LDS, so W has an array of its own)
    auto Cv = [&](int i, int k) -> double { return i == k ? dc[k] : (i < k ? L[i][k] : 0.0); };
#pragma unroll 1
    for (int e = tid; e < KB * KB; e += WG) {
        const int i = e / KB, j = e % KB;
        double v = 0.0;
        for (int k = max(i, j); k < KB; ++k) v += Cv(i, k) * Cv(j, k);
        Wl[i][j] = v;
        Wm[e] = v;
    }
    __syncthreads();
    // alpha = W (P^T R), P^T R read from the second Gram
    const double* __restrict__ PR = G2 + KB * KB;
#pragma unroll 1
    for (int e = tid; e < KB * KB; e += WG) {
        const int i = e / KB, c = e % KB;
        double v = 0.0;
#pragma unroll 8
        for (int k = 0; k < KB; ++k) v += Wl[i][k] * PR[k * KB + c];
        Am[e] = v;
    }
}

// beta = scale * W B (one workgroup; B a KB x KB matrix, e.g. Q^T Z).
template <int KB>
__global__ void __launch_bounds__(WG) k_small_mul(const double* __restrict__ Wm, const double* __restrict__ Bm,
                                                  double scale, double* __restrict__ out,
                                                  const Ctrl* __restrict__ ctrl) {
    if (ctrl[0].done != RUNNING) return;
    __shared__ double Ws[KB][KB + 1];
    __shared__ double Bs[KB][KB + 1];
    for (int e = threadIdx.x; e < KB * KB; e += WG) {
        Ws[e / KB][e % KB] = Wm[e];
        Bs[e / KB][e % KB] = Bm[e];
    }
    __syncthreads();
#pragma unroll 1
    for (int e = threadIdx.x; e < KB * KB; e += WG) {
        const int i = e / KB, c = e % KB;
        double v = 0.0;
#pragma unroll 8
        for (int k = 0; k < KB; ++k) v += Ws[i][k] * Bs[k][c];
        out[e] = scale * v;
    }
}

// Every column runs while the block runs: a block start (after the starts of
// fj_batched.hpp set each column's own status) marks all columns running,
// unless one of them was rejected; k_bcg_fin then decides for the block.
template <int KB>
__global__ void k_bcg_start(Ctrl* __restrict__ ctrl) {
    if (threadIdx.x != 0) return;
    for (int q = 0; q < KB; ++q)
        if (ctrl[q].done == BAD_INPUT || ctrl[q].done == BREAKDOWN) return;
    for (int q = 0; q < KB; ++q) ctrl[q].done = RUNNING;
}

// OUT = (ysc Y - 1 shift^T + psc IN C) diag(colscale) over node-major n x KB
// blocks (IN, Y, shift or colscale may be null), C a KB x KB matrix. A wave
// computes bands of 16 nodes: for each 16-column tile of OUT the products
// over the KB inner columns in steps of 4. OUT may be IN or Y: a band's
// loads all precede its stores.
template <int KB>
__global__ void __launch_bounds__(WG) k_block_mul(int n, const double* IN, const double* __restrict__ Cm, double psc,
                                                  const double* Y, double ysc, const double* __restrict__ shift,
                                                  const double* __restrict__ colscale, double* OUT,
                                                  const Ctrl* __restrict__ ctrl) {
    if (ctrl[0].done != RUNNING) return;
    constexpr int TT = KB / 16;
    __shared__ double C[KB * KB];
    for (int e = threadIdx.x; e < KB * KB; e += WG) C[e] = psc * Cm[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane & 15, kk = lane >> 4;
    const int64_t bands = (static_cast<int64_t>(n) + 15) / 16;
    for (int64_t band = static_cast<int64_t>(blockIdx.x) * NWAVE + wave; band < bands;
         band += static_cast<int64_t>(gridDim.x) * NWAVE) {
        const int64_t i0 = band * 16;
        dv4 acc[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t) acc[t] = dv4{0.0, 0.0, 0.0, 0.0};
        if (IN != nullptr) {
            const int64_t ia = i0 + sub;  // A operand: node i0 + sub, inner column k0 + kk
            const bool oka = ia < n;
            double a[KB / 4];  // the band's whole row block in flight before the first product
#pragma unroll
            for (int q = 0; q < KB / 4; ++q) a[q] = oka ? IN[ia * KB + 4 * q + kk] : 0.0;
#pragma unroll
            for (int q = 0; q < KB / 4; ++q) {
#pragma unroll
                for (int t = 0; t < TT; ++t) acc[t] = mfma16(a[q], C[(4 * q + kk) * KB + 16 * t + sub], acc[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < TT; ++t) {
            const int c = 16 * t + sub;
            const double sh = shift != nullptr ? shift[c] : 0.0;
            const double cs = colscale != nullptr ? colscale[c] : 1.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + 4 * r + kk;
                if (i < n) {
                    double v = acc[t][r] - sh;
                    if (Y != nullptr) v += ysc * Y[i * KB + c];
                    OUT[i * KB + c] = v * cs;
                }
            }
        }
    }
}

// Z = M^-1 R (Jacobi), with the per-column partial sums of r^T r (slot 0) and
// of Z (slot 1) for the centring and the stopping test.
template <int KB>
__global__ void __launch_bounds__(WG) k_bcg_precond(int n, const double* __restrict__ R, const float* __restrict__ minv,
                                                    double* __restrict__ Z, double* __restrict__ part,
                                                    const Ctrl* __restrict__ ctrl) {
    if (ctrl[0].done != RUNNING) return;
    __shared__ double lred[2 * WG];
    double v[2] = {0.0, 0.0};
    const int64_t total = static_cast<int64_t>(n) * KB;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * WG) {
        const int i = static_cast<int>(e / KB);
        const double r = R[e];
        const double z = static_cast<double>(minv[i]) * r;
        Z[e] = z;
        v[0] += r * r;
        v[1] += z;
    }
    constexpr int NG = WG / KB;
    lred[threadIdx.x] = v[0];
    lred[WG + threadIdx.x] = v[1];
    __syncthreads();
    if (threadIdx.x < KB) {
        double a = 0.0, b = 0.0;
        for (int g = 0; g < NG; ++g) {
            a += lred[g * KB + threadIdx.x];
            b += lred[WG + g * KB + threadIdx.x];
        }
        double* p = part + (static_cast<int64_t>(blockIdx.x) * KB + threadIdx.x) * BPART;
        p[0] = a;
        p[1] = b;
    }
}

// Per column (one workgroup each): r^T r and sum(Z) over the G partials,
// into tot[c] and tot[KB + c], a fixed-order tree over the workgroup.
template <int KB>
__global__ void __launch_bounds__(WG) k_bcg_colsum(int G, const double* __restrict__ part, double* __restrict__ tot,
                                                   const Ctrl* __restrict__ ctrl) {
    if (ctrl[0].done != RUNNING) return;
    __shared__ double red[NWAVE * 2];
    const int c = blockIdx.x;
    double v[2] = {0.0, 0.0};
    for (int g = threadIdx.x; g < G; g += WG) {
        const double* p = part + (static_cast<int64_t>(g) * KB + c) * BPART;
        v[0] += p[0];
        v[1] += p[1];
    }
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        tot[c] = v[0];
        tot[KB + c] = v[1];
    }
}

// From the column totals: mean(Z) (zcol[c], for the centring) and 1 / ||r_c||
// (zcol[KB + c], the column scaling of the next search block); the block
// stops when every column meets its residual target (the shared space keeps
// improving columns that already do). first = 1 at a start (the iteration
// count is not advanced).
template <int KB>
__global__ void k_bcg_decide(int n, const double* __restrict__ tot, int first, double* __restrict__ zcol,
                             Ctrl* __restrict__ ctrl) {
    if (ctrl[0].done != RUNNING) return;
    const int c = threadIdx.x;
    if (c < KB) {
        zcol[c] = tot[KB + c] / static_cast<double>(n);
        zcol[KB + c] = tot[c] > 0.0 ? 1.0 / sqrt(tot[c]) : 0.0;
    }
    __syncthreads();
    if (c == 0) {
        bool all = true, finite = true;
        for (int q = 0; q < KB; ++q) {
            all = all && tot[q] <= ctrl[q].tol2;
            finite = finite && isfinite(tot[q]) && isfinite(tot[KB + q]);
        }
        const int it = ctrl[0].iters + (first ? 0 : 1);
        int done = RUNNING;
        if (!finite) done = BREAKDOWN;
        else if (all) done = CONVERGED;
        else if (it >= ctrl[0].max_iter) done = ITER_CAP;
        for (int q = 0; q < KB; ++q) {
            Ctrl& C = ctrl[q];
            C.iters = it;
            C.rr = tot[q];
            C.hist[it % HIST] = tot[q];
            C.pbar = 0.0;  // the search block is centred explicitly: the SpMM applies no shift
            C.done = done;
        }
    }
}

}  // namespace fj
