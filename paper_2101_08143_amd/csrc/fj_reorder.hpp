// fj_reorder.hpp -- optional operator set-up: relabel the nodes by degree
// (fj_reorder_by_degree) and move opinion blocks between the two labellings
// (fj_permute). Part of fj_api.hip's translation unit (included once).
//
// Every CG step gathers p_j once per stored entry of column j, so a column is
// gathered as often as its node has neighbours. Labelling the nodes by
// non-increasing degree puts the most gathered values side by side at the
// front of the vector, where they share cache lines and stay in L2; a random
// labelling of the same graph scatters them (the bare gather over the 4M-node
// workload takes 1.21 ms hub-first and 1.61 ms randomly relabelled). The five
// indices are sums over nodes and edges, so they do not change under a
// relabelling; z comes back in the new labels and fj_permute returns it.
#pragma once

extern "C++" {  // the kernel keeps C++ linkage inside fj_api.hip's extern "C" block
namespace fj {

// y[i, c] = x[perm[i], c] (inverse = 0) or y[perm[i], c] = x[i, c] (inverse = 1),
// node-major blocks with strides ldx, ldy.
__global__ void __launch_bounds__(WG) k_permute(int n, int k, const int* __restrict__ perm,
                                                const double* __restrict__ x, int64_t ldx, double* __restrict__ y,
                                                int64_t ldy, int inverse) {
    const int64_t total = static_cast<int64_t>(n) * k;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * WG + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * WG) {
        const int i = static_cast<int>(e / k), c = static_cast<int>(e % k);
        const int j = perm[i];
        if (j < 0 || j >= n) continue;  // not a permutation of 0..n-1: the entry is skipped
        if (inverse) y[static_cast<int64_t>(j) * ldy + c] = x[static_cast<int64_t>(i) * ldx + c];
        else y[static_cast<int64_t>(i) * ldy + c] = x[static_cast<int64_t>(j) * ldx + c];
    }
}

}  // namespace fj
}  // extern "C++"

int fj_reorder_by_degree(const fj_csr* g, int32_t* perm, int32_t* row_ptr_out, int32_t* col_out, void* val_out,
                         void* stream) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (g->n > 0 && (!perm || !row_ptr_out)) return FJ_ERR_INVALID_ARG;
        if (g->nnz > 0 && (!col_out || (g->val_type != FJ_VAL_UNIT && !val_out))) return FJ_ERR_INVALID_ARG;
        if (g->n == 0) return FJ_OK;
        const int n = g->n;
        const int64_t nnz = g->nnz;
        const size_t vb = g->val_type == FJ_VAL_F64 ? 8 : g->val_type == FJ_VAL_F32 ? 4 : 0;
        std::vector<int> rp(static_cast<size_t>(n) + 1), col(static_cast<size_t>(nnz));
        std::vector<unsigned char> val(static_cast<size_t>(nnz) * vb);
        hipStream_t st = static_cast<hipStream_t>(stream);
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(rp.data(), g->row_ptr, rp.size() * sizeof(int), hipMemcpyDeviceToHost));
        if (nnz > 0) HIPCHK(hipMemcpy(col.data(), g->col_idx, col.size() * sizeof(int), hipMemcpyDeviceToHost));
        if (nnz > 0 && vb) HIPCHK(hipMemcpy(val.data(), g->val, val.size(), hipMemcpyDeviceToHost));
        // new node i is old node p[i]: degrees non-increasing, ties in old order
        std::vector<int> p(static_cast<size_t>(n)), inv(static_cast<size_t>(n));
        for (int i = 0; i < n; ++i) p[i] = i;
        std::stable_sort(p.begin(), p.end(),
                         [&](int a, int b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
        for (int i = 0; i < n; ++i) inv[p[i]] = i;
        std::vector<int> rp2(static_cast<size_t>(n) + 1, 0), col2(static_cast<size_t>(nnz));
        std::vector<unsigned char> val2(val.size());
        std::vector<std::pair<int, int64_t>> row;  // (new column, old entry)
        for (int i = 0; i < n; ++i) {
            const int o = p[i];
            row.clear();
            for (int e = rp[o]; e < rp[o + 1]; ++e) row.emplace_back(inv[col[e]], e);
            std::sort(row.begin(), row.end());
            int64_t at = rp2[i];
            for (const auto& pr : row) {
                col2[at] = pr.first;
                if (vb) std::memcpy(&val2[at * vb], &val[pr.second * vb], vb);
                ++at;
            }
            rp2[i + 1] = static_cast<int>(at);
        }
        HIPCHK(hipMemcpy(perm, p.data(), p.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(row_ptr_out, rp2.data(), rp2.size() * sizeof(int), hipMemcpyHostToDevice));
        if (nnz > 0) HIPCHK(hipMemcpy(col_out, col2.data(), col2.size() * sizeof(int), hipMemcpyHostToDevice));
        if (nnz > 0 && vb) HIPCHK(hipMemcpy(val_out, val2.data(), val2.size(), hipMemcpyHostToDevice));
        return FJ_OK;
    });
}

int fj_permute(int32_t n, int32_t k, const int32_t* perm, const double* x, int64_t ldx, double* y, int64_t ldy,
               int32_t inverse, void* stream) {
    return guarded([&]() -> int {
        if (n < 0 || k < 1 || ldx < k || ldy < k || (inverse != 0 && inverse != 1)) return FJ_ERR_INVALID_ARG;
        if (n == 0) return FJ_OK;
        if (!perm || !x || !y || x == y) return FJ_ERR_INVALID_ARG;
        int grid = 1;
        if (int rc = grid_for(k_permute, (static_cast<int64_t>(n) * k + WG - 1) / WG, &grid)) return rc;
        k_permute<<<grid, WG, 0, static_cast<hipStream_t>(stream)>>>(n, k, perm, x, ldx, y, ldy, inverse);
        HIPCHK(hipGetLastError());
        return FJ_OK;
    });
}
