// fj_aids.hpp -- measurement aids of the C ABI (fj_gather_bound,
// fj_gather_bound_sliced): bare gathers that bound the SpMV, not part of any
// solve. Part of fj_api.hip's translation unit (included once, after the
// solve machinery it shares: guarded, with_graph, grid_for).
#pragma once

int fj_gather_bound(const fj_csr* g, const double* x, double* y, void* stream) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if (g->nnz == 0) return FJ_OK;
        if (!x || !y) return FJ_ERR_INVALID_ARG;
        hipStream_t st = static_cast<hipStream_t>(stream);
        return with_graph(g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            int grid = 1;
            if (int rc = grid_for(k_gather_bound<Vc>, (g->nnz / 8 + WG) / WG, &grid)) return rc;
            k_gather_bound<Vc><<<grid, WG, 0, st>>>(G, x, y);
            HIPCHK(hipGetLastError());
            return FJ_OK;
        });
    });
}

namespace {
// The regrouped entry streams of fj_gather_bound_sliced, for the last graph
// it was called on (rebuilt when the graph, stream count or hub width changes).
struct SliceKey {
    int dev = -1, vt = 0, n = 0, slices = 0, hub = 0;
    int64_t nnz = 0;
    const void *rp = nullptr, *col = nullptr, *val = nullptr;
    bool operator==(const SliceKey& o) const {
        return dev == o.dev && vt == o.vt && n == o.n && slices == o.slices && hub == o.hub && nnz == o.nnz &&
               rp == o.rp && col == o.col && val == o.val;
    }
};
struct SlicedStreams {
    SliceKey key;
    void* mem = nullptr;  // col | val | off | cnt
    int* col = nullptr;
    void* val = nullptr;
    int64_t* off = nullptr;
    int64_t* cnt = nullptr;
    int64_t bounds[9] = {};
};
std::mutex g_slice_mu;
SlicedStreams g_slice;

// Stream s of S = 8: the tail columns [hub, n) are cut into eight ranges of
// about equal entry count, range s read by stream s only; the entries of the
// hub columns [0, hub) are dealt to the streams in CSR order in eight equal
// runs. Every stream keeps CSR order. S = 1: all entries in CSR order.
int build_slices(const fj_csr* g, const SliceKey& key, hipStream_t st, SlicedStreams* out) {
    const int n = g->n;
    const int64_t nnz = g->nnz;
    const int S = key.slices, H = key.hub;
    const size_t vb = g->val_type == FJ_VAL_F64 ? 8 : g->val_type == FJ_VAL_F32 ? 4 : 0;
    std::vector<int> rp(static_cast<size_t>(n) + 1), col(static_cast<size_t>(nnz));
    std::vector<unsigned char> val(static_cast<size_t>(nnz) * vb);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(rp.data(), g->row_ptr, rp.size() * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(col.data(), g->col_idx, col.size() * sizeof(int), hipMemcpyDeviceToHost));
    if (vb) HIPCHK(hipMemcpy(val.data(), g->val, val.size(), hipMemcpyDeviceToHost));
    std::vector<int64_t> bounds(9, n);
    bounds[0] = std::min(H, n);
    std::vector<int> sid(static_cast<size_t>(nnz), 0);
    if (S == 8) {
        std::vector<int64_t> per_col(static_cast<size_t>(n) + 1, 0);
        int64_t tail = 0, hub_total = 0;
        for (int64_t e = 0; e < nnz; ++e) {
            if (col[e] >= H) { ++per_col[col[e]]; ++tail; }
            else ++hub_total;
        }
        int64_t cum = 0;
        int next = 1;
        for (int c = bounds[0]; c < n && next < 8; ++c) {
            cum += per_col[c];
            while (next < 8 && cum * 8 >= tail * next) bounds[next++] = c + 1;
        }
        int64_t hub_seen = 0;
        for (int64_t e = 0; e < nnz; ++e) {
            const int c = col[e];
            if (c < H) {
                sid[e] = static_cast<int>(hub_seen * 8 / std::max<int64_t>(hub_total, 1));
                ++hub_seen;
            } else {
                sid[e] = static_cast<int>(std::upper_bound(bounds.begin() + 1, bounds.begin() + 8, c) -
                                          (bounds.begin() + 1));
            }
        }
    }
    int64_t cnt[8] = {}, off[9] = {};
    for (int64_t e = 0; e < nnz; ++e) ++cnt[sid[e]];
    for (int s = 0; s < S; ++s) off[s + 1] = off[s] + (cnt[s] + 7) / 8 * 8;
    const int64_t total = off[S];
    std::vector<int> hcol(static_cast<size_t>(total), 0);
    std::vector<unsigned char> hval(static_cast<size_t>(total) * vb, 0);
    int64_t at[8];
    std::copy(off, off + 8, at);
    for (int64_t e = 0; e < nnz; ++e) {
        const int64_t d = at[sid[e]]++;
        hcol[d] = col[e];
        if (vb) std::memcpy(&hval[d * vb], &val[e * vb], vb);
    }
    const size_t col_b = align_up(static_cast<size_t>(total) * 4), val_b = align_up(static_cast<size_t>(total) * vb);
    void* mem = nullptr;
    HIPCHK(hipMalloc(&mem, col_b + val_b + 2 * 256));
    unsigned char* base = static_cast<unsigned char*>(mem);
    out->mem = mem;
    out->col = reinterpret_cast<int*>(base);
    out->val = vb ? base + col_b : nullptr;
    out->off = reinterpret_cast<int64_t*>(base + col_b + val_b);
    out->cnt = reinterpret_cast<int64_t*>(base + col_b + val_b + 256);
    HIPCHK(hipMemcpy(out->col, hcol.data(), hcol.size() * 4, hipMemcpyHostToDevice));
    if (vb) HIPCHK(hipMemcpy(out->val, hval.data(), hval.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(out->off, off, sizeof(off), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(out->cnt, cnt, sizeof(cnt), hipMemcpyHostToDevice));
    std::copy(bounds.begin(), bounds.end(), out->bounds);
    out->key = key;
    return FJ_OK;
}
}  // namespace

int fj_gather_bound_sliced(const fj_csr* g, const void* x, int32_t x_bytes, double* y, int32_t slices,
                           int32_t hub_cols, int32_t* check, int64_t* bounds, void* stream) {
    return guarded([&]() -> int {
        if (int rc = check_graph_args(g)) return rc;
        if ((slices != 1 && slices != 8) || (x_bytes != 4 && x_bytes != 8) || hub_cols < 0)
            return FJ_ERR_INVALID_ARG;
        if (g->nnz == 0) return FJ_OK;
        if (!x || !y) return FJ_ERR_INVALID_ARG;
        hipStream_t st = static_cast<hipStream_t>(stream);
        int dev = 0;
        if (int rc = current_device(&dev)) return rc;
        const SliceKey key{dev, g->val_type, g->n, slices, slices == 8 ? hub_cols : 0, g->nnz,
                           g->row_ptr, g->col_idx, g->val};
        std::lock_guard<std::mutex> lock(g_slice_mu);
        if (!(g_slice.key == key)) {
            if (g_slice.mem) {
                HIPCHK(hipDeviceSynchronize());
                HIPCHK(hipFree(g_slice.mem));
            }
            g_slice = SlicedStreams{};
            if (int rc = build_slices(g, key, st, &g_slice)) {
                if (g_slice.mem) (void)hipFree(g_slice.mem);
                g_slice = SlicedStreams{};
                return rc;
            }
        }
        if (bounds) std::copy(g_slice.bounds, g_slice.bounds + 9, bounds);
        return with_graph(g, [&](auto G) -> int {
            using Vc = typename decltype(G)::value_type;
            const Vc* val = static_cast<const Vc*>(g_slice.val);
            int grid = 1;
            auto launch = [&](auto kern, auto xp) -> int {
                if (int rc = grid_for(kern, (g->nnz / 8 + WG) / WG + slices, &grid)) return rc;
                grid = std::max(slices, grid / slices * slices);
                kern<<<grid, WG, 0, st>>>(g_slice.col, val, xp, y, g_slice.off, g_slice.cnt, check);
                HIPCHK(hipGetLastError());
                return FJ_OK;
            };
            const double* x8 = static_cast<const double*>(x);
            const float* x4 = static_cast<const float*>(x);
            if (slices == 8)
                return x_bytes == 8 ? launch(k_gather_sliced<Vc, double, 8>, x8) : launch(k_gather_sliced<Vc, float, 8>, x4);
            return x_bytes == 8 ? launch(k_gather_sliced<Vc, double, 1>, x8) : launch(k_gather_sliced<Vc, float, 1>, x4);
        });
    });
}
