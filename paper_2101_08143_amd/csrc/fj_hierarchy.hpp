// fj_hierarchy.hpp -- the host side of FJ_MULTILEVEL: the aggregation
// hierarchy built from a device-to-host copy of the CSR, uploaded as one
// allocation, and fj_hierarchy_create / _shape / _destroy. The V-cycle that
// uses it is vcycle() in fj_api.hip with the kernels of fj_multilevel.hpp.
// Part of fj_api.hip's translation unit (included once).
#pragma once

namespace {
// One level of the hierarchy on the host: W (CSR, no diagonal) and the
// identity part mass (1 on level 0, the aggregate sizes further down).
struct HostLevel {
    int n = 0;
    std::vector<int> rp, col;
    std::vector<double> w, mass;
};

// Tie-break key of the edge {i, j} (SplitMix64 of the ordered pair): among
// equally heavy edges a node takes the one with the larger key, so that
// uniform weights do not chain a whole path or cycle into one aggregate.
uint64_t edge_key(int i, int j) {
    uint64_t x = (static_cast<uint64_t>(std::min(i, j)) << 32) | static_cast<uint32_t>(std::max(i, j));
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Heaviest-neighbour forest: node i, in index order, is joined to its
// heaviest neighbour (ties by edge_key) unless the merged group would exceed
// ML_LONG nodes; the groups are the aggregates, labelled in the order of their
// smallest node. The cap keeps a hub from gathering most of a power-law graph
// into one aggregate (one member list, and one coarse row, as long as the
// graph). Returns the number of aggregates.
int forest_aggregates(const HostLevel& L, std::vector<int>& agg) {
    std::vector<int> parent(static_cast<size_t>(L.n)), size(static_cast<size_t>(L.n), 1);
    for (int i = 0; i < L.n; ++i) parent[i] = i;
    auto find = [&](int x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    };
    for (int i = 0; i < L.n; ++i) {
        int best = -1;
        double bw = -INFINITY;
        uint64_t bk = 0;
        for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) {
            const uint64_t k = edge_key(i, L.col[e]);
            if (L.w[e] > bw || (L.w[e] == bw && k > bk)) {
                bw = L.w[e];
                bk = k;
                best = L.col[e];
            }
        }
        if (best >= 0) {
            const int a = find(i), b = find(best);
            if (a != b && size[a] + size[b] <= ML_LONG) {
                parent[std::max(a, b)] = std::min(a, b);
                size[std::min(a, b)] += size[std::max(a, b)];
            }
        }
    }
    agg.assign(static_cast<size_t>(L.n), -1);
    std::vector<int> label(static_cast<size_t>(L.n), -1);
    int nc = 0;
    for (int i = 0; i < L.n; ++i) {
        const int r = find(i);
        if (label[r] < 0) label[r] = nc++;
        agg[i] = label[r];
    }
    return nc;
}

// Members of each aggregate (CSR, ascending node order) and the next level:
// W' sums the weights between aggregates in member and entry order, columns
// ascending per row; mass' sums the members' mass.
void galerkin(const HostLevel& L, const std::vector<int>& agg, int nc, std::vector<int>& mrp,
              std::vector<int>& mem, HostLevel& C) {
    mrp.assign(static_cast<size_t>(nc) + 1, 0);
    for (int i = 0; i < L.n; ++i) ++mrp[agg[i] + 1];
    for (int a = 0; a < nc; ++a) mrp[a + 1] += mrp[a];
    mem.assign(static_cast<size_t>(L.n), 0);
    std::vector<int> at(mrp.begin(), mrp.end() - 1);
    for (int i = 0; i < L.n; ++i) mem[at[agg[i]]++] = i;
    C.n = nc;
    C.rp.assign(static_cast<size_t>(nc) + 1, 0);
    C.col.clear();
    C.w.clear();
    C.mass.assign(static_cast<size_t>(nc), 0.0);
    std::vector<int> slot(static_cast<size_t>(nc), -1);
    std::vector<std::pair<int, double>> row;
    for (int a = 0; a < nc; ++a) {
        row.clear();
        for (int k = mrp[a]; k < mrp[a + 1]; ++k) {
            const int i = mem[k];
            C.mass[a] += L.mass[i];
            for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) {
                const int b = agg[L.col[e]];
                if (b == a) continue;
                if (slot[b] < 0) {
                    slot[b] = static_cast<int>(row.size());
                    row.emplace_back(b, L.w[e]);
                } else {
                    row[slot[b]].second += L.w[e];
                }
            }
        }
        for (const auto& pr : row) slot[pr.first] = -1;
        std::sort(row.begin(), row.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
        for (const auto& pr : row) {
            C.col.push_back(pr.first);
            C.w.push_back(pr.second);
        }
        C.rp[a + 1] = static_cast<int>(C.col.size());
    }
}

// Dense inverse of the SPD matrix diag(a) - W (Cholesky, then L^-T L^-1).
void dense_inverse(const HostLevel& L, const std::vector<double>& a, std::vector<double>& inv) {
    const size_t n = static_cast<size_t>(L.n);
    std::vector<double> A(n * n, 0.0);
    for (size_t i = 0; i < n; ++i) {
        A[i * n + i] = a[i];
        for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) A[i * n + L.col[e]] -= L.w[e];
    }
    for (size_t j = 0; j < n; ++j) {  // lower Cholesky factor in place
        double d = A[j * n + j];
        for (size_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        d = std::sqrt(d);
        A[j * n + j] = d;
        for (size_t i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (size_t k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / d;
        }
    }
    std::vector<double> Li(n * n, 0.0);  // L^-1, lower
    for (size_t j = 0; j < n; ++j) {
        Li[j * n + j] = 1.0 / A[j * n + j];
        for (size_t i = j + 1; i < n; ++i) {
            double v = 0.0;
            for (size_t k = j; k < i; ++k) v -= A[i * n + k] * Li[k * n + j];
            Li[i * n + j] = v / A[i * n + i];
        }
    }
    inv.assign(n * n, 0.0);
    for (size_t i = 0; i < n; ++i)
        for (size_t j = 0; j <= i; ++j) {
            double v = 0.0;
            for (size_t k = i; k < n; ++k) v += Li[k * n + i] * Li[k * n + j];
            inv[i * n + j] = v;
            inv[j * n + i] = v;
        }
}

constexpr int ML_DENSE_MAX = 2048;

int build_hierarchy(const fj_csr* g, int coarse_max, hipStream_t st, fj_hierarchy* h) {
    const int n = g->n;
    const int64_t nnz = g->nnz;
    std::vector<HostLevel> lv(1);
    HostLevel& L0 = lv[0];
    L0.n = n;
    L0.rp.resize(static_cast<size_t>(n) + 1, 0);
    L0.col.resize(static_cast<size_t>(nnz));
    L0.w.assign(static_cast<size_t>(nnz), 1.0);
    L0.mass.assign(static_cast<size_t>(n), 1.0);
    HIPCHK(hipStreamSynchronize(st));
    if (n > 0) HIPCHK(hipMemcpy(L0.rp.data(), g->row_ptr, L0.rp.size() * sizeof(int), hipMemcpyDeviceToHost));
    if (nnz > 0) {
        HIPCHK(hipMemcpy(L0.col.data(), g->col_idx, L0.col.size() * sizeof(int), hipMemcpyDeviceToHost));
        if (g->val_type == FJ_VAL_F64) {
            HIPCHK(hipMemcpy(L0.w.data(), g->val, L0.w.size() * sizeof(double), hipMemcpyDeviceToHost));
        } else if (g->val_type == FJ_VAL_F32) {
            std::vector<float> wf(static_cast<size_t>(nnz));
            HIPCHK(hipMemcpy(wf.data(), g->val, wf.size() * sizeof(float), hipMemcpyDeviceToHost));
            for (size_t e = 0; e < wf.size(); ++e) L0.w[e] = wf[e];
        }
    }
    // coarsen
    std::vector<std::vector<int>> aggs, mrps, mems;
    while (static_cast<int>(lv.size()) < ML_MAXL && lv.back().n > coarse_max) {
        std::vector<int> agg, mrp, mem;
        const int nc = forest_aggregates(lv.back(), agg);
        if (static_cast<int64_t>(nc) * 10 > static_cast<int64_t>(lv.back().n) * 9) break;  // < 10 % smaller
        HostLevel C;
        galerkin(lv.back(), agg, nc, mrp, mem, C);
        aggs.push_back(std::move(agg));
        mrps.push_back(std::move(mrp));
        mems.push_back(std::move(mem));
        lv.push_back(std::move(C));
    }
    const int levels = static_cast<int>(lv.size());
    std::vector<std::vector<double>> a(levels);
    std::vector<std::vector<int>> longs(levels), clongs(levels);
    for (int l = 0; l < levels; ++l) {
        const HostLevel& L = lv[l];
        a[l].resize(static_cast<size_t>(L.n));
        for (int i = 0; i < L.n; ++i) {
            double d = L.mass[i];
            for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) d += L.w[e];
            a[l][i] = d;
            if (L.rp[i + 1] - L.rp[i] > ML_LONG) longs[l].push_back(i);
        }
        if (l + 1 < levels)
            for (int c = 0; c + 1 < static_cast<int>(mrps[l].size()); ++c)
                if (mrps[l][c + 1] - mrps[l][c] > ML_LONG) clongs[l].push_back(c);
    }
    const HostLevel& last = lv.back();
    std::vector<double> inv;
    if (last.n > 0 && last.n <= ML_DENSE_MAX) dense_inverse(last, a.back(), inv);
    // device layout: per level rp, col, w, longs, a, ainv (+ agg, mrp, mem, clongs, t for levels with a
    // coarser one), rbuf and xbuf for l >= 1, then the dense inverse
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    struct Off { size_t rp, col, w, longs, a, ainv, agg, mrp, mem, clongs, t, y, rbuf, xbuf; };
    std::vector<Off> o(levels);
    for (int l = 0; l < levels; ++l) {
        const HostLevel& L = lv[l];
        const size_t nl = static_cast<size_t>(L.n);
        o[l].rp = take(sizeof(int) * (nl + 1));
        o[l].col = take(sizeof(int) * L.col.size());
        o[l].w = take(sizeof(double) * L.w.size());
        o[l].longs = take(sizeof(int) * longs[l].size());
        o[l].a = take(sizeof(double) * nl);
        o[l].ainv = take(sizeof(double) * nl);
        o[l].y = take(sizeof(double) * nl);
        if (l + 1 < levels) {
            o[l].agg = take(sizeof(int) * nl);
            o[l].mrp = take(sizeof(int) * mrps[l].size());
            o[l].mem = take(sizeof(int) * nl);
            o[l].clongs = take(sizeof(int) * clongs[l].size());
            o[l].t = take(sizeof(double) * nl);
        }
        if (l >= 1) {
            o[l].rbuf = take(sizeof(double) * nl);
            o[l].xbuf = take(sizeof(double) * nl);
        }
    }
    const size_t inv_off = take(sizeof(double) * inv.size());
    void* mem = nullptr;
    HIPCHK(hipMalloc(&mem, off));
    h->mem = mem;
    char* base = static_cast<char*>(mem);
    auto put = [&](size_t at, const void* src, size_t bytes) -> int {
        if (bytes) HIPCHK(hipMemcpy(base + at, src, bytes, hipMemcpyHostToDevice));
        return FJ_OK;
    };
    h->levels = levels;
    for (int l = 0; l < levels; ++l) {
        const HostLevel& L = lv[l];
        const size_t nl = static_cast<size_t>(L.n);
        std::vector<double> ainv(nl);
        for (size_t i = 0; i < nl; ++i) ainv[i] = 1.0 / a[l][i];
        if (int rc = put(o[l].rp, L.rp.data(), sizeof(int) * (nl + 1))) return rc;
        if (int rc = put(o[l].col, L.col.data(), sizeof(int) * L.col.size())) return rc;
        if (int rc = put(o[l].w, L.w.data(), sizeof(double) * L.w.size())) return rc;
        if (int rc = put(o[l].longs, longs[l].data(), sizeof(int) * longs[l].size())) return rc;
        if (int rc = put(o[l].a, a[l].data(), sizeof(double) * nl)) return rc;
        if (int rc = put(o[l].ainv, ainv.data(), sizeof(double) * nl)) return rc;
        h->n[l] = L.n;
        h->nnz[l] = static_cast<int64_t>(L.col.size());
        h->ybuf[l] = reinterpret_cast<double*>(base + o[l].y);
        h->ainvs[l] = reinterpret_cast<const double*>(base + o[l].ainv);
        if (l >= 1) {
            h->rbuf[l] = reinterpret_cast<double*>(base + o[l].rbuf);
            h->xbuf[l] = reinterpret_cast<double*>(base + o[l].xbuf);
        }
        if (l + 1 < levels) {
            if (int rc = put(o[l].agg, aggs[l].data(), sizeof(int) * nl)) return rc;
            if (int rc = put(o[l].mrp, mrps[l].data(), sizeof(int) * mrps[l].size())) return rc;
            if (int rc = put(o[l].mem, mems[l].data(), sizeof(int) * nl)) return rc;
            if (int rc = put(o[l].clongs, clongs[l].data(), sizeof(int) * clongs[l].size())) return rc;
            MlLevel& M = h->lv[l];
            M.n = L.n;
            M.nc = lv[l + 1].n;
            M.nlong = static_cast<int>(longs[l].size());
            M.nclong = static_cast<int>(clongs[l].size());
            M.rp = reinterpret_cast<const int*>(base + o[l].rp);
            M.col = reinterpret_cast<const int*>(base + o[l].col);
            M.w = reinterpret_cast<const double*>(base + o[l].w);
            M.longs = reinterpret_cast<const int*>(base + o[l].longs);
            M.a = reinterpret_cast<const double*>(base + o[l].a);
            M.ainv = reinterpret_cast<const double*>(base + o[l].ainv);
            M.agg = reinterpret_cast<const int*>(base + o[l].agg);
            M.mrp = reinterpret_cast<const int*>(base + o[l].mrp);
            M.mem = reinterpret_cast<const int*>(base + o[l].mem);
            M.clongs = reinterpret_cast<const int*>(base + o[l].clongs);
            M.t = reinterpret_cast<double*>(base + o[l].t);
        }
    }
    h->nL = last.n;
    h->ainvL = reinterpret_cast<const double*>(base + o[levels - 1].ainv);
    if (!inv.empty()) {
        if (int rc = put(inv_off, inv.data(), sizeof(double) * inv.size())) return rc;
        h->inv = reinterpret_cast<const double*>(base + inv_off);
    }
    return FJ_OK;
}
}  // namespace

int fj_hierarchy_create(const fj_csr* g, int32_t coarse_max, fj_hierarchy** out, void* stream) {
    return guarded([&]() -> int {
        if (!out) return FJ_ERR_INVALID_ARG;
        *out = nullptr;
        if (int rc = check_graph_args(g)) return rc;
        if (coarse_max < 0) return FJ_ERR_INVALID_ARG;
        std::unique_ptr<fj_hierarchy> h(new fj_hierarchy);
        if (int rc = current_device(&h->dev)) return rc;
        h->n0 = g->n;
        h->nnz0 = g->nnz;
        int rc = build_hierarchy(g, coarse_max > 0 ? coarse_max : 1024, static_cast<hipStream_t>(stream), h.get());
        if (rc) {
            if (h->mem) (void)hipFree(h->mem);
            return rc;
        }
        *out = h.release();
        return FJ_OK;
    });
}

int fj_hierarchy_shape(const fj_hierarchy* h, int32_t* levels, int32_t* n, int64_t* nnz, int32_t* dense) {
    return guarded([&]() -> int {
        if (!h) return FJ_ERR_INVALID_ARG;
        if (levels) *levels = h->levels;
        for (int l = 0; l < ML_MAXL; ++l) {
            if (n) n[l] = l < h->levels ? h->n[l] : 0;
            if (nnz) nnz[l] = l < h->levels ? h->nnz[l] : 0;
        }
        if (dense) *dense = h->inv != nullptr ? 1 : 0;
        return FJ_OK;
    });
}

int fj_hierarchy_destroy(fj_hierarchy* h) {
    return guarded([&]() -> int {
        if (!h) return FJ_OK;
        int rc = FJ_OK;
        if (h->mem) {
            if (hipDeviceSynchronize() != hipSuccess || hipFree(h->mem) != hipSuccess) rc = FJ_ERR_HIP;
        }
        delete h;
        return rc;
    });
}
