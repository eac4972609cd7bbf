// Code and batch handles: argument validation, host-side table construction
// and the device copies the kernels read.
#include "cvr_internal.h"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace cvr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

cvr_status fail(cvr_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

cvr_status check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CVR_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return CVR_OK;
}

template <typename T>
static cvr_status upload(std::vector<void*>& owned, const T* host, size_t count, T** dev)
{
    *dev = nullptr;
    if (count == 0) return CVR_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) return fail(CVR_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    owned.push_back(p);
    CVR_HIP_TRY(hipMemcpy(p, host, count * sizeof(T), hipMemcpyHostToDevice));
    *dev = static_cast<T*>(p);
    return CVR_OK;
}

static void free_all(std::vector<void*>& owned)
{
    for (void* p : owned) (void)hipFree(p);
    owned.clear();
}

// Builds the device tables of a code from its CSR form (+ optional QC tables).
static cvr_status finish_code(cvr_code_s* h, int32_t n, int32_t m, const std::vector<int32_t>& row_ptr,
                              const std::vector<int32_t>& col_idx, const std::vector<uint8_t>& etype,
                              int32_t n_types)
{
    const int64_t E = row_ptr[m];
    // column view: edges of each variable in ascending check order
    std::vector<int32_t> col_ptr(size_t(n) + 1, 0), col_edge(static_cast<size_t>(E));
    for (int64_t e = 0; e < E; ++e) col_ptr[size_t(col_idx[e]) + 1]++;
    for (int32_t v = 0; v < n; ++v) col_ptr[v + 1] += col_ptr[v];
    std::vector<int32_t> fill(col_ptr.begin(), col_ptr.end() - 1);
    for (int32_t c = 0; c < m; ++c)
        for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) col_edge[fill[col_idx[e]]++] = int32_t(e);
    int32_t max_col = 0, max_row = 0, min_row = INT32_MAX;
    for (int32_t v = 0; v < n; ++v) max_col = std::max(max_col, col_ptr[v + 1] - col_ptr[v]);
    for (int32_t c = 0; c < m; ++c) {
        max_row = std::max(max_row, row_ptr[c + 1] - row_ptr[c]);
        min_row = std::min(min_row, row_ptr[c + 1] - row_ptr[c]);
    }

    DevCode& d = h->dev;
    d.n = n;
    d.m = m;
    d.E = E;
    d.max_row_deg = max_row;
    d.min_row_deg = min_row;
    d.max_col_deg = max_col;
    d.n_types = n_types;
    h->E = E;
    cvr_status st;
    int32_t *p_rp, *p_ci, *p_cp, *p_ce;
    uint8_t* p_et;
    if ((st = upload(h->allocations, row_ptr.data(), row_ptr.size(), &p_rp))) return st;
    if ((st = upload(h->allocations, col_idx.data(), col_idx.size(), &p_ci))) return st;
    if ((st = upload(h->allocations, etype.data(), etype.size(), &p_et))) return st;
    if ((st = upload(h->allocations, col_ptr.data(), col_ptr.size(), &p_cp))) return st;
    if ((st = upload(h->allocations, col_edge.data(), col_edge.size(), &p_ce))) return st;
    d.row_ptr = p_rp;
    d.col_idx = p_ci;
    d.edge_type = p_et;
    d.col_ptr = p_cp;
    d.col_edge = p_ce;
    return CVR_OK;
}

}  // namespace cvr

using namespace cvr;

extern "C" const char* cvr_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t cvr_version(void) { return 100; }

extern "C" cvr_status cvr_code_create_csr(int32_t n, int32_t m, const int32_t* row_ptr,
                                          const int32_t* col_idx, const uint8_t* edge_type,
                                          int32_t n_types, cvr_code_t* out)
{
    if (!out) return fail(CVR_EINVAL, "cvr_code_create_csr: out is NULL");
    *out = nullptr;
    if (n < 1 || m < 1) return fail(CVR_EINVAL, "cvr_code_create_csr: need n >= 1 and m >= 1");
    if (!row_ptr || !col_idx) return fail(CVR_EINVAL, "cvr_code_create_csr: NULL row_ptr/col_idx");
    if (n_types < 1 || n_types > kMaxTypes) return fail(CVR_EINVAL, "cvr_code_create_csr: n_types must be in [1, 16]");
    if (row_ptr[0] != 0) return fail(CVR_EINVAL, "cvr_code_create_csr: row_ptr[0] != 0");
    for (int32_t c = 0; c < m; ++c) {
        int32_t d = row_ptr[c + 1] - row_ptr[c];
        if (d < 1 || d > kMaxRowDeg)
            return fail(CVR_EINVAL, "cvr_code_create_csr: row " + std::to_string(c) + " has degree " +
                                        std::to_string(d) + " (allowed 1..32)");
        for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
            if (col_idx[e] < 0 || col_idx[e] >= n)
                return fail(CVR_EINVAL, "cvr_code_create_csr: column index out of range in row " + std::to_string(c));
            if (e > row_ptr[c] && col_idx[e] <= col_idx[e - 1])
                return fail(CVR_EINVAL, "cvr_code_create_csr: columns of row " + std::to_string(c) +
                                            " are not strictly ascending");
            if (edge_type && edge_type[e] >= n_types)
                return fail(CVR_EINVAL, "cvr_code_create_csr: edge_type >= n_types");
        }
    }
    const int64_t E = row_ptr[m];
    std::vector<int32_t> rp(row_ptr, row_ptr + m + 1), ci(col_idx, col_idx + E);
    std::vector<uint8_t> et(size_t(E), 0);
    if (edge_type) std::memcpy(et.data(), edge_type, size_t(E));
    auto* h = new cvr_code_s();
    h->dev = DevCode{};
    cvr_status st = finish_code(h, n, m, rp, ci, et, n_types);
    if (st) {
        free_all(h->allocations);
        delete h;
        return st;
    }
    *out = h;
    return CVR_OK;
}

extern "C" cvr_status cvr_code_create_qc(int32_t nb, int32_t mb, int32_t Z, const int32_t* shift,
                                         const uint8_t* block_type, int32_t n_types, cvr_code_t* out)
{
    if (!out) return fail(CVR_EINVAL, "cvr_code_create_qc: out is NULL");
    *out = nullptr;
    if (nb < 1 || mb < 1 || Z < 1) return fail(CVR_EINVAL, "cvr_code_create_qc: need nb, mb, Z >= 1");
    if (int64_t(nb) * Z > INT32_MAX || int64_t(mb) * Z > INT32_MAX)
        return fail(CVR_EINVAL, "cvr_code_create_qc: n or m exceeds int32");
    if (!shift) return fail(CVR_EINVAL, "cvr_code_create_qc: shift is NULL");
    if (n_types < 1 || n_types > kMaxTypes) return fail(CVR_EINVAL, "cvr_code_create_qc: n_types must be in [1, 16]");
    int32_t NB = 0;
    for (int32_t i = 0; i < mb; ++i) {
        int32_t deg = 0;
        for (int32_t j = 0; j < nb; ++j) {
            int32_t s = shift[i * nb + j];
            if (s < -1 || s >= Z) return fail(CVR_EINVAL, "cvr_code_create_qc: shift out of [-1, Z)");
            if (s >= 0) {
                ++deg;
                if (block_type && block_type[i * nb + j] >= n_types)
                    return fail(CVR_EINVAL, "cvr_code_create_qc: block_type >= n_types");
            }
        }
        if (deg < 1 || deg > kMaxRowDeg)
            return fail(CVR_EINVAL, "cvr_code_create_qc: block row " + std::to_string(i) + " has degree " +
                                        std::to_string(deg) + " (allowed 1..32)");
        NB += deg;
    }
    const int32_t n = nb * Z, m = mb * Z;
    // block tables; block ids numbered row-major over the nonzero blocks
    std::vector<int32_t> qrow_ptr(size_t(mb) + 1, 0), qcol_ptr(size_t(nb) + 1, 0);
    std::vector<QcBlock> qrow, qcol(static_cast<size_t>(NB));
    std::vector<int32_t> blk_of(size_t(mb) * nb, -1);
    for (int32_t i = 0; i < mb; ++i) {
        for (int32_t j = 0; j < nb; ++j) {
            int32_t s = shift[i * nb + j];
            if (s < 0) continue;
            int32_t b = int32_t(qrow.size());
            blk_of[size_t(i) * nb + j] = b;
            qrow.push_back(QcBlock{j, s, b, block_type ? block_type[i * nb + j] : 0});
            qcol_ptr[j + 1]++;
        }
        qrow_ptr[i + 1] = int32_t(qrow.size());
    }
    for (int32_t j = 0; j < nb; ++j) qcol_ptr[j + 1] += qcol_ptr[j];
    {
        std::vector<int32_t> fill(qcol_ptr.begin(), qcol_ptr.end() - 1);
        for (int32_t i = 0; i < mb; ++i)                  // rows ascending -> per column ascending
            for (int32_t j = 0; j < nb; ++j) {
                int32_t b = blk_of[size_t(i) * nb + j];
                if (b < 0) continue;
                qcol[fill[j]++] = QcBlock{i, shift[i * nb + j], b, block_type ? block_type[i * nb + j] : 0};
            }
    }
    std::vector<int32_t> rank(static_cast<size_t>(nb));
    for (int32_t j = 0; j < nb; ++j) rank[size_t(j)] = j;
    std::stable_sort(rank.begin(), rank.end(), [&](int32_t x, int32_t y) {
        return qcol_ptr[x + 1] - qcol_ptr[x] > qcol_ptr[y + 1] - qcol_ptr[y];
    });
    // explicit CSR expansion (the generic kernels and syndrome checks use it)
    const int64_t E = int64_t(NB) * Z;
    std::vector<int32_t> rp(size_t(m) + 1, 0), ci(static_cast<size_t>(E));
    std::vector<uint8_t> et(static_cast<size_t>(E));
    int64_t e = 0;
    for (int32_t i = 0; i < mb; ++i)
        for (int32_t k = 0; k < Z; ++k) {
            for (int32_t q = qrow_ptr[i]; q < qrow_ptr[i + 1]; ++q) {
                const QcBlock& blk = qrow[q];
                ci[size_t(e)] = blk.other * Z + (k + blk.shift) % Z;
                et[size_t(e)] = uint8_t(blk.type);
                ++e;
            }
            rp[size_t(i) * Z + k + 1] = int32_t(e);
        }
    auto* h = new cvr_code_s();
    h->dev = DevCode{};
    cvr_status st = finish_code(h, n, m, rp, ci, et, n_types);
    if (!st) {
        DevCode& d = h->dev;
        d.is_qc = 1;
        d.nb = nb;
        d.mb = mb;
        d.Z = Z;
        d.NB = NB;
        int32_t *p_rp, *p_cp, *p_rk;
        QcBlock *p_r, *p_c;
        if (!st) st = upload(h->allocations, qrow_ptr.data(), qrow_ptr.size(), &p_rp);
        if (!st) st = upload(h->allocations, qrow.data(), qrow.size(), &p_r);
        if (!st) st = upload(h->allocations, qcol_ptr.data(), qcol_ptr.size(), &p_cp);
        if (!st) st = upload(h->allocations, qcol.data(), qcol.size(), &p_c);
        if (!st) st = upload(h->allocations, rank.data(), rank.size(), &p_rk);
        int32_t *p_rpk = nullptr, *p_cpk = nullptr;
        if (!st && Z <= 65535 && nb <= 512) {
            std::vector<int32_t> rpk(qrow.size()), cpk(qcol.size());
            for (size_t q = 0; q < qrow.size(); ++q)
                rpk[q] = qrow[q].shift | (qrow[q].other << 16) | (qrow[q].type << 25);
            for (size_t q = 0; q < qcol.size(); ++q) cpk[q] = qcol[q].shift | (qcol[q].blk << 16);
            st = upload(h->allocations, rpk.data(), rpk.size(), &p_rpk);
            if (!st) st = upload(h->allocations, cpk.data(), cpk.size(), &p_cpk);
        }
        if (!st) {
            d.qrow_pk = p_rpk;
            d.qcol_pk = p_cpk;
            d.qcol_rank = p_rk;
            d.qrow_ptr = p_rp;
            d.qrow = p_r;
            d.qcol_ptr = p_cp;
            d.qcol = p_c;
        }
    }
    if (st) {
        free_all(h->allocations);
        delete h;
        return st;
    }
    *out = h;
    return CVR_OK;
}

extern "C" cvr_status cvr_code_info(cvr_code_t code, int32_t* n, int32_t* m, int64_t* n_edges,
                                    int32_t* n_types, int32_t* is_qc)
{
    if (!code) return fail(CVR_EINVAL, "cvr_code_info: NULL code");
    if (n) *n = code->dev.n;
    if (m) *m = code->dev.m;
    if (n_edges) *n_edges = code->dev.E;
    if (n_types) *n_types = code->dev.n_types;
    if (is_qc) *is_qc = code->dev.is_qc;
    return CVR_OK;
}

extern "C" cvr_status cvr_code_destroy(cvr_code_t code)
{
    if (!code) return CVR_OK;
    free_all(code->allocations);
    delete code;
    return CVR_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
static void free_batch(cvr_batch_s* b)
{
    (void)hipFree(b->d_codes);
    (void)hipFree(b->d_frames);
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_cn_tiles);
    (void)hipFree(b->d_vn_tiles);
    (void)hipFree(b->d_qcn_tiles);
    (void)hipFree(b->d_qvn_tiles);
    delete b;
}

template <typename T>
static cvr_status upload_vec(const std::vector<T>& v, T** dev)
{
    *dev = nullptr;
    if (v.empty()) return CVR_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, v.size() * sizeof(T));
    if (e != hipSuccess) return fail(CVR_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    *dev = static_cast<T*>(p);
    CVR_HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return CVR_OK;
}

extern "C" cvr_status cvr_batch_create(const cvr_code_t* codes, int32_t n_codes, const cvr_frame* frames,
                                       int32_t F, cvr_batch_t* out)
{
    if (!out) return fail(CVR_EINVAL, "cvr_batch_create: out is NULL");
    *out = nullptr;
    if (F < 0 || n_codes < 1 || !codes) return fail(CVR_EINVAL, "cvr_batch_create: need F >= 0 and >= 1 code");
    if (F > 0 && !frames) return fail(CVR_EINVAL, "cvr_batch_create: frames is NULL");
    for (int32_t c = 0; c < n_codes; ++c)
        if (!codes[c]) return fail(CVR_EINVAL, "cvr_batch_create: NULL code handle");

    auto* b = new cvr_batch_s();
    b->F = F;
    b->codes.assign(codes, codes + n_codes);
    b->all_qc = true;
    std::vector<DevCode> dc(static_cast<size_t>(n_codes));
    for (int32_t c = 0; c < n_codes; ++c) dc[c] = codes[c]->dev;
    // frame table, overlap checks
    std::vector<std::pair<int64_t, int64_t>> vspan, cspan;
    int64_t msg = 0;
    for (int32_t f = 0; f < F; ++f) {
        const cvr_frame& fr = frames[f];
        if (fr.code_idx < 0 || fr.code_idx >= n_codes || fr.vn_offset < 0 || fr.chk_offset < 0) {
            delete b;
            return fail(CVR_EINVAL, "cvr_batch_create: frame " + std::to_string(f) + " has a bad code index or offset");
        }
        const DevCode& d = dc[fr.code_idx];
        DevFrame df{};
        df.code = fr.code_idx;
        df.n = d.n;
        df.m = d.m;
        df.vn_off = fr.vn_offset;
        df.chk_off = fr.chk_offset;
        df.msg_off = msg;
        msg += (d.E + 63) / 64 * 64;    // keep every frame's messages 256-byte aligned (fp32)
        b->frames_host.push_back(df);
        vspan.emplace_back(fr.vn_offset, fr.vn_offset + d.n);
        cspan.emplace_back(fr.chk_offset, fr.chk_offset + d.m);
        b->total_n = std::max(b->total_n, fr.vn_offset + d.n);
        b->total_m = std::max(b->total_m, fr.chk_offset + d.m);
        b->max_row_deg = std::max(b->max_row_deg, d.max_row_deg);
        b->max_types = std::max(b->max_types, d.n_types);
        if (d.is_qc) {
            b->max_mb = std::max(b->max_mb, d.mb);
            b->max_nb = std::max(b->max_nb, d.nb);
            b->max_NB = std::max(b->max_NB, d.NB);
        }
        if (!d.is_qc) b->all_qc = false;
    }
    b->total_E = msg;
    for (auto* spans : {&vspan, &cspan}) {
        std::sort(spans->begin(), spans->end());
        for (size_t i = 1; i < spans->size(); ++i)
            if ((*spans)[i].first < (*spans)[i - 1].second) {
                delete b;
                return fail(CVR_EINVAL, "cvr_batch_create: frames overlap");
            }
    }
    if (b->total_n > INT64_C(1) << 40) {
        delete b;
        return fail(CVR_EINVAL, "cvr_batch_create: batch too large");
    }
    // work lists
    std::vector<Tile> cn, vn, qcn, qvn;
    for (int32_t f = 0; f < F; ++f) {
        const DevCode& d = dc[b->frames_host[f].code];
        for (int32_t r = 0; r < d.m; r += kTile) cn.push_back(Tile{f, r, 0, std::min(kTile, d.m - r)});
        for (int32_t v = 0; v < d.n; v += kTile)
            vn.push_back(Tile{f, v, 0, std::min(kTile, d.n - v) | (v == 0 ? kFirstTile : 0)});
        if (d.is_qc) {
            for (int32_t i = 0; i < d.mb; ++i)
                for (int32_t k = 0; k < d.Z; k += kTile) qcn.push_back(Tile{f, i, k, std::min(kTile, d.Z - k)});
            for (int32_t j = 0; j < d.nb; ++j)
                for (int32_t u = 0; u < d.Z; u += kTile)
                    qvn.push_back(Tile{f, j, u, std::min(kTile, d.Z - u) | (j == 0 && u == 0 ? kFirstTile : 0)});
        }
    }
    // the persistent decoder hands frames out largest first (longest-processing-
    // time order), so a few long frames do not trail at the end of a launch
    std::vector<int32_t> order(static_cast<size_t>(F));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return dc[b->frames_host[x].code].E > dc[b->frames_host[y].code].E;
    });
    cvr_status st = CVR_OK;
    if (!st) st = upload_vec(order, &b->d_order);
    if (!st) st = upload_vec(dc, &b->d_codes);
    if (!st) st = upload_vec(b->frames_host, &b->d_frames);
    if (!st) st = upload_vec(cn, &b->d_cn_tiles);
    if (!st) st = upload_vec(vn, &b->d_vn_tiles);
    if (!st && b->all_qc) st = upload_vec(qcn, &b->d_qcn_tiles);
    if (!st && b->all_qc) st = upload_vec(qvn, &b->d_qvn_tiles);
    if (st) {
        free_batch(b);
        return st;
    }
    b->n_cn_tiles = int64_t(cn.size());
    b->n_vn_tiles = int64_t(vn.size());
    b->n_qcn_tiles = b->all_qc ? int64_t(qcn.size()) : 0;
    b->n_qvn_tiles = b->all_qc ? int64_t(qvn.size()) : 0;
    *out = b;
    return CVR_OK;
}

extern "C" cvr_status cvr_batch_info(cvr_batch_t batch, int32_t* F, int64_t* total_n, int64_t* total_m,
                                     int64_t* total_edges)
{
    if (!batch) return fail(CVR_EINVAL, "cvr_batch_info: NULL batch");
    if (F) *F = batch->F;
    if (total_n) *total_n = batch->total_n;
    if (total_m) *total_m = batch->total_m;
    if (total_edges) {
        int64_t e = 0;
        for (const auto& f : batch->frames_host) e += batch->codes[f.code]->E;
        *total_edges = e;
    }
    return CVR_OK;
}

extern "C" cvr_status cvr_batch_destroy(cvr_batch_t batch)
{
    if (!batch) return CVR_OK;
    free_batch(batch);
    return CVR_OK;
}
