// Differentiable unrolled normalized min-sum: forward with checkpoints and the
// hand-written adjoint, for learning one scale per (iteration, edge type).
//
// Forward (T iterations, no early stop) is the persistent QC decoder in binary32
// with c2v(t) checkpointed at t = 0, K, 2K, ...; its posteriors are bit-identical
// to ldpc_decode_batch with the same weights and early_stop = 0.
//
// Backward, per frame and per segment [t0, t1) from the last one down:
//   recompute c2v(t0+1 .. t1-1) from the checkpoint c2v(t0) (same arithmetic as
//   the forward, keeping the posteriors L(t0 .. t1-2) it forms on the way),
//   then for t = t1-1 .. t0:
//     L(t)  = L_ch + sum_e c2v(t)                   (kept, or formed for t1-1)
//     v2c_e = L(t) - c2v(t)_e                                   (as the forward)
//     through c2v(t+1)_e = w[t][type_e] * s_e * M_e with s_e the syndrome-and-
//       sign product over the other edges and M_e = min_{k != e} |v2c_k|:
//         dl/dw[t][type_e] += g_e s_e M_e,
//         dl/dv2c_a += g_e w_e s_e sign(v2c_a), a = the lowest-index minimiser
//         over k != e (min1's edge for every e but itself, min2's for it);
//     through v2c_e = L_ch + sum_{e' != e} c2v(t)_{e'}:
//         dl/dc2v(t)_{e'} = sum_{e != e'} dl/dv2c_e, dl/dL_ch += sum_e dl/dv2c_e;
//         kept as the column sums S_v of dl/dv2c and dl/dv2c itself, the next
//         step forming dl/dc2v_{e'} = S_v - dl/dv2c_{e'} as it reads its rows.
// Sign products and the choice of minimiser are piecewise constant; |x| has
// derivative sign(x) with sign(0) = +1.  Workgroups own fixed frame sets and
// reduce the weight gradient in a fixed order (wave butterfly, waves in order,
// frames in order, workgroups in order), so results are run-to-run identical.
#include "cvr_decode_impl.h"

namespace cvr {

constexpr int kGradTypes = 4;
constexpr int kGradMaxT = 128;

struct GradArgs {
    const DevCode* codes;
    const DevFrame* frames;
    const float* llr;
    const uint8_t* syn;
    const float* weights;      // [T][n_types]
    const float* ckpt;         // [nseg][stride]
    int64_t stride;
    const float* dpost;        // [total_n]
    float* dllr;               // [total_n] or NULL
    float* slots;              // [K - 1][stride]: c2v(t0 + 1 .. t0 + K - 1)
    float* S;                  // [total_n]: column sums of dl/dv2c (so dl/dc2v_e = S[v(e)] - GV_e),
                               // used when they do not fit in LDS
    float* GV;                 // [stride]: dl/dv2c
    float* Lp;                 // [K][lstride]: L(t0 .. t0 + K - 1) of the current segment
    int64_t lstride;           // total_n
    float* partials;           // [gridDim.x][T][n_types]
    int32_t T, K, n_types, F;
};

// protograph tables of the current code, in LDS
struct LdsCode {
    int32_t rptr[kMaxLdsDim + 1];
    int32_t cptr[kMaxLdsDim + 1];
    int2 row[kMaxLdsBlocks];   // x = shift, y = block column | type << 20 (block id = position)
    int2 col[kMaxLdsBlocks];   // x = shift, y = block id
};

// Every step below issues all of its loads before using any of them (so a
// wavefront keeps them in flight together); with WU (Z % 64 == 0) the block
// row / column of a wavefront, and so its degree and table entries, are
// wave-uniform.
// SL: the column sums S of the frame in (dynamic) LDS, else in the workspace.
template <int MAXD, bool WU, int NT, bool SL>
__global__ __launch_bounds__(NT) void k_nms_bwd_qc(GradArgs a)
{
    extern __shared__ float s_S[];
    __shared__ LdsCode sc;
    __shared__ float s_red[NT / 64][kGradTypes];
    __shared__ float s_dw[kGradMaxT * kGradTypes];
    const int tid = int(threadIdx.x);
    const int lane = tid & 63, wave = tid >> 6;
    for (int q = tid; q < a.T * kGradTypes; q += NT) s_dw[q] = 0.0f;
    int cur = -1;
    for (int f = blockIdx.x; f < a.F; f += gridDim.x) {
        const DevFrame fr = a.frames[f];
        const DevCode& cd = a.codes[fr.code];
        __syncthreads();
        if (fr.code != cur) {
            for (int q = tid; q <= cd.mb; q += NT) sc.rptr[q] = cd.qrow_ptr[q];
            for (int q = tid; q <= cd.nb; q += NT) sc.cptr[q] = cd.qcol_ptr[q];
            for (int q = tid; q < cd.NB; q += NT) {
                const QcBlock br = cd.qrow[q];
                sc.row[q] = make_int2(br.shift, br.other | (br.type << 20));
                const QcBlock bc = cd.qcol[q];
                sc.col[q] = make_int2(bc.shift, bc.blk);
            }
            cur = fr.code;
            __syncthreads();
        }
        const int Z = cd.Z;
        const int m = cd.mb * Z, n = cd.nb * Z;
        const int zsh = (Z & (Z - 1)) == 0 ? __ffs(Z) - 1 : -1;
        const float* Lc = a.llr + fr.vn_off;
        float* Lbase = a.Lp + fr.vn_off;
        const uint8_t* syn = a.syn ? a.syn + fr.chk_off : nullptr;
        float* S = SL ? s_S : a.S + fr.vn_off;
        float* GV = a.GV + fr.msg_off;
        const float* dpost = a.dpost + fr.vn_off;
        float* dllr = a.dllr ? a.dllr + fr.vn_off : nullptr;

        auto row_of = [&](int r, int& q0, int& d, int& k) {
            const int i = uni<WU>(zsh >= 0 ? (r >> zsh) : r / Z);
            k = r - i * Z;
            q0 = uni<WU>(sc.rptr[i]);
            d = uni<WU>(sc.rptr[i + 1]) - q0;
        };
        auto var_of = [&](int v, int& qa, int& dv, int& u) {
            const int j = uni<WU>(zsh >= 0 ? (v >> zsh) : v / Z);
            u = v - j * Z;
            qa = uni<WU>(sc.cptr[j]);
            dv = uni<WU>(sc.cptr[j + 1]) - qa;
        };
        auto edge_var = [&](int q, int k) -> int {       // variable of row-table entry q at check offset k
            const int2 e = sc.row[q];
            int u = k + uni<WU>(e.x);
            u = u >= Z ? u - Z : u;
            return uni<WU>(e.y & 0xfffff) * Z + u;
        };
        auto col_edge = [&](int q, int u) -> int {       // message index of column-table entry q at variable offset u
            const int2 e = sc.col[q];
            int k = u - uni<WU>(e.x);
            k = k < 0 ? k + Z : k;
            return uni<WU>(e.y) * Z + k;
        };
        // L = L_ch + sum of c2v, block rows ascending (the forward's order)
        auto posterior = [&](const float* c2v, float* Lp) {
            for (int v = tid; v < n; v += NT) {
                int qa, dv, u;
                var_of(v, qa, dv, u);
                float acc = Lc[v];
                for (int q8 = 0; q8 < dv; q8 += 8) {
                    float c[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) c[q] = (q8 + q < dv) ? c2v[col_edge(qa + q8 + q, u)] : 0.0f;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (q8 + q < dv) acc += opaque(c[q]);
                }
                Lp[v] = acc;
            }
        };
        // posteriors and messages of a row and, with Sin, the adjoints of its
        // messages dl/dc2v_e = Sin[v(e)] - GVin_e (GVin NULL: zero), all loaded
        // first; then the incoming v2c as the forward forms it (L_post - c2v; the
        // checkpoint at t = 0 holds zeros)
        auto row_inputs = [&](const float* c2v, const float* Lp, int q0, int d, int k, float (&x)[MAXD],
                              const float* Sin, const float* GVin, float (&g)[MAXD]) {
            float lp[MAXD], cv[MAXD], sv[MAXD], gv[MAXD];
#pragma unroll
            for (int q = 0; q < MAXD; ++q) {
                lp[q] = 0.0f;
                cv[q] = 0.0f;
                sv[q] = 0.0f;
                gv[q] = 0.0f;
                if (q < d) {
                    const int v = edge_var(q0 + q, k);
                    lp[q] = Lp[v];
                    cv[q] = c2v[(q0 + q) * Z + k];
                    if (Sin) sv[q] = Sin[v];
                    if (GVin) gv[q] = GVin[(q0 + q) * Z + k];
                }
            }
#pragma unroll
            for (int q = 0; q < MAXD; ++q) x[q] = (q < d) ? opaque(lp[q]) - opaque(cv[q]) : 0.0f;
#pragma unroll
            for (int q = 0; q < MAXD; ++q) g[q] = (q < d && Sin) ? opaque(sv[q]) - opaque(gv[q]) : 0.0f;
        };

        // dl/dc2v(T)_e = dl/dL(T)_v(e): the first reverse step reads S = dl/dL(T)
        // and no GV; dl/dL_ch starts at dl/dL(T)
        for (int v = tid; v < n; v += NT) S[v] = dpost[v];
        if (dllr)
            for (int v = tid; v < n; v += NT) dllr[v] = dpost[v];
        __syncthreads();

        const int nseg = (a.T + a.K - 1) / a.K;
        for (int seg = nseg - 1; seg >= 0; --seg) {
            const int t0 = seg * a.K, t1 = min(a.T, t0 + a.K);
            const float* ck = a.ckpt + int64_t(seg) * a.stride + fr.msg_off;
            auto c2v_at = [&](int t) -> const float* {
                return t == t0 ? ck : a.slots + int64_t(t - t0 - 1) * a.stride + fr.msg_off;
            };
            auto L_at = [&](int t) -> float* { return Lbase + int64_t(t - t0) * a.lstride; };
            // recompute c2v(t0 + 1 .. t1 - 1), keeping L(t0 .. t1 - 2) for the reverse sweep
            for (int t = t0; t < t1 - 1; ++t) {
                const float* cin = c2v_at(t);
                float* cout = a.slots + int64_t(t - t0) * a.stride + fr.msg_off;
                posterior(cin, L_at(t));
                __syncthreads();
                const float* wt = a.weights + int64_t(t) * a.n_types;
                for (int r = tid; r < m; r += NT) {
                    int q0, d, k;
                    row_of(r, q0, d, k);
                    const int sbit = syn ? (syn[r] & 1) : 0;
                    float x[MAXD], unused[MAXD];
                    row_inputs(cin, L_at(t), q0, d, k, x, nullptr, nullptr, unused);
                    auto weight = [&](int q) -> float { return wt[uni<WU>(sc.row[q0 + q].y >> 20)]; };
                    auto emit = [&](int q, float v) { cout[(q0 + q) * Z + k] = v; };
                    check_rule<float, CVR_NMS, MAXD>(x, d, sbit, 0.0f, weight, emit);
                }
                __syncthreads();
            }
            // reverse through t = t1 - 1 .. t0 (L(t1 - 1) is the one posterior
            // the recomputation did not form)
            for (int t = t1 - 1; t >= t0; --t) {
                const float* cin = c2v_at(t);
                if (t == t1 - 1) {
                    posterior(cin, L_at(t));
                    __syncthreads();
                }
                const float* wt = a.weights + int64_t(t) * a.n_types;
                float acc[kGradTypes] = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int r = tid; r < m; r += NT) {
                    int q0, d, k;
                    row_of(r, q0, d, k);
                    const int sbit = syn ? (syn[r] & 1) : 0;
                    float x[MAXD], g[MAXD];
                    const bool first = seg == nseg - 1 && t == t1 - 1;
                    row_inputs(cin, L_at(t), q0, d, k, x, S, first ? nullptr : GV, g);
                    // signs, and the smallest and second smallest |x| with their
                    // first positions (branch-free, the forward's tie rule)
                    uint32_t negm = 0;
                    float m1 = INFINITY, m2 = INFINITY;
                    int i1 = -1, i2 = -1;
#pragma unroll
                    for (int q = 0; q < MAXD; ++q) {
                        if (q < d) {
                            if (x[q] < 0.0f) negm |= 1u << q;
                            const float v = fabsf(x[q]);
                            const bool lt = v < m1;
                            const bool lt2 = !lt && v < m2;
                            m2 = lt ? m1 : (lt2 ? v : m2);
                            i2 = lt ? i1 : (lt2 ? q : i2);
                            m1 = lt ? v : m1;
                            i1 = lt ? q : i1;
                        }
                    }
                    const uint32_t tot = uint32_t(__popc(negm) & 1) ^ uint32_t(sbit);
                    float s1 = 0.0f, u1 = 0.0f;
#pragma unroll
                    for (int q = 0; q < MAXD; ++q) {
                        if (q < d) {
                            const int ty = uni<WU>(sc.row[q0 + q].y >> 20);
                            const float sg = ((tot ^ ((negm >> q) & 1u)) != 0) ? -1.0f : 1.0f;
                            const float mag = (q == i1) ? m2 : m1;
                            const float contrib = g[q] * sg * mag;
#pragma unroll
                            for (int tt = 0; tt < kGradTypes; ++tt) acc[tt] += (tt == ty) ? contrib : 0.0f;
                            const float u = g[q] * wt[ty] * sg;
                            if (q == i1) u1 = u;
                            else s1 += u;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < MAXD; ++q) {
                        if (q < d) {
                            float gv = 0.0f;
                            if (q == i1) gv = (x[q] < 0.0f) ? -s1 : s1;
                            else if (q == i2) gv = (x[q] < 0.0f) ? -u1 : u1;
                            GV[(q0 + q) * Z + k] = gv;
                        }
                    }
                }
                // fixed-order reduction of this iteration's weight gradient
#pragma unroll
                for (int tt = 0; tt < kGradTypes; ++tt) {
                    float v = acc[tt];
                    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                    if (lane == 0) s_red[wave][tt] = v;
                }
                __syncthreads();
                if (tid == 0)
                    for (int tt = 0; tt < a.n_types; ++tt) {
                        float v = 0.0f;
                        for (int w = 0; w < NT / 64; ++w) v += s_red[w][tt];
                        s_dw[t * kGradTypes + tt] += v;
                    }
                // through the variable nodes: S = the sum of the column's GV (the
                // next reverse step forms dl/dc2v_e = S[v(e)] - GV_e from it)
                for (int v = tid; v < n; v += NT) {
                    int qa, dv, u;
                    var_of(v, qa, dv, u);
                    float gsum = 0.0f;
                    if (dv <= 8) {
                        float gv[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) gv[q] = (q < dv) ? GV[col_edge(qa + q, u)] : 0.0f;
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (q < dv) gsum += opaque(gv[q]);
                    } else {
                        for (int q = 0; q < dv; ++q) gsum += GV[col_edge(qa + q, u)];
                    }
                    if (t > 0) S[v] = gsum;
                    if (dllr) dllr[v] += gsum;
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < a.T * a.n_types; q += NT)
        a.partials[int64_t(blockIdx.x) * a.T * a.n_types + q] = s_dw[(q / a.n_types) * kGradTypes + q % a.n_types];
}

__global__ __launch_bounds__(256) void k_sum_partials(const float* partials, int nblk, int count, float* out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    float v = 0.0f;
    for (int b = 0; b < nblk; ++b) v += partials[int64_t(b) * count + q];
    out[q] = v;
}

// Rows of up to 8 edges run 1024 threads per workgroup (a frame per workgroup,
// so batches of about one frame per CU still have 16 waves per CU); wider rows
// need more registers than that leaves and run 512.
template <int MAXD, bool WU, int NT, bool SL>
static int bwd_per_cu(int dyn)
{
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_nms_bwd_qc<MAXD, WU, NT, SL>, NT, size_t(dyn)) != hipSuccess ||
        v < 1)
        v = 1;
    return v;
}

// Dynamic LDS of the adjoint for batch b: the column sums of its largest
// frame when they fit beside the static tables, else none (they go to the
// workspace).
template <int MAXD, bool WU, int NT>
static int bwd_dyn_lds(const cvr_batch_s* b)
{
    static int room = -1;
    if (room < 0) {
        const int lds_blk = std::min(device_attr(hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, 65536),
                                     device_attr(hipDeviceAttributeMaxSharedMemoryPerBlock, 65536));
        hipFuncAttributes fa{};
        const int st = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_nms_bwd_qc<MAXD, WU, NT, true>)) ==
                               hipSuccess ? int(fa.sharedSizeBytes) : 65536;
        room = std::max(0, lds_blk - st);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_nms_bwd_qc<MAXD, WU, NT, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, room);
    }
    int64_t max_n = 0;
    for (const cvr_code_t c : b->codes) max_n = std::max<int64_t>(max_n, c->dev.n);
    return max_n * 4 <= room ? int(max_n * 4) : 0;
}

// The adjoint launch for batch b: grid (one partial weight-gradient row per
// workgroup) and, when launch is true, the launch itself.
template <int MAXD, bool WU>
static int bwd_launch_wu(const cvr_batch_s* b, const GradArgs* g, hipStream_t s)
{
    constexpr int NT = MAXD <= 8 ? 1024 : 512;
    const int dyn = bwd_dyn_lds<MAXD, WU, NT>(b);
    const int per_cu = dyn > 0 ? bwd_per_cu<MAXD, WU, NT, true>(dyn) : bwd_per_cu<MAXD, WU, NT, false>(0);
    const int grid = int(std::min<int64_t>(b->F, int64_t(device_cus()) * per_cu));
    if (g) {
        if (dyn > 0) hipLaunchKernelGGL((k_nms_bwd_qc<MAXD, WU, NT, true>), dim3(grid), dim3(NT), size_t(dyn), s, *g);
        else hipLaunchKernelGGL((k_nms_bwd_qc<MAXD, WU, NT, false>), dim3(grid), dim3(NT), 0, s, *g);
    }
    return grid;
}

template <int MAXD>
static int bwd_launch(const cvr_batch_s* b, const GradArgs* g, hipStream_t s)
{
    return wave_uniform(b) ? bwd_launch_wu<MAXD, true>(b, g, s) : bwd_launch_wu<MAXD, false>(b, g, s);
}

static int grad_grid(const cvr_batch_s* b)
{
    if (b->max_row_deg <= 8) return bwd_launch<8>(b, nullptr, nullptr);
    if (b->max_row_deg <= 16) return bwd_launch<16>(b, nullptr, nullptr);
    return bwd_launch<32>(b, nullptr, nullptr);
}

static cvr_status check_unrolled(const char* fn, const cvr_batch_s* b, int32_t T, int32_t K)
{
    if (!b) return fail(CVR_EINVAL, std::string(fn) + ": NULL batch");
    if (T < 1 || T > kGradMaxT) return fail(CVR_EINVAL, std::string(fn) + ": T must be in [1, 128]");
    if (K < 1) return fail(CVR_EINVAL, std::string(fn) + ": ckpt_every must be >= 1");
    if (!frames_fit(b)) return fail(CVR_EUNSUPPORTED, std::string(fn) + ": needs QC codes whose tables fit in LDS");
    if (b->max_types > kGradTypes) return fail(CVR_EUNSUPPORTED, std::string(fn) + ": at most 4 edge types");
    if (b->max_row_deg > 32) return fail(CVR_EUNSUPPORTED, std::string(fn) + ": row degree > 32");
    for (const cvr_code_t c : b->codes)
        if (c->dev.min_row_deg < 2)
            return fail(CVR_EUNSUPPORTED, std::string(fn) + ": a check of degree 1 has no finite min-sum message");
    return CVR_OK;
}

struct UnrolledLayout {
    size_t dec, bits, iters, ok, slots, S, GV, Lp, partials, total_fwd, total_bwd;
};

static UnrolledLayout unrolled_layout(const cvr_batch_s* b, int32_t T, int32_t K)
{
    cvr_decode_params p{};
    p.algo = CVR_NMS;
    p.math = CVR_F32;
    p.store = CVR_F32;
    p.max_iter = T;
    UnrolledLayout u{};
    size_t off = 0;
    u.dec = off;
    off = align256(off + layout(b, &p).total);
    u.bits = off;
    off = align256(off + size_t(b->total_n));
    u.iters = off;
    off = align256(off + size_t(b->F) * 4);
    u.ok = off;
    off = align256(off + size_t(b->F));
    u.total_fwd = off;
    off = 0;
    u.slots = off;
    off = align256(off + size_t(K > 1 ? K - 1 : 0) * size_t(b->total_E) * 4);
    u.S = off;
    off = align256(off + size_t(b->total_n) * 4);
    u.GV = off;
    off = align256(off + size_t(b->total_E) * 4);
    u.Lp = off;
    off = align256(off + size_t(std::max<int32_t>(std::min<int32_t>(K, T), 1)) * size_t(b->total_n) * 4);
    u.partials = off;
    off = align256(off + size_t(std::max<int32_t>(b->F, 1)) * size_t(T) * size_t(b->max_types) * 4);
    u.total_bwd = off;
    return u;
}

}  // namespace cvr

using namespace cvr;

extern "C" cvr_status nms_unrolled_sizes(cvr_batch_t batch, int32_t T, int32_t ckpt_every, size_t* ckpt_floats,
                                         size_t* fwd_workspace, size_t* bwd_workspace)
{
    if (cvr_status st = check_unrolled("nms_unrolled_sizes", batch, T, ckpt_every)) return st;
    const UnrolledLayout u = unrolled_layout(batch, T, ckpt_every);
    if (ckpt_floats) *ckpt_floats = size_t((T + ckpt_every - 1) / ckpt_every) * size_t(batch->total_E);
    if (fwd_workspace) *fwd_workspace = u.total_fwd;
    if (bwd_workspace) *bwd_workspace = u.total_bwd;
    return CVR_OK;
}

extern "C" cvr_status nms_unrolled_fwd(cvr_batch_t batch, int32_t T, int32_t ckpt_every, const float* weights,
                                       const float* llr, const uint8_t* syndrome, float* llr_post_out, float* ckpt,
                                       void* workspace, size_t ws_bytes, void* stream)
{
    if (cvr_status st = check_unrolled("nms_unrolled_fwd", batch, T, ckpt_every)) return st;
    if (batch->F == 0) return CVR_OK;
    if (!weights || !llr || !llr_post_out || !ckpt) return fail(CVR_EINVAL, "nms_unrolled_fwd: NULL pointer");
    const UnrolledLayout u = unrolled_layout(batch, T, ckpt_every);
    if (!workspace || ws_bytes < u.total_fwd) return fail(CVR_ENOMEM, "nms_unrolled_fwd: workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(CVR_EINVAL, "nms_unrolled_fwd: workspace not 256-byte aligned");
    char* ws = static_cast<char*>(workspace);
    cvr_decode_params p{};
    p.algo = CVR_NMS;
    p.math = CVR_F32;
    p.store = CVR_F32;
    p.max_iter = T;
    const WsLayout w = layout(batch, &p);
    char* dws = ws + u.dec;
    DecArgs a{};
    a.codes = batch->d_codes;
    a.frames = batch->d_frames;
    a.llr = llr;
    a.syn = syndrome;
    a.c2v = dws + w.c2v;
    a.post = llr_post_out;
    a.trace = nullptr;
    a.bits = reinterpret_cast<uint8_t*>(ws + u.bits);
    a.iters = reinterpret_cast<int32_t*>(ws + u.iters);
    a.ok = reinterpret_cast<uint8_t*>(ws + u.ok);
    a.active = reinterpret_cast<int32_t*>(dws + w.active);
    a.unsat = reinterpret_cast<int32_t*>(dws + w.unsat);
    a.weights = weights;
    a.total_n = batch->total_n;
    a.alpha = 1.0f;
    a.clamp = 0.0f;
    a.T = T;
    a.early_stop = 0;
    a.n_types = batch->max_types;
    a.ckpt = ckpt;
    a.ckpt_stride = batch->total_E;
    a.ckpt_every = ckpt_every;
    return decode_f32_nms(batch, a, hipStream_t(stream), true, 1, reinterpret_cast<int32_t*>(dws + w.queue),
                          reinterpret_cast<int32_t*>(dws + w.grid), LaunchShape{1024, 0, 0, 0});
}

extern "C" cvr_status nms_unrolled_bwd(cvr_batch_t batch, int32_t T, int32_t ckpt_every, const float* weights,
                                       const float* llr, const uint8_t* syndrome, const float* ckpt,
                                       const float* dloss_dpost, float* dweights, float* dllr, void* workspace,
                                       size_t ws_bytes, void* stream)
{
    if (cvr_status st = check_unrolled("nms_unrolled_bwd", batch, T, ckpt_every)) return st;
    if (!dweights) return fail(CVR_EINVAL, "nms_unrolled_bwd: NULL dweights");
    const hipStream_t s = hipStream_t(stream);
    const int count = T * batch->max_types;
    if (batch->F == 0) {
        hipLaunchKernelGGL(k_zero_i32, dim3((count + 255) / 256), dim3(256), 0, s, reinterpret_cast<int32_t*>(dweights),
                           int64_t(count));
        return check_launch("nms_unrolled_bwd zero");
    }
    if (!weights || !llr || !ckpt || !dloss_dpost) return fail(CVR_EINVAL, "nms_unrolled_bwd: NULL pointer");
    const UnrolledLayout u = unrolled_layout(batch, T, ckpt_every);
    if (!workspace || ws_bytes < u.total_bwd) return fail(CVR_ENOMEM, "nms_unrolled_bwd: workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(CVR_EINVAL, "nms_unrolled_bwd: workspace not 256-byte aligned");
    char* ws = static_cast<char*>(workspace);
    GradArgs g{};
    g.codes = batch->d_codes;
    g.frames = batch->d_frames;
    g.llr = llr;
    g.syn = syndrome;
    g.weights = weights;
    g.ckpt = ckpt;
    g.stride = batch->total_E;
    g.dpost = dloss_dpost;
    g.dllr = dllr;
    g.slots = reinterpret_cast<float*>(ws + u.slots);
    g.S = reinterpret_cast<float*>(ws + u.S);
    g.GV = reinterpret_cast<float*>(ws + u.GV);
    g.Lp = reinterpret_cast<float*>(ws + u.Lp);
    g.lstride = batch->total_n;
    g.partials = reinterpret_cast<float*>(ws + u.partials);
    g.T = T;
    g.K = ckpt_every;
    g.n_types = batch->max_types;
    g.F = batch->F;
    const int grid = grad_grid(batch);
    {
        ProfScope prof(CVR_PROF_ADJOINT, s);
        if (batch->max_row_deg <= 8) bwd_launch<8>(batch, &g, s);
        else if (batch->max_row_deg <= 16) bwd_launch<16>(batch, &g, s);
        else bwd_launch<32>(batch, &g, s);
    }
    if (cvr_status st = check_launch("nms_unrolled_bwd")) return st;
    hipLaunchKernelGGL(k_sum_partials, dim3((count + 255) / 256), dim3(256), 0, s, g.partials, grid, count, dweights);
    return check_launch("nms_unrolled_bwd reduce");
}
