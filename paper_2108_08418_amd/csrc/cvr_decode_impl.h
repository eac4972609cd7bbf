// Batched flooding belief-propagation decoding of sub-blocks (Sec. III-A,
// Sec. III-C) and syndrome checks (Sec. II Step 5).
//
// State kept between the two half-iterations of frame f:
//   c2v  [msg_off .. msg_off + E)  check-to-variable messages (store dtype)
//   Lpost[vn_off .. vn_off + n)    posteriors of the last finished iteration
// The variable-to-check message is never stored: the check pass forms it as
// Lpost[v] - c2v[e] from the two arrays above (for t = 0, c2v = 0).
//
// Iteration t (t = 0..T) of one frame is
//   check pass:    count checks unsatisfied by the decisions of Lpost(t) and,
//                  if t < T, compute c2v(t+1) from Lpost(t) and c2v(t);
//   variable pass: if the count is 0 (early stop) or t == T the frame ends
//                  at t; else Lpost(t+1) = Lch + sum_e c2v(t+1).
// Every pass reads a per-frame `active` flag, so finished frames cost one
// flag read per tile.  Two layouts share this schedule:
//   generic  -- explicit CSR; messages in CSR order; one thread per check row
//               / variable, gathers through col_idx / col_edge;
//   QC       -- quasi-cyclic codes; messages block-major ([block][k]), so both
//               passes touch consecutive addresses per wavefront and need no
//               index arrays (the block tables are wave-uniform).
// Both sum in the same order, so they give bit-identical results.
#pragma once
#include "cvr_internal.h"

#include <algorithm>

namespace cvr {

// ---------------------------------------------------------------------------
// arithmetic helpers
// ---------------------------------------------------------------------------
// phi(x) = -ln tanh(x/2) = 2 atanh(e^-x) = ln((1 + e^-x) / (1 - e^-x)), x >= 0;
// phi(0) = inf, phi(inf) = 0, and phi(phi(x)) = x.
// binary32: one hardware exponential, then either the odd series of 2 atanh(u)
// (u = e^-x < 1/4, truncation < 5e-9 relative) or one hardware logarithm of
// (1 + u) / (1 - u), with 1 - u from its Taylor series below x = 1/8 where the
// subtraction would cancel.  Relative error stays near 2e-6.
__device__ __forceinline__ float phi(float x)
{
    const float u = __expf(-x);
    if (u < 0.25f) {
        const float u2 = u * u;
        float p = 1.0f / 11.0f;
        p = p * u2 + 1.0f / 9.0f;
        p = p * u2 + 1.0f / 7.0f;
        p = p * u2 + 1.0f / 5.0f;
        p = p * u2 + 1.0f / 3.0f;
        p = p * u2 + 1.0f;
        return 2.0f * u * p;
    }
    const float omu = (x < 0.125f)
        ? x * (1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f - x * (1.0f / 120.0f)))))
        : 1.0f - u;
    return __logf(__fdividef(1.0f + u, omu));
}
// binary64: the library's correctly rounded-ish expm1 / log1p.
__device__ __forceinline__ double phi(double x) { return log1p(2.0 / expm1(x)); }

template <typename S> struct StoreT;
template <> struct StoreT<double> {
    __device__ static double put(double v) { return v; }
    __device__ static double get(double s) { return s; }
};
template <> struct StoreT<float> {
    template <typename M> __device__ static float put(M v) { return float(v); }
    __device__ static float get(float s) { return s; }
};
template <> struct StoreT<__half> {
    // round to nearest even, saturating at the largest finite half (NaN kept)
    __device__ static __half put(float v)
    {
        v = v > 65504.0f ? 65504.0f : (v < -65504.0f ? -65504.0f : v);
        return __float2half_rn(v);
    }
    __device__ static float get(__half s) { return __half2float(s); }
};

template <typename M> __device__ __forceinline__ M mabs(M v) { return v < M(0) ? -v : v; }

// Check-node rule on d <= MAXD incoming v2c values x[] (sign flags in negm).
// Writes the outgoing messages through `emit(k, value)`.
template <typename M, int ALGO, int MAXD, typename W, typename Emit>
__device__ __forceinline__ void check_rule(const M (&x)[MAXD], int d, int syn, M clampv, W weight, Emit emit)
{
    uint32_t negm = 0;
#pragma unroll
    for (int k = 0; k < MAXD; ++k)
        if (k < d && x[k] < M(0)) negm |= 1u << k;
    const uint32_t tot = uint32_t(__popc(negm) & 1) ^ uint32_t(syn);
    if (ALGO == CVR_SP) {
        M a[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            M v = mabs(x[k]);
            v = v > clampv ? clampv : v;
            a[k] = (k < d) ? phi(v) : M(0);
        }
        // exclusive sums by prefix + suffix (no total-minus-self cancellation)
        M suf[MAXD];
        M acc = M(0);
#pragma unroll
        for (int k = MAXD - 1; k >= 0; --k) {
            suf[k] = acc;
            if (k < d) acc += a[k];
        }
        acc = M(0);
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            if (k < d) {
                const M mag = phi(acc + suf[k]);
                const bool neg = (tot ^ ((negm >> k) & 1u)) != 0;
                emit(k, neg ? -mag : mag);
                acc += a[k];
            }
        }
    } else {
        M m1 = M(INFINITY), m2 = M(INFINITY);
        int i1 = -1;
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            if (k < d) {
                const M v = mabs(x[k]);
                if (v < m1) {
                    m2 = m1;
                    m1 = v;
                    i1 = k;
                } else if (v < m2) {
                    m2 = v;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            if (k < d) {
                const M mag = (k == i1) ? m2 : m1;
                const bool neg = (tot ^ ((negm >> k) & 1u)) != 0;
                const M w = weight(k);
                emit(k, w * (neg ? -mag : mag));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------
struct DecArgs {
    const DevCode* codes;
    const DevFrame* frames;
    const Tile* tiles;
    const void* llr;          // math dtype
    const uint8_t* syn;       // may be NULL
    void* c2v;                // store dtype
    void* post;               // math dtype
    void* trace;              // math dtype or NULL
    uint8_t* bits;
    int32_t* iters;
    uint8_t* ok;
    int32_t* active;          // [F]
    int32_t* unsat;           // [F][2]
    const float* weights;     // [T][n_types] or NULL
    int64_t total_n;
    float alpha;
    float clamp;
    int32_t t;
    int32_t T;
    int32_t early_stop;
    int32_t n_types;
    float* ckpt;              // [ceil(T / ckpt_every)][ckpt_stride] c2v(t) at t = 0, K, 2K, ... or NULL
    int64_t ckpt_stride;
    int32_t ckpt_every;
};

__device__ __forceinline__ void add_unsat(int32_t* slot, int pred)
{
    const int cnt = __syncthreads_count(pred);
    if (threadIdx.x == 0 && cnt) atomicAdd(slot, cnt);
}

// ---------------------------------------------------------------------------
// generic (explicit CSR) passes
// ---------------------------------------------------------------------------
template <typename M, typename S, int ALGO, int MAXD>
__global__ __launch_bounds__(kTile) void k_check_generic(DecArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    if (!a.active[tl.frame]) return;
    const DevFrame fr = a.frames[tl.frame];
    const DevCode& cd = a.codes[fr.code];
    const int count = tl.count & 0x7fffffff;
    const int r = tl.a + int(threadIdx.x);
    const M* Lp = static_cast<const M*>(a.post) + fr.vn_off;
    S* msg = static_cast<S*>(a.c2v) + fr.msg_off;
    int bad = 0;
    if (int(threadIdx.x) < count) {
        const int e0 = cd.row_ptr[r];
        const int d = cd.row_ptr[r + 1] - e0;
        const int syn = a.syn ? (a.syn[fr.chk_off + r] & 1) : 0;
        int par = syn;
        bool nan = false;
        M x[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            x[k] = M(0);
            if (k < d) {
                const M lp = Lp[cd.col_idx[e0 + k]];
                par ^= (lp < M(0)) ? 1 : 0;
                nan |= (lp != lp);
                x[k] = (a.t == 0) ? lp : lp - M(StoreT<S>::get(msg[e0 + k]));
            }
        }
        bad = par | (nan ? 1 : 0);
        if (a.t < a.T) {
            const float* wt = a.weights ? a.weights + int64_t(a.t) * a.n_types : nullptr;
            auto weight = [&](int k) -> M {
                return wt ? M(wt[cd.edge_type[e0 + k]]) : M(a.alpha);
            };
            auto emit = [&](int k, M v) { msg[e0 + k] = StoreT<S>::put(v); };
            check_rule<M, ALGO, MAXD>(x, d, syn, M(a.clamp), weight, emit);
        }
    }
    add_unsat(&a.unsat[2 * tl.frame + (a.t & 1)], bad);
}

// Ends finished frames; returns true when this tile's frame must not update.
__device__ __forceinline__ bool frame_stops(const DecArgs& a, const Tile& tl)
{
    const int u = a.unsat[2 * tl.frame + (a.t & 1)];
    const bool stop = (a.early_stop && u == 0) || a.t >= a.T;
    if ((tl.count & kFirstTile) && threadIdx.x == 0) {
        if (stop) {
            a.iters[tl.frame] = a.t;
            a.ok[tl.frame] = uint8_t(u == 0);
            a.active[tl.frame] = 0;
        } else {
            a.unsat[2 * tl.frame + ((a.t + 1) & 1)] = 0;
        }
    }
    return stop;
}

template <typename M, typename S>
__global__ __launch_bounds__(kTile) void k_var_generic(DecArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    if (!a.active[tl.frame]) return;
    if (frame_stops(a, tl)) return;
    const DevFrame fr = a.frames[tl.frame];
    const DevCode& cd = a.codes[fr.code];
    const int count = tl.count & 0x7fffffff;
    const int v = tl.a + int(threadIdx.x);
    if (int(threadIdx.x) >= count) return;
    const S* msg = static_cast<const S*>(a.c2v) + fr.msg_off;
    M acc = static_cast<const M*>(a.llr)[fr.vn_off + v];
    for (int k = cd.col_ptr[v]; k < cd.col_ptr[v + 1]; ++k) acc += M(StoreT<S>::get(msg[cd.col_edge[k]]));
    static_cast<M*>(a.post)[fr.vn_off + v] = acc;
    if (a.trace) static_cast<M*>(a.trace)[int64_t(a.t + 1) * a.total_n + fr.vn_off + v] = acc;
}

// ---------------------------------------------------------------------------
// quasi-cyclic passes: tile = (frame, block row / column, first k / u)
// ---------------------------------------------------------------------------
template <typename M, typename S, int ALGO, int MAXD>
__global__ __launch_bounds__(kTile) void k_check_qc(DecArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    if (!a.active[tl.frame]) return;
    const DevFrame fr = a.frames[tl.frame];
    const DevCode& cd = a.codes[fr.code];
    const int count = tl.count & 0x7fffffff;
    const int i = tl.a;
    const int k = tl.b + int(threadIdx.x);
    const int Z = cd.Z;
    const int q0 = cd.qrow_ptr[i];
    const int d = cd.qrow_ptr[i + 1] - q0;
    const M* Lp = static_cast<const M*>(a.post) + fr.vn_off;
    S* msg = static_cast<S*>(a.c2v) + fr.msg_off;
    int bad = 0;
    if (int(threadIdx.x) < count) {
        const int syn = a.syn ? (a.syn[fr.chk_off + int64_t(i) * Z + k] & 1) : 0;
        int par = syn;
        bool nan = false;
        M x[MAXD];
#pragma unroll
        for (int q = 0; q < MAXD; ++q) {
            x[q] = M(0);
            if (q < d) {
                const QcBlock blk = cd.qrow[q0 + q];
                int u = k + blk.shift;
                u = u >= Z ? u - Z : u;
                const M lp = Lp[int64_t(blk.other) * Z + u];
                par ^= (lp < M(0)) ? 1 : 0;
                nan |= (lp != lp);
                x[q] = (a.t == 0) ? lp : lp - M(StoreT<S>::get(msg[int64_t(blk.blk) * Z + k]));
            }
        }
        bad = par | (nan ? 1 : 0);
        if (a.t < a.T) {
            const float* wt = a.weights ? a.weights + int64_t(a.t) * a.n_types : nullptr;
            auto weight = [&](int q) -> M { return wt ? M(wt[cd.qrow[q0 + q].type]) : M(a.alpha); };
            auto emit = [&](int q, M v) { msg[int64_t(cd.qrow[q0 + q].blk) * Z + k] = StoreT<S>::put(v); };
            check_rule<M, ALGO, MAXD>(x, d, syn, M(a.clamp), weight, emit);
        }
    }
    add_unsat(&a.unsat[2 * tl.frame + (a.t & 1)], bad);
}

template <typename M, typename S>
__global__ __launch_bounds__(kTile) void k_var_qc(DecArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    if (!a.active[tl.frame]) return;
    if (frame_stops(a, tl)) return;
    const DevFrame fr = a.frames[tl.frame];
    const DevCode& cd = a.codes[fr.code];
    const int count = tl.count & 0x7fffffff;
    if (int(threadIdx.x) >= count) return;
    const int j = tl.a;
    const int u = tl.b + int(threadIdx.x);
    const int Z = cd.Z;
    const S* msg = static_cast<const S*>(a.c2v) + fr.msg_off;
    const int64_t v = int64_t(j) * Z + u;
    M acc = static_cast<const M*>(a.llr)[fr.vn_off + v];
    for (int q = cd.qcol_ptr[j]; q < cd.qcol_ptr[j + 1]; ++q) {      // block rows ascending
        const QcBlock blk = cd.qcol[q];
        int k = u - blk.shift;
        k = k < 0 ? k + Z : k;
        acc += M(StoreT<S>::get(msg[int64_t(blk.blk) * Z + k]));
    }
    static_cast<M*>(a.post)[fr.vn_off + v] = acc;
    if (a.trace) static_cast<M*>(a.trace)[int64_t(a.t + 1) * a.total_n + fr.vn_off + v] = acc;
}

// ---------------------------------------------------------------------------
// persistent frame-per-workgroup decoder for quasi-cyclic codes
// ---------------------------------------------------------------------------
// Each workgroup takes whole frames from an atomic queue and runs all of a
// frame's iterations itself: the two half-iterations are separated by
// __syncthreads only, so frames stop independently, no grid-wide barrier or
// per-iteration launch exists, and a frame's state is touched by one CU only
// (it stays in that XCD's L2 / the Infinity Cache while the frame is decoded).
// The protograph tables of the current code are cached in LDS.
constexpr int kMaxLdsBlocks = 2048;
constexpr int kMaxLdsDim = 512;

struct LdsCode {
    int32_t rptr[kMaxLdsDim + 1];
    int32_t cptr[kMaxLdsDim + 1];
    int2 row[kMaxLdsBlocks];   // x = shift, y = block column | type << 20 (block id = position)
    int2 col[kMaxLdsBlocks];   // x = shift, y = block id
};

// Wave-uniform values: with WU every wavefront's 64 rows (variables) lie in one
// block row (column), which holds when Z is a multiple of 64; the protograph
// entries, degrees and base pointers then live in scalar registers.
template <bool WU>
__device__ __forceinline__ int uni(int v)
{
    if constexpr (WU) return __builtin_amdgcn_readfirstlane(v);
    else return v;
}

// Element idx of a per-frame array as base + zero-extended 32-bit byte offset,
// the form the global-load unit takes with a scalar base.
template <typename T>
__device__ __forceinline__ T& at(T* base, uint32_t idx)
{
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * uint32_t(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T& at(const T* base, uint32_t idx)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * uint32_t(sizeof(T)));
}

// Returns v unchanged through an empty asm statement.  A conditionally loaded
// value whose only use is a conversion would otherwise get that conversion
// moved next to its load, and with it the wait for the load, which would
// serialize the loads of a step.
template <typename T>
__device__ __forceinline__ T opaque(T v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// One frame, all iterations.  Each pass is written in three phases per step:
// protograph entries from LDS, then every global load of the step with no use
// in between (so a wavefront has all of them in flight at once), then the
// arithmetic.  The per-iteration min-sum weights are staged in LDS.
template <typename M, typename S, int ALGO, int MAXD, int NT, int ROWS, bool WU>
__device__ __forceinline__ void decode_frame(const DecArgs& a, const LdsCode& sc, int32_t (&s_unsat)[2],
                                             float (&s_w)[kMaxTypes], int f, const DevFrame& fr, const DevCode& cd)
{
    const int tid = int(threadIdx.x);
    const int Z = cd.Z;
    const int m = cd.mb * Z, n = cd.nb * Z;
    const int zsh = (Z & (Z - 1)) == 0 ? __ffs(Z) - 1 : -1;
    M* Lp = static_cast<M*>(a.post) + fr.vn_off;
    const M* Lc = static_cast<const M*>(a.llr) + fr.vn_off;
    S* msg = static_cast<S*>(a.c2v) + fr.msg_off;
    const uint8_t* syn = a.syn ? a.syn + fr.chk_off : nullptr;
    M* tr = a.trace ? static_cast<M*>(a.trace) + fr.vn_off : nullptr;
    for (int v = tid; v < n; v += NT) {
        const M l = at(Lc, v);
        at(Lp, v) = l;
        if (tr) tr[v] = l;
    }
    if (tid == 0) {
        s_unsat[0] = 0;
        s_unsat[1] = 0;
    }
    if (a.weights && a.T > 0 && tid < a.n_types) s_w[tid] = a.weights[tid];
    __syncthreads();
    for (int t = 0;; ++t) {
        if (a.ckpt && t < a.T && t % a.ckpt_every == 0) {
            // checkpoint c2v(t) (all zero at t = 0) before the check pass overwrites it
            float* ck = a.ckpt + int64_t(t / a.ckpt_every) * a.ckpt_stride + fr.msg_off;
            const int ef = cd.NB * Z;
            for (int e = tid; e < ef; e += NT) ck[e] = (t == 0) ? 0.0f : float(StoreT<S>::get(msg[e]));
            __syncthreads();
        }
        // check pass: syndrome test of Lpost(t) and c2v(t+1); ROWS rows per
        // thread per step
        int bad = 0;
        for (int r0 = tid; r0 < m; r0 += ROWS * NT) {
            int q0[ROWS], d[ROWS], kk[ROWS], sraw[ROWS];
            int2 ent[ROWS][MAXD];
            M lr[ROWS][MAXD];
            S mr[ROWS][MAXD];
#pragma unroll
            for (int h = 0; h < ROWS; ++h) {
                const int r = r0 + h * NT;
                const bool live = r < m;
                const int rr = live ? r : r0;
                const int i = uni<WU>(zsh >= 0 ? (rr >> zsh) : rr / Z);
                kk[h] = rr - i * Z;
                q0[h] = uni<WU>(sc.rptr[i]);
                d[h] = live ? uni<WU>(sc.rptr[i + 1]) - q0[h] : 0;
                sraw[h] = (syn && live) ? int(at(syn, rr)) : 0;
#pragma unroll
                for (int q = 0; q < MAXD; ++q) ent[h][q] = (q < d[h]) ? sc.row[q0[h] + q] : make_int2(0, 0);
            }
#pragma unroll
            for (int h = 0; h < ROWS; ++h) {
#pragma unroll
                for (int q = 0; q < MAXD; ++q) {
                    lr[h][q] = M(0);
                    mr[h][q] = S(0);
                    if (q < d[h]) {
                        const int shift = uni<WU>(ent[h][q].x);
                        const int col = uni<WU>(ent[h][q].y & 0xfffff);
                        int uu = kk[h] + shift;
                        uu = uu >= Z ? uu - Z : uu;
                        lr[h][q] = at(Lp, uint32_t(col * Z + uu));
                        if (t > 0) mr[h][q] = at(msg, uint32_t((q0[h] + q) * Z + kk[h]));
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < ROWS; ++h) {
                if (d[h] == 0) continue;
                M x[MAXD];
                int par = sraw[h] & 1;
                bool nan = false;
#pragma unroll
                for (int q = 0; q < MAXD; ++q) {
                    x[q] = M(0);
                    if (q < d[h]) {
                        const M lp = lr[h][q];
                        par ^= (lp < M(0)) ? 1 : 0;
                        nan |= (lp != lp);
                        x[q] = (t == 0) ? lp : lp - M(StoreT<S>::get(opaque(mr[h][q])));
                    }
                }
                bad += par | (nan ? 1 : 0);
                if (t < a.T) {
                    const int qb = q0[h], kh = kk[h];
                    const int2(&eh)[MAXD] = ent[h];
                    auto weight = [&](int q) -> M { return a.weights ? M(s_w[uni<WU>(eh[q].y >> 20)]) : M(a.alpha); };
                    auto emit = [&](int q, M v) { at(msg, uint32_t((qb + q) * Z + kh)) = StoreT<S>::put(v); };
                    check_rule<M, ALGO, MAXD>(x, d[h], sraw[h] & 1, M(a.clamp), weight, emit);
                }
            }
        }
        if (bad) atomicAdd(&s_unsat[t & 1], bad);
        __syncthreads();
        const int u = s_unsat[t & 1];
        if ((a.early_stop && u == 0) || t >= a.T) {
            if (tid == 0) {
                a.iters[f] = t;
                a.ok[f] = uint8_t(u == 0);
            }
            break;
        }
        if (tid == 0) s_unsat[(t + 1) & 1] = 0;
        // the next iteration's weights: every read of s_w for iteration t
        // happened before the barrier above
        if (a.weights && t + 1 < a.T && tid < a.n_types) s_w[tid] = a.weights[int64_t(t + 1) * a.n_types + tid];
        // variable pass: Lpost(t+1) = Lch + sum of c2v(t+1) over block rows
        // ascending; the messages are loaded 8 at a time, then summed in order
        for (int v = tid; v < n; v += NT) {
            const int j = uni<WU>(zsh >= 0 ? (v >> zsh) : v / Z);
            const int uu = v - j * Z;
            const int qa = uni<WU>(sc.cptr[j]);
            const int dv = uni<WU>(sc.cptr[j + 1]) - qa;
            M acc = at(Lc, v);
            for (int q8 = 0; q8 < dv; q8 += 8) {
                int2 e[8];
                S c[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) e[q] = (q8 + q < dv) ? sc.col[qa + q8 + q] : make_int2(0, 0);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    c[q] = S(0);
                    if (q8 + q < dv) {
                        const int shift = uni<WU>(e[q].x);
                        const int blk = uni<WU>(e[q].y);
                        int k = uu - shift;
                        k = k < 0 ? k + Z : k;
                        c[q] = at(msg, uint32_t(blk * Z + k));
                    }
                }
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q8 + q < dv) acc += M(StoreT<S>::get(opaque(c[q])));
            }
            at(Lp, v) = acc;
            if (tr) tr[int64_t(t + 1) * a.total_n + v] = acc;
        }
        __syncthreads();
    }
    for (int v = tid; v < n; v += NT) a.bits[fr.vn_off + v] = at(Lp, v) < M(0) ? 1 : 0;
}

template <typename M, typename S, int ALGO, int MAXD, int NT, int ROWS, bool WU, int MINW>
__global__ __launch_bounds__(NT, MINW) void k_frames_qc(DecArgs a, int32_t* queue, int32_t F, const int32_t* order)
{
    __shared__ LdsCode sc;
    __shared__ int32_t s_frame;
    __shared__ int32_t s_unsat[2];
    __shared__ float s_w[kMaxTypes];
    const int tid = int(threadIdx.x);
    int cur = -1;
    for (;;) {
        if (tid == 0) {
            const int slot = atomicAdd(queue, 1);
            s_frame = slot < F ? order[slot] : F;
        }
        __syncthreads();
        const int f = __builtin_amdgcn_readfirstlane(s_frame);     // the same for the whole workgroup
        if (f >= F) break;
        const DevFrame fr = a.frames[f];
        const DevCode& cd = a.codes[fr.code];
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
        }
        decode_frame<M, S, ALGO, MAXD, NT, ROWS, WU>(a, sc, s_unsat, s_w, f, fr, cd);
    }
}

// ---------------------------------------------------------------------------
// set-up and output passes (over the generic variable tiles)
// ---------------------------------------------------------------------------
template <typename M>
__global__ __launch_bounds__(kTile) void k_dec_init(DecArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    const DevFrame fr = a.frames[tl.frame];
    const int count = tl.count & 0x7fffffff;
    if ((tl.count & kFirstTile) && threadIdx.x == 0) {
        a.active[tl.frame] = 1;
        a.unsat[2 * tl.frame] = 0;
        a.unsat[2 * tl.frame + 1] = 0;
        a.iters[tl.frame] = 0;
        a.ok[tl.frame] = 0;
    }
    if (int(threadIdx.x) >= count) return;
    const int64_t v = fr.vn_off + tl.a + int(threadIdx.x);
    const M l = static_cast<const M*>(a.llr)[v];
    static_cast<M*>(a.post)[v] = l;
    if (a.trace) static_cast<M*>(a.trace)[v] = l;
}

template <typename M>
__global__ __launch_bounds__(kTile) void k_dec_final(DecArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    const DevFrame fr = a.frames[tl.frame];
    const int count = tl.count & 0x7fffffff;
    if (int(threadIdx.x) >= count) return;
    const int64_t v = fr.vn_off + tl.a + int(threadIdx.x);
    a.bits[v] = static_cast<const M*>(a.post)[v] < M(0) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// host side (templated launch sequences, instantiated per precision/rule TU)
__global__ __launch_bounds__(256) static void k_zero_i32(int32_t* p, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
template <typename M, typename S, int ALGO, int MAXD>
static cvr_status run_decode(const cvr_batch_s* b, DecArgs a, hipStream_t s, bool qc)
{
    const int64_t nvt = b->n_vn_tiles;
    a.tiles = b->d_vn_tiles;
    {
        ProfScope prof(CVR_PROF_DEC_SETUP, s);
        hipLaunchKernelGGL(k_dec_init<M>, dim3(nvt), dim3(kTile), 0, s, a);
    }
    if (cvr_status st = check_launch("decode init")) return st;
    for (int t = 0; t <= a.T; ++t) {
        a.t = t;
        if (qc) {
            a.tiles = b->d_qcn_tiles;
            {
                ProfScope prof(CVR_PROF_CHECK, s);
                hipLaunchKernelGGL((k_check_qc<M, S, ALGO, MAXD>), dim3(b->n_qcn_tiles), dim3(kTile), 0, s, a);
            }
            a.tiles = b->d_qvn_tiles;
            {
                ProfScope prof(CVR_PROF_VAR, s);
                hipLaunchKernelGGL((k_var_qc<M, S>), dim3(b->n_qvn_tiles), dim3(kTile), 0, s, a);
            }
        } else {
            a.tiles = b->d_cn_tiles;
            {
                ProfScope prof(CVR_PROF_CHECK, s);
                hipLaunchKernelGGL((k_check_generic<M, S, ALGO, MAXD>), dim3(b->n_cn_tiles), dim3(kTile), 0, s, a);
            }
            a.tiles = b->d_vn_tiles;
            {
                ProfScope prof(CVR_PROF_VAR, s);
                hipLaunchKernelGGL((k_var_generic<M, S>), dim3(nvt), dim3(kTile), 0, s, a);
            }
        }
        if (cvr_status st = check_launch("decode iteration")) return st;
    }
    a.tiles = b->d_vn_tiles;
    {
        ProfScope prof(CVR_PROF_DEC_SETUP, s);
        hipLaunchKernelGGL(k_dec_final<M>, dim3(nvt), dim3(kTile), 0, s, a);
    }
    return check_launch("decode final");
}

static inline int device_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

template <typename M, typename S, int ALGO, int MAXD, int NT, int ROWS, bool WU, int MINW>
static cvr_status launch_frames(const cvr_batch_s* b, DecArgs a, int32_t* queue, hipStream_t s)
{
    static int per_cu = 0;      // resident workgroups per CU of this instantiation
    if (per_cu == 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_frames_qc<M, S, ALGO, MAXD, NT, ROWS, WU, MINW>, NT, 0) !=
                hipSuccess ||
            v < 1)
            v = 1;
        per_cu = v;
    }
    const int grid = int(std::min<int64_t>(b->F, int64_t(device_cus()) * per_cu));
    ProfScope prof(CVR_PROF_FRAMES, s);
    hipLaunchKernelGGL((k_frames_qc<M, S, ALGO, MAXD, NT, ROWS, WU, MINW>), dim3(grid), dim3(NT), 0, s, a, queue, b->F,
                       b->d_order);
    return check_launch("decode (persistent)");
}

// Every code of the batch has Z % 64 == 0: each wavefront stays inside one
// block row / column, and the wave-uniform kernel applies.
static inline bool wave_uniform(const cvr_batch_s* b)
{
    for (const cvr_code_t c : b->codes)
        if (c->dev.Z % 64) return false;
    return true;
}

template <typename M, typename S, int ALGO, int MAXD>
static cvr_status run_frames(const cvr_batch_s* b, DecArgs a, int32_t* queue, hipStream_t s, int wg, int rows,
                             int minw)
{
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, s, queue, int64_t(1));
    if (cvr_status st = check_launch("decode queue reset")) return st;
    if (!wave_uniform(b)) return launch_frames<M, S, ALGO, MAXD, 512, 1, false, 1>(b, a, queue, s);
    if constexpr (MAXD > 8) {
        // rows of more than 8 edges need more registers than the wide shapes
        // leave (they would spill): 256 or 512 threads, one row per step
        if (wg == 256) return launch_frames<M, S, ALGO, MAXD, 256, 1, true, 1>(b, a, queue, s);
        return launch_frames<M, S, ALGO, MAXD, 512, 1, true, 1>(b, a, queue, s);
    }
    if (minw == 8) {
        if (wg == 1024) return launch_frames<M, S, ALGO, MAXD, 1024, 1, true, 8>(b, a, queue, s);
        return launch_frames<M, S, ALGO, MAXD, 512, 1, true, 8>(b, a, queue, s);
    }
    if (rows == 2) {
        if (wg == 256) return launch_frames<M, S, ALGO, MAXD, 256, 2, true, 1>(b, a, queue, s);
        if (wg == 1024) return launch_frames<M, S, ALGO, MAXD, 1024, 2, true, 1>(b, a, queue, s);
        return launch_frames<M, S, ALGO, MAXD, 512, 2, true, 1>(b, a, queue, s);
    }
    if (wg == 256) return launch_frames<M, S, ALGO, MAXD, 256, 1, true, 1>(b, a, queue, s);
    if (wg == 1024) return launch_frames<M, S, ALGO, MAXD, 1024, 1, true, 1>(b, a, queue, s);
    return launch_frames<M, S, ALGO, MAXD, 512, 1, true, 1>(b, a, queue, s);
}

template <typename M, typename S, int ALGO>
static cvr_status dispatch_deg(const cvr_batch_s* b, DecArgs a, hipStream_t s, bool qc, bool frames, int32_t* queue,
                               int wg, int rows, int minw)
{
    if (frames) {
        if (b->max_row_deg <= 8) return run_frames<M, S, ALGO, 8>(b, a, queue, s, wg, rows, minw);
        if (b->max_row_deg <= 16) return run_frames<M, S, ALGO, 16>(b, a, queue, s, wg, rows, minw);
        return run_frames<M, S, ALGO, 32>(b, a, queue, s, wg, rows, minw);
    }
    if (b->max_row_deg <= 8) return run_decode<M, S, ALGO, 8>(b, a, s, qc);
    if (b->max_row_deg <= 16) return run_decode<M, S, ALGO, 16>(b, a, s, qc);
    return run_decode<M, S, ALGO, 32>(b, a, s, qc);
}


}  // namespace cvr

namespace cvr {
static inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

static inline size_t msize(int32_t p) { return p == CVR_F64 ? 8 : (p == CVR_F32 ? 4 : 2); }

struct WsLayout {
    size_t c2v, post, active, unsat, queue, total;
};

static inline WsLayout layout(const cvr_batch_s* b, const cvr_decode_params* p)
{
    WsLayout w{};
    size_t off = 0;
    w.c2v = off;
    off = align256(off + size_t(b->total_E) * msize(p->store));
    w.post = off;
    off = align256(off + size_t(b->total_n) * msize(p->math));
    w.active = off;
    off = align256(off + size_t(b->F) * 4);
    w.unsat = off;
    off = align256(off + size_t(b->F) * 8);
    w.queue = off;
    off = align256(off + 4);
    w.total = off;
    return w;
}

// The persistent path needs a quasi-cyclic batch whose protograph tables fit in LDS.
static inline bool frames_fit(const cvr_batch_s* b)
{
    if (!b->all_qc) return false;
    for (const cvr_code_t c : b->codes)
        if (c->dev.NB > kMaxLdsBlocks || c->dev.mb > kMaxLdsDim || c->dev.nb > kMaxLdsDim || c->dev.Z >= (1 << 20))
            return false;
    return true;
}


// One instantiation per (math, store, rule); each lives in its own translation unit.
#define CVR_DECL_DISPATCH(NAME)                                                                      \
    cvr_status NAME(const cvr_batch_s* b, DecArgs a, hipStream_t s, bool qc, bool frames, int32_t* queue, \
                    int wg, int rows, int minw)
CVR_DECL_DISPATCH(decode_f64_sp);
CVR_DECL_DISPATCH(decode_f64_nms);
CVR_DECL_DISPATCH(decode_f32_sp);
CVR_DECL_DISPATCH(decode_f32_nms);
CVR_DECL_DISPATCH(decode_f16_sp);
CVR_DECL_DISPATCH(decode_f16_nms);
}  // namespace cvr
