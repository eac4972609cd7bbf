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
#include <type_traits>

namespace cvr {

// ---------------------------------------------------------------------------
// arithmetic helpers
// ---------------------------------------------------------------------------
// phi(x) = -ln tanh(x/2) = 2 atanh(e^-x) = ln((1 + e^-x) / (1 - e^-x)), x >= 0;
// phi(0) = inf, phi(inf) = 0, and phi(phi(x)) = x.
// binary32, branch-free on the hardware exp2 / reciprocal / log2 (about 1 ulp
// each): u = e^-x; where u < 1/8 the odd series of 2 atanh(u) to u^7 (the rest
// is below u^8/9 / (1 - u^2) < 7e-9 relative), elsewhere ln of
// coth(x/2) = (1 + u) / (1 - u) (>= 9/7, so the log keeps its relative
// accuracy).  Below x = 1/8, where 1 - u would cancel, the quotient is taken
// from the Laurent series coth(x/2) = (2 + x^2/6 - x^4/360 + ...) / x, cut
// after x^2 (the rest is below x^4/720 < 4e-7 relative, against ln coth >
// 2.7).  Relative error stays below about 1e-6 (1.3e-6 with every hardware
// operation 1 ulp off).
__device__ __forceinline__ float phi(float x)
{
    const float u = __builtin_amdgcn_exp2f(x * -1.44269504f);
    const float u2 = u * u;
    float p = 2.0f / 7.0f;
    p = p * u2 + 2.0f / 5.0f;
    p = p * u2 + 2.0f / 3.0f;
    p = p * u2 + 2.0f;
    const float series = u * p;
    const bool small = x < 0.125f;
    const float num = small ? x * x * (1.0f / 6.0f) + 2.0f : 1.0f + u;
    const float den = small ? x : 1.0f - u;
    const float lg = __builtin_amdgcn_logf(num * __builtin_amdgcn_rcpf(den)) * 0.693147181f;
    return (u < 0.125f) ? series : lg;
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

// |v| as fabs gives it: the sign bit cleared, so -0 has magnitude +0 (phi(-0)
// would otherwise take 1 / -0 = -inf into its logarithm).
__device__ __forceinline__ float mabs(float v) { return __builtin_fabsf(v); }
__device__ __forceinline__ double mabs(double v) { return __builtin_fabs(v); }

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
        // smallest and second smallest |x| and the first position of the
        // smallest, branch-free; a NaN compares false and changes nothing
        M m1 = M(INFINITY), m2 = M(INFINITY);
        int i1 = -1;
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            if (k < d) {
                const M v = mabs(x[k]);
                const bool lt = v < m1;
                const M c = (v < m2) ? v : m2;
                m2 = lt ? m1 : c;
                i1 = lt ? k : i1;
                m1 = lt ? v : m1;
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
    uint32_t* synw;           // layered schedule, when LDS is short: syndrome bit arrays, frame f at word chk_off / 32 + f
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

// Tuning knobs of the persistent decoder (none of them changes results).
struct LaunchShape {
    int32_t wg, min_waves, lds_kb, group_wgs;
};

__device__ __forceinline__ void add_unsat(int32_t* slot, int pred)
{
    const int cnt = __syncthreads_count(pred);
    if (threadIdx.x == 0 && cnt) atomicAdd(slot, cnt);
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

// A load of data that other workgroups of the same launch write: with COH a
// device-scope load, which skips this CU's L1 (the XCD's L2 holds the current
// value); otherwise a plain load.
template <bool COH, typename T>
__device__ __forceinline__ T ldc(const T* p)
{
    if constexpr (!COH) {
        return *p;
    } else if constexpr (sizeof(T) == 2) {
        const unsigned short v =
            __hip_atomic_load(reinterpret_cast<const unsigned short*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        T r;
        __builtin_memcpy(&r, &v, 2);
        return r;
    } else {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Every pass below is written in phases: indices / protograph entries, then all
// global loads of the step with no use in between (so they are in flight
// together), then the arithmetic.

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
        int col[MAXD];
        M lr[MAXD];
        S mr[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            col[k] = 0;
            mr[k] = S(0);
            if (k < d) {
                col[k] = cd.col_idx[e0 + k];
                if (a.t > 0) mr[k] = msg[e0 + k];
            }
        }
#pragma unroll
        for (int k = 0; k < MAXD; ++k) lr[k] = (k < d) ? at(Lp, uint32_t(col[k])) : M(0);
        int par = syn;
        bool nan = false;
        M x[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            x[k] = M(0);
            if (k < d) {
                const M lp = lr[k];
                par ^= (lp < M(0)) ? 1 : 0;
                nan |= (lp != lp);
                x[k] = (a.t == 0) ? lp : lp - M(StoreT<S>::get(opaque(mr[k])));
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
    // the counts are updated by atomics: read and reset them with atomics too
    const int u = __hip_atomic_load(&a.unsat[2 * tl.frame + (a.t & 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool stop = (a.early_stop && u == 0) || a.t >= a.T;
    if ((tl.count & kFirstTile) && threadIdx.x == 0) {
        if (stop) {
            a.iters[tl.frame] = a.t;
            a.ok[tl.frame] = uint8_t(u == 0);
            a.active[tl.frame] = 0;
        } else {
            __hip_atomic_store(&a.unsat[2 * tl.frame + ((a.t + 1) & 1)], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    const int k0 = cd.col_ptr[v], dv = cd.col_ptr[v + 1] - k0;
    for (int q8 = 0; q8 < dv; q8 += 8) {            // CSR edge order, 8 loads at a time
        int ed[8];
        S c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) ed[q] = (q8 + q < dv) ? cd.col_edge[k0 + q8 + q] : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = (q8 + q < dv) ? at(msg, uint32_t(ed[q])) : S(0);
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q8 + q < dv) acc += M(StoreT<S>::get(opaque(c[q])));
    }
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
        QcBlock blk[MAXD];
        M lr[MAXD];
        S mr[MAXD];
#pragma unroll
        for (int q = 0; q < MAXD; ++q)
            if (q < d) blk[q] = cd.qrow[q0 + q];
#pragma unroll
        for (int q = 0; q < MAXD; ++q) {
            lr[q] = M(0);
            mr[q] = S(0);
            if (q < d) {
                int u = k + blk[q].shift;
                u = u >= Z ? u - Z : u;
                lr[q] = at(Lp, uint32_t(blk[q].other * Z + u));
                if (a.t > 0) mr[q] = at(msg, uint32_t(blk[q].blk * Z + k));
            }
        }
        int par = syn;
        bool nan = false;
        M x[MAXD];
#pragma unroll
        for (int q = 0; q < MAXD; ++q) {
            x[q] = M(0);
            if (q < d) {
                const M lp = lr[q];
                par ^= (lp < M(0)) ? 1 : 0;
                nan |= (lp != lp);
                x[q] = (a.t == 0) ? lp : lp - M(StoreT<S>::get(opaque(mr[q])));
            }
        }
        bad = par | (nan ? 1 : 0);
        if (a.t < a.T) {
            const float* wt = a.weights ? a.weights + int64_t(a.t) * a.n_types : nullptr;
            auto weight = [&](int q) -> M { return wt ? M(wt[blk[q].type]) : M(a.alpha); };
            auto emit = [&](int q, M v) { at(msg, uint32_t(blk[q].blk * Z + k)) = StoreT<S>::put(v); };
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
    const int qa = cd.qcol_ptr[j], dv = cd.qcol_ptr[j + 1] - qa;
    for (int q8 = 0; q8 < dv; q8 += 8) {            // block rows ascending, 8 loads at a time
        QcBlock blk[8];
        S c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q8 + q < dv) blk[q] = cd.qcol[qa + q8 + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            c[q] = S(0);
            if (q8 + q < dv) {
                int k = u - blk[q].shift;
                k = k < 0 ? k + Z : k;
                c[q] = at(msg, uint32_t(blk[q].blk * Z + k));
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q8 + q < dv) acc += M(StoreT<S>::get(opaque(c[q])));
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
// per-iteration launch exists, and a frame's state is touched by one CU only.
constexpr int kMaxLdsBlocks = 2048;   // protograph limits of the persistent path
constexpr int kMaxLdsDim = 512;
constexpr int kMaxLdsZ = 65535;

// Dynamic LDS of the persistent decoder, in 32-bit words at the offsets that
// LdsMap carries (sized for the largest code of the batch):
//   rptr [mb+1], cptr [nb+1]   block-row / block-column pointers
//   row  [NB]   shift | loc << 16 | type << 25 | cached << 29; loc is the block
//               column, or its cache slot when the column is cached
//   col  [NB]   shift | block id << 16
//   cslot[nb]   cache slot of each block column, -1 when it is not cached
//   cache       posteriors of the cached block columns, Z per slot
// The cached columns are the code's highest-degree ones: a posterior is
// gathered once per edge and written once per iteration, so a column of
// degree d kept in LDS saves d + 1 HBM accesses per value and iteration.
struct LdsMap {
    int32_t rptr, cptr, row, col, cslot, cache;   // word offsets
    int32_t cache_bytes;
    int32_t hard;                                 // layered schedule: hard-decision bits
    int32_t synb;                                 // layered schedule: syndrome bits
    int32_t grp;                                  // layered schedule: layer groups
};
constexpr int32_t kCached = 1 << 29;

// An LDS read that the compiler cannot merge with a global load of the other
// branch (a merged load would be a slower generic-address FLAT load); the
// explicit LDS address space keeps the volatile access a ds_read.
template <typename T>
__device__ __forceinline__ T lds_read(const T* p)
{
    return *(const volatile __attribute__((address_space(3))) T*)(p);
}

// Wave-uniform values: with WU every wavefront's 64 rows (variables) lie in one
// block row (column), which holds when Z is a multiple of 64; the protograph
// entries, degrees and base pointers then live in scalar registers.
template <bool WU>
__device__ __forceinline__ int uni(int v)
{
    if constexpr (WU) return __builtin_amdgcn_readfirstlane(v);
    else return v;
}

// What the row and column steps of one frame need.
template <typename M, typename S>
struct FrameCtx {
    M* Lp;
    const M* Lc;
    S* msg;
    const int32_t* s_row;
    const int32_t* s_col;
    const int32_t* s_cslot;
    M* s_post;
    const float* s_w;
    int Z, t, T;
    bool weighted;
    float alpha, clamp;
};

// Check rows k[0..R) of the block row whose table entries start at q0, with
// exactly D edges (D and the entries wave-uniform): the R x D posteriors and,
// for t > 0, the R x D stored messages are loaded before any arithmetic, so
// they are in flight together; the code is straight-line.  Returns the number
// of the R rows whose syndrome test fails on Lpost(t).
template <typename M, typename S, int ALGO, int D, bool WU, bool CACHE, bool COH, int R>
__device__ __forceinline__ int check_rows(const FrameCtx<M, S>& c, int q0, const int (&k)[R], const int (&sraw)[R])
{
    int32_t e[D];
#pragma unroll
    for (int q = 0; q < D; ++q) e[q] = uni<WU>(c.s_row[q0 + q]);
    M lr[R][D];
    S mr[R][D];
#pragma unroll
    for (int h = 0; h < R; ++h) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            int uu = k[h] + (e[q] & 0xffff);
            uu = uu >= c.Z ? uu - c.Z : uu;
            const int idx = ((e[q] >> 16) & 0x1ff) * c.Z + uu;
            if (CACHE && (e[q] & kCached)) lr[h][q] = lds_read(c.s_post + idx);
            else lr[h][q] = ldc<COH>(&at(c.Lp, uint32_t(idx)));
        }
    }
    if (c.t > 0) {
#pragma unroll
        for (int h = 0; h < R; ++h) {
#pragma unroll
            for (int q = 0; q < D; ++q) mr[h][q] = ldc<COH>(&at(c.msg, uint32_t((q0 + q) * c.Z + k[h])));
        }
    } else {
#pragma unroll
        for (int h = 0; h < R; ++h) {
#pragma unroll
            for (int q = 0; q < D; ++q) mr[h][q] = S(0);      // c2v(0) = 0
        }
    }
    int bad = 0;
#pragma unroll
    for (int h = 0; h < R; ++h) {
        M x[D];
        int par = sraw[h] & 1;
        bool nan = false;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            par ^= (lr[h][q] < M(0)) ? 1 : 0;
            nan |= (lr[h][q] != lr[h][q]);
            x[q] = lr[h][q] - M(StoreT<S>::get(mr[h][q]));
        }
        if (c.t < c.T) {
            auto weight = [&](int q) -> M { return c.weighted ? M(c.s_w[(e[q] >> 25) & 0xf]) : M(c.alpha); };
            auto emit = [&](int q, M v) { at(c.msg, uint32_t((q0 + q) * c.Z + k[h])) = StoreT<S>::put(v); };
            check_rule<M, ALGO, D>(x, D, sraw[h] & 1, M(c.clamp), weight, emit);
        }
        bad += par | (nan ? 1 : 0);
    }
    return bad;
}

template <typename M, typename S, int ALGO, int D, bool WU, bool CACHE, bool COH = false>
__device__ __forceinline__ int check_row(const FrameCtx<M, S>& c, int q0, int k, int sraw)
{
    const int kk[1] = {k}, ss[1] = {sraw};
    return check_rows<M, S, ALGO, D, WU, CACHE, COH, 1>(c, q0, kk, ss);
}

// The same for any degree d <= MAXD (masked; entries may differ across lanes).
template <typename M, typename S, int ALGO, int MAXD, bool WU, bool CACHE, bool COH = false>
__device__ __forceinline__ int check_row_any(const FrameCtx<M, S>& c, int q0, int d, int k, int sraw)
{
    int32_t e[MAXD];
    M lr[MAXD];
    S mr[MAXD];
#pragma unroll
    for (int q = 0; q < MAXD; ++q) e[q] = (q < d) ? c.s_row[q0 + q] : 0;
#pragma unroll
    for (int q = 0; q < MAXD; ++q) {
        lr[q] = M(0);
        mr[q] = S(0);
        if (q < d) {
            const int eq = uni<WU>(e[q]);
            int uu = k + (eq & 0xffff);
            uu = uu >= c.Z ? uu - c.Z : uu;
            const int idx = ((eq >> 16) & 0x1ff) * c.Z + uu;
            if (CACHE && (eq & kCached)) lr[q] = lds_read(c.s_post + idx);
            else lr[q] = ldc<COH>(&at(c.Lp, uint32_t(idx)));
            if (c.t > 0) mr[q] = ldc<COH>(&at(c.msg, uint32_t((q0 + q) * c.Z + k)));
        }
    }
    M x[MAXD];
    int par = sraw & 1;
    bool nan = false;
#pragma unroll
    for (int q = 0; q < MAXD; ++q) {
        x[q] = M(0);
        if (q < d) {
            par ^= (lr[q] < M(0)) ? 1 : 0;
            nan |= (lr[q] != lr[q]);
            x[q] = lr[q] - M(StoreT<S>::get(opaque(mr[q])));
        }
    }
    if (c.t < c.T) {
        auto weight = [&](int q) -> M {
            return c.weighted ? M(c.s_w[uni<WU>((e[q] >> 25) & 0xf)]) : M(c.alpha);
        };
        auto emit = [&](int q, M v) { at(c.msg, uint32_t((q0 + q) * c.Z + k)) = StoreT<S>::put(v); };
        check_rule<M, ALGO, MAXD>(x, d, sraw & 1, M(c.clamp), weight, emit);
    }
    return par | (nan ? 1 : 0);
}

// Lch + the D messages of variables u[0..R) of the block column whose table
// entries start at qa, each summed in table order (block rows ascending); D
// wave-uniform; the R x D loads are issued before any sum.
template <typename M, typename S, int D, bool WU, bool COH, int R>
__device__ __forceinline__ void var_sums(const FrameCtx<M, S>& c, int qa, const int (&u)[R], M (&acc)[R])
{
    int32_t e[D];
    S m[R][D];
#pragma unroll
    for (int q = 0; q < D; ++q) e[q] = uni<WU>(c.s_col[qa + q]);
#pragma unroll
    for (int h = 0; h < R; ++h) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            int k = u[h] - (e[q] & 0xffff);
            k = k < 0 ? k + c.Z : k;
            m[h][q] = ldc<COH>(&at(c.msg, uint32_t((e[q] >> 16) * c.Z + k)));
        }
    }
#pragma unroll
    for (int h = 0; h < R; ++h) {
#pragma unroll
        for (int q = 0; q < D; ++q) acc[h] += M(StoreT<S>::get(m[h][q]));
    }
}

template <typename M, typename S, int D, bool WU, bool COH = false>
__device__ __forceinline__ M var_sum(const FrameCtx<M, S>& c, int qa, int u, M acc)
{
    const int uu[1] = {u};
    M a[1] = {acc};
    var_sums<M, S, D, WU, COH, 1>(c, qa, uu, a);
    return a[0];
}

// The same for any degree (8 loads at a time, masked).
template <typename M, typename S, bool WU, bool COH = false>
__device__ __forceinline__ M var_sum_any(const FrameCtx<M, S>& c, int qa, int dv, int u, M acc)
{
    for (int q8 = 0; q8 < dv; q8 += 8) {
        int32_t e[8];
        S m[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = (q8 + q < dv) ? c.s_col[qa + q8 + q] : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            m[q] = S(0);
            if (q8 + q < dv) {
                const int eq = uni<WU>(e[q]);
                int k = u - (eq & 0xffff);
                k = k < 0 ? k + c.Z : k;
                m[q] = ldc<COH>(&at(c.msg, uint32_t((eq >> 16) * c.Z + k)));
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q8 + q < dv) acc += M(StoreT<S>::get(opaque(m[q])));
    }
    return acc;
}

// ---------------------------------------------------------------------------
// frame groups: G workgroups resident on one XCD decode one frame together
// ---------------------------------------------------------------------------
// The group shares the XCD's L2, so its barrier is one L2 atomic per member
// and the loads of data that other members wrote are device-scope loads that
// read that L2 (ldc<true>); no cache is written back or invalidated.
constexpr int kXcds = 8;

struct GroupCtx {
    int member, G;
    uint64_t* word;         // arrivals (low half) and added counts (high half), both cumulative
    int32_t* err;           // set to 1 when a barrier wait gave up
    uint32_t gen;           // barriers passed so far
    uint32_t unsat_seen;    // high half at the last check-pass barrier
    uint64_t wait_ticks;    // bound of one wait, 100 MHz wall-clock ticks
};

constexpr uint64_t kGroupWaitTicks = 20000000ull;   // 0.2 s

// Barrier of the G workgroups of a group, which also sums `add` over them.
// Each wave first waits for its own stores to complete (they are then in the
// L2), the workgroup meets, and one thread adds (add << 32) + 1 to the group
// word and reads it until the arrivals of this generation are complete,
// bounded in wall-clock time (g.wait_ticks, 0.2 s by default; once a wait has
// given up no later one waits, so the launch always ends, and the frames are
// then reported as not decoded).  Returns the high half read then: every member's adds up to this
// barrier.  A member that has passed it can arrive at the next barrier first,
// so a barrier that follows one with adds must add 0.
__device__ __forceinline__ uint32_t group_sync(GroupCtx& g, uint32_t add = 0)
{
    __shared__ uint32_t s_hi;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(g.word, (uint64_t(add) << 32) | 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = (g.gen + 1u) * uint32_t(g.G);
        uint64_t v = __hip_atomic_load(g.word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (int32_t(uint32_t(v) - target) < 0 && __hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            const uint64_t t0 = wall_clock64();
            do {
                __builtin_amdgcn_s_sleep(1);
                v = __hip_atomic_load(g.word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (wall_clock64() - t0 > g.wait_ticks) {
                    atomicExch(g.err, 1);
                    break;
                }
            } while (int32_t(uint32_t(v) - target) < 0);
        }
        s_hi = uint32_t(v >> 32);
    }
    ++g.gen;
    __syncthreads();
    return s_hi;
}

// One frame, all iterations.  With WU every wavefront's rows (variables) share
// one block row (column), so the degree is wave-uniform and each step runs
// the straight-line body of its exact degree (1..8); larger degrees and
// codes with Z % 64 != 0 take the masked bodies.  The per-iteration min-sum
// weights are staged in LDS.
//
// GRP: the workgroup is member gc->member of a group of gc->G that decode the
// frame together (rows and variables interleaved by workgroup), with group
// barriers between the passes and the stop decision taken from the group's
// count; no posterior cache and no checkpoints.
template <typename M, typename S, int ALGO, int MAXD, int NT, bool WU, bool CACHE, bool GRP = false, bool PAIR = false>
__device__ __forceinline__ void decode_frame(const DecArgs& a, const LdsMap& lm, int32_t* dsm, int32_t (&s_unsat)[2],
                                             float (&s_w)[kMaxTypes], int f, const DevFrame& fr, const DevCode& cd,
                                             GroupCtx* gc = nullptr)
{
    static_assert(!(GRP && CACHE), "frame groups keep no posterior cache");
    const int tid = int(threadIdx.x);
    int first = tid, stride = NT;
    bool lead = true;                       // writes the frame's iteration count and status
    if constexpr (GRP) {
        first = gc->member * NT + tid;
        stride = gc->G * NT;
        lead = gc->member == 0;
    }
    auto sync = [&]() {
        if constexpr (GRP) group_sync(*gc);
        else __syncthreads();
    };
    const int Z = cd.Z;
    const int m = cd.mb * Z, n = cd.nb * Z;
    const int zsh = (Z & (Z - 1)) == 0 ? __ffs(Z) - 1 : -1;
    // group kernels, and the one-workgroup-per-CU shapes (PAIR), give each
    // thread R rows (variables) of one block row (column) per body,
    // k0 + h Z / R, so R times the loads are in flight: R = 2 at Z % 128 == 0,
    // and with PAIR R = 4 at Z % 256 == 0 (rows of at most 8 edges)
    constexpr bool kPairs = (GRP || PAIR) && WU && MAXD <= 8;
    const int rows_per_body = !kPairs ? 1 : (PAIR && Z % 256 == 0) ? 4 : (Z % 128 == 0 ? 2 : 1);
    const bool paired = rows_per_body > 1;
    const int32_t* s_rptr = dsm + lm.rptr;
    const int32_t* s_cptr = dsm + lm.cptr;
    FrameCtx<M, S> c;
    c.Lp = static_cast<M*>(a.post) + fr.vn_off;
    c.Lc = static_cast<const M*>(a.llr) + fr.vn_off;
    c.msg = static_cast<S*>(a.c2v) + fr.msg_off;
    c.s_row = dsm + lm.row;
    c.s_col = dsm + lm.col;
    c.s_cslot = dsm + lm.cslot;
    c.s_post = reinterpret_cast<M*>(dsm + lm.cache);
    c.s_w = s_w;
    c.Z = Z;
    c.T = a.T;
    c.weighted = a.weights != nullptr;
    c.alpha = a.alpha;
    c.clamp = a.clamp;
    const uint8_t* syn = a.syn ? a.syn + fr.chk_off : nullptr;
    M* tr = a.trace ? static_cast<M*>(a.trace) + fr.vn_off : nullptr;
    auto column = [&](int v) { return uni<WU>(zsh >= 0 ? (v >> zsh) : v / Z); };
    auto slot_of = [&](int j) { return CACHE ? uni<WU>(c.s_cslot[j]) : -1; };
    for (int v = first; v < n; v += stride) {
        const int j = column(v);
        const int slot = slot_of(j);
        const M l = at(c.Lc, v);
        if (slot >= 0) c.s_post[slot * Z + (v - j * Z)] = l;
        else at(c.Lp, v) = l;
        if (tr) tr[v] = l;
    }
    if (tid == 0) {
        s_unsat[0] = 0;
        s_unsat[1] = 0;
    }
    if (a.weights && a.T > 0 && tid < a.n_types) s_w[tid] = a.weights[tid];
    sync();
    for (int t = 0;; ++t) {
        c.t = t;
        if constexpr (!GRP) {
            if (a.ckpt && t < a.T && t % a.ckpt_every == 0) {
                // checkpoint c2v(t) (all zero at t = 0) before the check pass overwrites it
                float* ck = a.ckpt + int64_t(t / a.ckpt_every) * a.ckpt_stride + fr.msg_off;
                const int ef = cd.NB * Z;
                for (int e = tid; e < ef; e += NT) ck[e] = (t == 0) ? 0.0f : float(StoreT<S>::get(c.msg[e]));
                __syncthreads();
            }
        }
        // check pass: syndrome test of Lpost(t) and c2v(t+1)
        int bad = 0;
        if constexpr (kPairs) {
            // rows k0 + h Z / R, h < R, of a block row in one body
            auto check_multi = [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                const int qz = Z / R;
                const int qsh = zsh >= 0 ? zsh - (R == 4 ? 2 : 1) : -1;
                for (int p = first; p < m / R; p += stride) {
                    const int i = uni<WU>(qsh >= 0 ? (p >> qsh) : p / qz);
                    const int k0 = p - i * qz;
                    const int q0 = uni<WU>(s_rptr[i]);
                    const int d = uni<WU>(s_rptr[i + 1]) - q0;
                    int kk[R], ss[R];
#pragma unroll
                    for (int h = 0; h < R; ++h) {
                        kk[h] = k0 + h * qz;
                        ss[h] = syn ? int(at(syn, i * Z + kk[h])) : 0;
                    }
                    // wide rows take R = 4 as two bodies of 2 where the registers of
                    // four such rows would spill (measured: sum-product in the
                    // persistent kernel does better with all four at once)
                    constexpr int kSplitD = (ALGO == CVR_SP && !GRP) ? MAXD + 1 : 7;
                    auto body = [&](auto dc) {
                        constexpr int D = decltype(dc)::value;
                        if constexpr (R == 4 && D >= kSplitD) {
                            const int ka[2] = {kk[0], kk[1]}, sa[2] = {ss[0], ss[1]};
                            const int kb[2] = {kk[2], kk[3]}, sb[2] = {ss[2], ss[3]};
                            bad += check_rows<M, S, ALGO, D, WU, CACHE, GRP, 2>(c, q0, ka, sa);
                            bad += check_rows<M, S, ALGO, D, WU, CACHE, GRP, 2>(c, q0, kb, sb);
                        } else {
                            bad += check_rows<M, S, ALGO, D, WU, CACHE, GRP, R>(c, q0, kk, ss);
                        }
                    };
                    switch (d) {
                    case 1: body(std::integral_constant<int, 1>{}); break;
                    case 2: body(std::integral_constant<int, 2>{}); break;
                    case 3: body(std::integral_constant<int, 3>{}); break;
                    case 4: body(std::integral_constant<int, 4>{}); break;
                    case 5: body(std::integral_constant<int, 5>{}); break;
                    case 6: body(std::integral_constant<int, 6>{}); break;
                    case 7: body(std::integral_constant<int, 7>{}); break;
                    case 8: body(std::integral_constant<int, 8>{}); break;
                    default: break;
                    }
                }
            };
            if constexpr (PAIR) {
                if (rows_per_body == 4) check_multi(std::integral_constant<int, 4>{});
            }
            if (rows_per_body == 2) check_multi(std::integral_constant<int, 2>{});
        }
        for (int r = first; !paired && r < m; r += stride) {
            const int i = uni<WU>(zsh >= 0 ? (r >> zsh) : r / Z);
            const int k = r - i * Z;
            const int q0 = uni<WU>(s_rptr[i]);
            const int d = uni<WU>(s_rptr[i + 1]) - q0;
            const int sraw = syn ? int(at(syn, r)) : 0;
            if constexpr (WU) {
                switch (d) {
                case 1: bad += check_row<M, S, ALGO, 1, WU, CACHE, GRP>(c, q0, k, sraw); break;
                case 2: bad += check_row<M, S, ALGO, 2, WU, CACHE, GRP>(c, q0, k, sraw); break;
                case 3: bad += check_row<M, S, ALGO, 3, WU, CACHE, GRP>(c, q0, k, sraw); break;
                case 4: bad += check_row<M, S, ALGO, 4, WU, CACHE, GRP>(c, q0, k, sraw); break;
                case 5: bad += check_row<M, S, ALGO, 5, WU, CACHE, GRP>(c, q0, k, sraw); break;
                case 6: bad += check_row<M, S, ALGO, 6, WU, CACHE, GRP>(c, q0, k, sraw); break;
                case 7: bad += check_row<M, S, ALGO, 7, WU, CACHE, GRP>(c, q0, k, sraw); break;
                case 8: bad += check_row<M, S, ALGO, 8, WU, CACHE, GRP>(c, q0, k, sraw); break;
                default:
                    if constexpr (MAXD > 8) bad += check_row_any<M, S, ALGO, MAXD, WU, CACHE, GRP>(c, q0, d, k, sraw);
                    break;
                }
            } else {
                bad += check_row_any<M, S, ALGO, MAXD, WU, CACHE, GRP>(c, q0, d, k, sraw);
            }
        }
        if (bad) atomicAdd(&s_unsat[t & 1], bad);
        __syncthreads();
        int u = s_unsat[t & 1];
        if constexpr (GRP) {
            // the group's count: the barrier's sum since the previous check
            // pass (the barriers in between add nothing)
            const uint32_t hi = group_sync(*gc, uint32_t(u));
            u = int(hi - gc->unsat_seen);
            gc->unsat_seen = hi;
        }
        if ((a.early_stop && u == 0) || t >= a.T) {
            if (tid == 0 && lead) {
                a.iters[f] = t;
                a.ok[f] = uint8_t(u == 0);
            }
            break;
        }
        if (tid == 0) s_unsat[(t + 1) & 1] = 0;
        // the next iteration's weights: every read of s_w for iteration t
        // happened before the barrier above
        if (a.weights && t + 1 < a.T && tid < a.n_types) s_w[tid] = a.weights[int64_t(t + 1) * a.n_types + tid];
        // variable pass: Lpost(t+1) = Lch + sum of c2v(t+1) over block rows ascending
        if constexpr (kPairs) {
            // variables u0 + h Z / R, h < R, of a block column in one body
            auto var_multi = [&](auto rc) {
                constexpr int R = decltype(rc)::value;
                const int qz = Z / R;
                const int qsh = zsh >= 0 ? zsh - (R == 4 ? 2 : 1) : -1;
                for (int p = first; p < n / R; p += stride) {
                    const int j = uni<WU>(qsh >= 0 ? (p >> qsh) : p / qz);
                    const int u0 = p - j * qz;
                    const int qa = uni<WU>(s_cptr[j]);
                    const int dv = uni<WU>(s_cptr[j + 1]) - qa;
                    int uu[R];
                    M acc[R];
#pragma unroll
                    for (int h = 0; h < R; ++h) {
                        uu[h] = u0 + h * qz;
                        acc[h] = at(c.Lc, j * Z + uu[h]);
                    }
                    switch (dv) {
                    case 1: var_sums<M, S, 1, WU, GRP, R>(c, qa, uu, acc); break;
                    case 2: var_sums<M, S, 2, WU, GRP, R>(c, qa, uu, acc); break;
                    case 3: var_sums<M, S, 3, WU, GRP, R>(c, qa, uu, acc); break;
                    case 4: var_sums<M, S, 4, WU, GRP, R>(c, qa, uu, acc); break;
                    case 5: var_sums<M, S, 5, WU, GRP, R>(c, qa, uu, acc); break;
                    case 6: var_sums<M, S, 6, WU, GRP, R>(c, qa, uu, acc); break;
                    case 7: var_sums<M, S, 7, WU, GRP, R>(c, qa, uu, acc); break;
                    case 8: var_sums<M, S, 8, WU, GRP, R>(c, qa, uu, acc); break;
                    default:
                        for (int h = 0; h < R; ++h) acc[h] = var_sum_any<M, S, WU, GRP>(c, qa, dv, uu[h], acc[h]);
                        break;
                    }
                    const int slot = slot_of(j);
#pragma unroll
                    for (int h = 0; h < R; ++h) {
                        const int v = j * Z + uu[h];
                        if (slot >= 0) c.s_post[slot * Z + uu[h]] = acc[h];
                        else at(c.Lp, v) = acc[h];
                        if (tr) tr[int64_t(t + 1) * a.total_n + v] = acc[h];
                    }
                }
            };
            if constexpr (PAIR) {
                if (rows_per_body == 4) var_multi(std::integral_constant<int, 4>{});
            }
            if (rows_per_body == 2) var_multi(std::integral_constant<int, 2>{});
        }
        for (int v = first; !paired && v < n; v += stride) {
            const int j = column(v);
            const int uu = v - j * Z;
            const int qa = uni<WU>(s_cptr[j]);
            const int dv = uni<WU>(s_cptr[j + 1]) - qa;
            const int slot = slot_of(j);
            M acc = at(c.Lc, v);
            if constexpr (WU) {
                switch (dv) {
                case 1: acc = var_sum<M, S, 1, WU, GRP>(c, qa, uu, acc); break;
                case 2: acc = var_sum<M, S, 2, WU, GRP>(c, qa, uu, acc); break;
                case 3: acc = var_sum<M, S, 3, WU, GRP>(c, qa, uu, acc); break;
                case 4: acc = var_sum<M, S, 4, WU, GRP>(c, qa, uu, acc); break;
                case 5: acc = var_sum<M, S, 5, WU, GRP>(c, qa, uu, acc); break;
                case 6: acc = var_sum<M, S, 6, WU, GRP>(c, qa, uu, acc); break;
                case 7: acc = var_sum<M, S, 7, WU, GRP>(c, qa, uu, acc); break;
                case 8: acc = var_sum<M, S, 8, WU, GRP>(c, qa, uu, acc); break;
                default: acc = var_sum_any<M, S, WU, GRP>(c, qa, dv, uu, acc); break;
                }
            } else {
                acc = var_sum_any<M, S, WU, GRP>(c, qa, dv, uu, acc);
            }
            if (slot >= 0) c.s_post[slot * Z + uu] = acc;
            else at(c.Lp, v) = acc;
            if (tr) tr[int64_t(t + 1) * a.total_n + v] = acc;
        }
        sync();
    }
    // hard decisions; cached posteriors go back to HBM.  In a group the last
    // posteriors may come from another member (the paired bodies map threads
    // differently), so they are read past this CU's L1.
    for (int v = first; v < n; v += stride) {
        const int j = column(v);
        const int slot = slot_of(j);
        M l;
        if (slot >= 0) {
            l = c.s_post[slot * Z + (v - j * Z)];
            at(c.Lp, v) = l;
        } else {
            l = ldc<GRP>(&at(c.Lp, v));
        }
        a.bits[fr.vn_off + v] = l < M(0) ? 1 : 0;
    }
}

// Per-pass kernels on the packed global tables (QC codes with Z <= 65535):
// the tile's rows (variables) run the same exact-degree bodies as the
// persistent decoder.
template <typename M, typename S>
__device__ __forceinline__ FrameCtx<M, S> pass_ctx(const DecArgs& a, const DevFrame& fr, const DevCode& cd)
{
    FrameCtx<M, S> c;
    c.Lp = static_cast<M*>(a.post) + fr.vn_off;
    c.Lc = static_cast<const M*>(a.llr) + fr.vn_off;
    c.msg = static_cast<S*>(a.c2v) + fr.msg_off;
    c.s_row = cd.qrow_pk;
    c.s_col = cd.qcol_pk;
    c.s_cslot = nullptr;
    c.s_post = nullptr;
    c.s_w = a.weights ? a.weights + int64_t(a.t) * a.n_types : nullptr;
    c.Z = cd.Z;
    c.t = a.t;
    c.T = a.T;
    c.weighted = a.weights != nullptr;
    c.alpha = a.alpha;
    c.clamp = a.clamp;
    return c;
}

// The check step of tile tl (every thread of the workgroup calls it).
template <typename M, typename S, int ALGO, int MAXD, bool WU>
__device__ __forceinline__ void check_tile(const DecArgs& a, const Tile& tl)
{
    if (!a.active[tl.frame]) return;
    const DevFrame fr = a.frames[tl.frame];
    const DevCode& cd = a.codes[fr.code];
    const int count = tl.count & 0x7fffffff;
    const int i = tl.a;
    const int k = tl.b + int(threadIdx.x);
    const FrameCtx<M, S> c = pass_ctx<M, S>(a, fr, cd);
    const int q0 = uni<WU>(cd.qrow_ptr[i]);
    const int d = uni<WU>(cd.qrow_ptr[i + 1]) - q0;
    int bad = 0;
    if (int(threadIdx.x) < count) {
        const int sraw = a.syn ? int(a.syn[fr.chk_off + int64_t(i) * cd.Z + k]) : 0;
        if constexpr (WU) {
            switch (d) {
            case 1: bad = check_row<M, S, ALGO, 1, WU, false>(c, q0, k, sraw); break;
            case 2: bad = check_row<M, S, ALGO, 2, WU, false>(c, q0, k, sraw); break;
            case 3: bad = check_row<M, S, ALGO, 3, WU, false>(c, q0, k, sraw); break;
            case 4: bad = check_row<M, S, ALGO, 4, WU, false>(c, q0, k, sraw); break;
            case 5: bad = check_row<M, S, ALGO, 5, WU, false>(c, q0, k, sraw); break;
            case 6: bad = check_row<M, S, ALGO, 6, WU, false>(c, q0, k, sraw); break;
            case 7: bad = check_row<M, S, ALGO, 7, WU, false>(c, q0, k, sraw); break;
            case 8: bad = check_row<M, S, ALGO, 8, WU, false>(c, q0, k, sraw); break;
            default:
                if constexpr (MAXD > 8) bad = check_row_any<M, S, ALGO, MAXD, WU, false>(c, q0, d, k, sraw);
                break;
            }
        } else {
            bad = check_row_any<M, S, ALGO, MAXD, WU, false>(c, q0, d, k, sraw);
        }
    }
    add_unsat(&a.unsat[2 * tl.frame + (a.t & 1)], bad);
}

// The variable step of tile tl, after the frame's stop decision.
template <typename M, typename S, bool WU>
__device__ __forceinline__ void var_tile(const DecArgs& a, const Tile& tl)
{
    if (!a.active[tl.frame]) return;
    if (frame_stops(a, tl)) return;
    const DevFrame fr = a.frames[tl.frame];
    const DevCode& cd = a.codes[fr.code];
    const int count = tl.count & 0x7fffffff;
    if (int(threadIdx.x) >= count) return;
    const int j = tl.a;
    const int u = tl.b + int(threadIdx.x);
    const FrameCtx<M, S> c = pass_ctx<M, S>(a, fr, cd);
    const int qa = uni<WU>(cd.qcol_ptr[j]);
    const int dv = uni<WU>(cd.qcol_ptr[j + 1]) - qa;
    const int v = j * cd.Z + u;
    M acc = at(c.Lc, v);
    if constexpr (WU) {
        switch (dv) {
        case 1: acc = var_sum<M, S, 1, WU>(c, qa, u, acc); break;
        case 2: acc = var_sum<M, S, 2, WU>(c, qa, u, acc); break;
        case 3: acc = var_sum<M, S, 3, WU>(c, qa, u, acc); break;
        case 4: acc = var_sum<M, S, 4, WU>(c, qa, u, acc); break;
        case 5: acc = var_sum<M, S, 5, WU>(c, qa, u, acc); break;
        case 6: acc = var_sum<M, S, 6, WU>(c, qa, u, acc); break;
        case 7: acc = var_sum<M, S, 7, WU>(c, qa, u, acc); break;
        case 8: acc = var_sum<M, S, 8, WU>(c, qa, u, acc); break;
        default: acc = var_sum_any<M, S, WU>(c, qa, dv, u, acc); break;
        }
    } else {
        acc = var_sum_any<M, S, WU>(c, qa, dv, u, acc);
    }
    at(c.Lp, v) = acc;
    if (a.trace) static_cast<M*>(a.trace)[int64_t(a.t + 1) * a.total_n + fr.vn_off + v] = acc;
}

template <typename M, typename S, int ALGO, int MAXD, bool WU>
__global__ __launch_bounds__(kTile) void k_check_qc_pk(DecArgs a)
{
    check_tile<M, S, ALGO, MAXD, WU>(a, a.tiles[blockIdx.x]);
}

template <typename M, typename S, bool WU>
__global__ __launch_bounds__(kTile) void k_var_qc_pk(DecArgs a)
{
    var_tile<M, S, WU>(a, a.tiles[blockIdx.x]);
}

// Loads the LDS tables of code cd (see LdsMap) and assigns the posterior cache
// slots to its highest-degree block columns; every thread of the workgroup
// calls it, and it ends with a barrier.
template <typename M, int NT>
__device__ __forceinline__ void load_code_tables(const LdsMap& lm, int32_t* dsm, const DevCode& cd)
{
    const int tid = int(threadIdx.x);
    int32_t* s_rptr = dsm + lm.rptr;
    int32_t* s_cptr = dsm + lm.cptr;
    int32_t* s_row = dsm + lm.row;
    int32_t* s_col = dsm + lm.col;
    int32_t* s_cslot = dsm + lm.cslot;
    const int nslot = min(cd.nb, int(lm.cache_bytes / (int64_t(cd.Z) * int64_t(sizeof(M)))));
    for (int q = tid; q <= cd.mb; q += NT) s_rptr[q] = cd.qrow_ptr[q];
    for (int q = tid; q <= cd.nb; q += NT) s_cptr[q] = cd.qcol_ptr[q];
    for (int q = tid; q < cd.nb; q += NT) s_cslot[q] = -1;
    __syncthreads();
    for (int q = tid; q < nslot; q += NT) s_cslot[cd.qcol_rank[q]] = q;
    __syncthreads();
    for (int q = tid; q < cd.NB; q += NT) {
        const QcBlock br = cd.qrow[q];
        const int slot = s_cslot[br.other];
        const int loc = slot >= 0 ? slot : br.other;
        s_row[q] = br.shift | (loc << 16) | (br.type << 25) | (slot >= 0 ? kCached : 0);
        const QcBlock bc = cd.qcol[q];
        s_col[q] = bc.shift | (bc.blk << 16);
    }
    __syncthreads();
}

template <typename M, typename S, int ALGO, int MAXD, int NT, bool WU, int MINW, bool CACHE>
__global__ __launch_bounds__(NT, MINW) void k_frames_qc(DecArgs a, LdsMap lm, int32_t* queue, int32_t F,
                                                        const int32_t* order)
{
    extern __shared__ __align__(16) int32_t dsm[];
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
            load_code_tables<M, NT>(lm, dsm, cd);
            cur = fr.code;
        }
        // the 1024-thread shape without the 8-wave register bound (one
        // workgroup per CU, the most LDS for the posterior cache) runs the
        // paired bodies to keep as many loads in flight as two workgroups would
        decode_frame<M, S, ALGO, MAXD, NT, WU, CACHE, false, NT == 1024 && MINW == 1>(a, lm, dsm, s_unsat, s_w, f, fr, cd);
    }
}

// Frame groups.  A workgroup reads its XCD from the XCC_ID register and takes
// the next place of that XCD: places [g G, (g + 1) G) form group g.  Each
// group takes the XCD's frames (order[q * 8 + XCD], q = 0, 1, ...: largest
// first) from that XCD's queue and decodes them together; nothing depends on
// how the dispatcher numbers workgroups across XCDs.  The launch has as many
// workgroups per CU as the launch bounds guarantee resident (MINW waves per
// SIMD) and the same number of places per XCD.
// Group workspace, in 32-bit words:
//   [0] error flag (1: a barrier wait gave up; 2: an XCC_ID outside 0..7)
//   [4, 12) place tickets, [12, 20) frame queues, one per XCD
//   [64 + 64 g, ...) group g: barrier word (64 bits), [+ 4] frame; 256 bytes
//   apart, so groups never share a cache line (with two groups of 16 on an
//   XCD polling words in one line, a barrier took 3.3 us instead of 0.7 us)
constexpr int kGwErr = 0, kGwTicket = 4, kGwQueue = 12, kGwGroups = 64, kGwGroupWords = 64;
constexpr int kMaxGroups = 1024;
constexpr size_t kGroupWsBytes = size_t(kGwGroups + kMaxGroups * kGwGroupWords) * 4;

struct GroupArgs {
    const int32_t* order;     // [F] frames, largest first
    int32_t* ws;              // group workspace, zeroed by k_group_init
    int32_t F, G, NG;         // frames, workgroups per group, groups per XCD
    uint64_t wait_ticks;      // bound of one barrier wait
};

// The bound of a barrier wait for later launches (cvr_debug_group_wait_ticks).
uint64_t group_wait_ticks();

template <typename M, typename S, int ALGO, int MAXD, int NT, bool WU, int MINW>
__global__ __launch_bounds__(NT, MINW) void k_group_qc(DecArgs a, LdsMap lm, GroupArgs g)
{
    extern __shared__ __align__(16) int32_t dsm[];
    __shared__ int32_t s_place[2];
    __shared__ int32_t s_unsat[2];
    __shared__ float s_w[kMaxTypes];
    const int tid = int(threadIdx.x);
    int32_t* err = g.ws + kGwErr;
    if (tid == 0) {
        uint32_t xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
        int xcd = int(xcc & 0xf);
        if (xcd >= kXcds) {
            atomicExch(err, 2);
            xcd = 0;
        }
        s_place[0] = xcd;
        s_place[1] = atomicAdd(g.ws + kGwTicket + xcd, 1);
    }
    __syncthreads();
    const int xcd = s_place[0], place = s_place[1];
    const int gi = place / g.G;
    if (gi >= g.NG) return;                                  // a surplus place
    int32_t* gw = g.ws + kGwGroups + (xcd * g.NG + gi) * kGwGroupWords;
    GroupCtx gc{place % g.G, g.G, reinterpret_cast<uint64_t*>(gw), err, 0u, 0u, g.wait_ticks};
    int cur = -1;
    for (;;) {
        if (gc.member == 0 && tid == 0) {
            // every member read the previous frame's index before the barrier
            // that ended that frame
            const int q = atomicAdd(g.ws + kGwQueue + xcd, 1);
            const int64_t o = int64_t(q) * kXcds + xcd;
            const int f = o < g.F ? g.order[o] : g.F;
            __hip_atomic_store(gw + 4, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        group_sync(gc);
        const int f = __builtin_amdgcn_readfirstlane(ldc<true>(gw + 4));
        if (f >= g.F) break;
        const DevFrame fr = a.frames[f];
        const DevCode& cd = a.codes[fr.code];
        if (fr.code != cur) {
            load_code_tables<M, NT>(lm, dsm, cd);
            cur = fr.code;
        }
        decode_frame<M, S, ALGO, MAXD, NT, WU, false, true, NT == 1024 && MINW == 1>(a, lm, dsm, s_unsat, s_w, f, fr, cd, &gc);
        group_sync(gc);
    }
}

[[maybe_unused]] __global__ __launch_bounds__(256) static void k_group_init(int32_t* ws, int32_t words)
{
    for (int q = int(threadIdx.x); q < words; q += 256) ws[q] = 0;
}

// A barrier that gave up leaves the frames' results unreliable: every frame
// of the decode is reported as abandoned, iters = -1 and ok = 0, which a
// caller tells apart from a decoding failure (iters >= 0, ok = 0).
[[maybe_unused]] __global__ __launch_bounds__(256) static void k_group_final(uint8_t* ok, int32_t* iters,
                                                                             const int32_t* ws, int32_t F)
{
    const int f = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (f < F && ws[kGwErr]) {
        ok[f] = 0;
        iters[f] = -1;
    }
}

// ---------------------------------------------------------------------------
// layered (row-serial) schedule for quasi-cyclic codes, one workgroup per frame
// ---------------------------------------------------------------------------
// Layer i is block row i: its Z checks touch every block column at most once
// (one circulant per protograph entry), so they share no variable and update
// in parallel.  Iteration t runs the layers i = 0 .. mb-1 in order; for row k
// of layer i and its edge q at variable v = j_q Z + (k + s_q) mod Z:
//     x_q   = L[v] - c2v_q          (c2v_q from iteration t-1; 0 at t = 0)
//     c2v_q = the check rule over x (weights of iteration t), stored
//     L[v]  = x_q + c2v_q           (the stored value, as it will be read back)
// L is the running posterior (L_ch before the first iteration), so a layer
// sees every update of the layers before it in the same iteration.  The
// syndrome of the hard decisions of L is tested before the first iteration
// and after each one.
//
// State: c2v in HBM in the flooding layout ([block][k]); L in LDS for the
// cached (highest-degree) block columns and in the frame's posterior array
// otherwise; the hard decisions as a bit array in LDS (bit j Z + p for
// variable p of block column j), kept equal to [L < 0] by flipping a bit
// whenever an update changes the sign; a flag that any posterior is NaN (a
// NaN posterior stays NaN: x = NaN - c and L = NaN + c), which makes the
// syndrome test fail as a NaN does in the flooding schedule.
//
// Dynamic LDS (LdsMap, 32-bit words): rptr [mb+1], cptr [nb+1] (unused),
// row [NB] (shift | loc << 16 | type << 25 | cached << 29, as the persistent
// decoder's), col [NB] (block column of row entry q), cslot [nb], hard
// [n / 32], then the posterior cache.
// Consecutive block rows that share no block column update disjoint
// variables, so their rows can run in one step between two barriers with
// results identical to updating them one after another.  Layer groups:
// greedy runs of up to kGroupRows consecutive block rows with pairwise
// disjoint columns (when Z % 64 != 0 a wavefront's rows span block rows and
// take the masked body).  s_grp[0..ng] holds the first block row of each group
// and mb; s_grp[kMaxLdsDim + 1] holds ng.
constexpr int kGroupRows = 8;

template <typename M, int NT>
__device__ __forceinline__ void load_layer_tables(const LdsMap& lm, int32_t* dsm, const DevCode& cd)
{
    const int tid = int(threadIdx.x);
    int32_t* s_rptr = dsm + lm.rptr;
    int32_t* s_row = dsm + lm.row;
    int32_t* s_lcol = dsm + lm.col;
    int32_t* s_cslot = dsm + lm.cslot;
    int32_t* s_grp = dsm + lm.grp;
    const int nslot = min(cd.nb, int(lm.cache_bytes / (int64_t(cd.Z) * int64_t(sizeof(M)))));
    for (int q = tid; q <= cd.mb; q += NT) s_rptr[q] = cd.qrow_ptr[q];
    for (int q = tid; q < cd.nb; q += NT) s_cslot[q] = -1;
    for (int q = tid; q < cd.NB; q += NT) s_lcol[q] = cd.qrow[q].other;
    __syncthreads();
    for (int q = tid; q < nslot; q += NT) s_cslot[cd.qcol_rank[q]] = q;
    __syncthreads();
    for (int q = tid; q < cd.NB; q += NT) {
        const QcBlock br = cd.qrow[q];
        const int slot = s_cslot[br.other];
        const int loc = slot >= 0 ? slot : br.other;
        s_row[q] = br.shift | (loc << 16) | (br.type << 25) | (slot >= 0 ? kCached : 0);
    }
    if (tid == 0) {
        const int cap = kGroupRows;
        int ng = 0, first = 0;
        for (int i = 1; i <= cd.mb; ++i) {
            bool split = i == cd.mb || i - first >= cap;
            for (int q = s_rptr[i]; !split && q < s_rptr[i + 1]; ++q)
                for (int qp = s_rptr[first]; qp < s_rptr[i]; ++qp) split |= s_lcol[qp] == s_lcol[q];
            if (split) {
                s_grp[ng++] = first;
                first = i;
            }
        }
        s_grp[ng] = cd.mb;
        s_grp[kMaxLdsDim + 1] = ng;
    }
    __syncthreads();
}

// What the layer steps of one frame need beyond FrameCtx.
struct LayerCtx {
    const int32_t* s_lcol;
    uint32_t* s_hard;
    int32_t* s_nan;
};

// The update of rows k[0..R) of the layer whose table entries start at q0,
// with exactly D edges, from their loaded posteriors lr and stored messages
// mr: x = L - c2v, the check rule, c2v and L written back, decision bits
// flipped where the sign changed.
template <typename M, typename S, int ALGO, int D, bool CACHE, int R>
__device__ __forceinline__ void layer_update(const FrameCtx<M, S>& c, const LayerCtx& lc, int q0, const int (&k)[R],
                                             const int (&sraw)[R], const int32_t (&e)[D], const int32_t (&jc)[D],
                                             const int (&idx)[R][D], const M (&lr)[R][D], const S (&mr)[R][D])
{
    bool nan = false;
#pragma unroll
    for (int h = 0; h < R; ++h) {
        M x[D], nl[D];
#pragma unroll
        for (int q = 0; q < D; ++q) x[q] = lr[h][q] - M(StoreT<S>::get(mr[h][q]));
        auto weight = [&](int q) -> M { return c.weighted ? M(c.s_w[(e[q] >> 25) & 0xf]) : M(c.alpha); };
        auto emit = [&](int q, M v) {
            const S sv = StoreT<S>::put(v);
            at(c.msg, uint32_t((q0 + q) * c.Z + k[h])) = sv;
            nl[q] = x[q] + M(StoreT<S>::get(sv));
        };
        check_rule<M, ALGO, D>(x, D, sraw[h] & 1, M(c.clamp), weight, emit);
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const int at_loc = ((e[q] >> 16) & 0x1ff) * c.Z + idx[h][q];
            if (CACHE && (e[q] & kCached)) c.s_post[at_loc] = nl[q];
            else at(c.Lp, uint32_t(at_loc)) = nl[q];
            nan |= nl[q] != nl[q];
            if ((lr[h][q] < M(0)) != (nl[q] < M(0))) {
                const uint32_t b = uint32_t(jc[q] * c.Z + idx[h][q]);
                atomicXor(lc.s_hard + (b >> 5), 1u << (b & 31));
            }
        }
    }
    if (nan) *lc.s_nan = 1;
}

// Rows k[0..R) of the layer whose table entries start at q0, with exactly D
// edges: all R x D posteriors and stored messages are loaded before any
// arithmetic, then each row is updated and written back.
template <typename M, typename S, int ALGO, int D, bool CACHE, int R>
__device__ __forceinline__ void layer_rows(const FrameCtx<M, S>& c, const LayerCtx& lc, int q0, const int (&k)[R],
                                           const int (&sraw)[R])
{
    int32_t e[D], jc[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        e[q] = __builtin_amdgcn_readfirstlane(c.s_row[q0 + q]);
        jc[q] = __builtin_amdgcn_readfirstlane(lc.s_lcol[q0 + q]);
    }
    int idx[R][D];
    M lr[R][D];
    S mr[R][D];
#pragma unroll
    for (int h = 0; h < R; ++h) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            int p = k[h] + (e[q] & 0xffff);
            p = p >= c.Z ? p - c.Z : p;
            idx[h][q] = p;
            const int at_loc = ((e[q] >> 16) & 0x1ff) * c.Z + p;
            if (CACHE && (e[q] & kCached)) lr[h][q] = lds_read(c.s_post + at_loc);
            else lr[h][q] = at(c.Lp, uint32_t(at_loc));
        }
    }
    if (c.t > 0) {
#pragma unroll
        for (int h = 0; h < R; ++h) {
#pragma unroll
            for (int q = 0; q < D; ++q) mr[h][q] = at(c.msg, uint32_t((q0 + q) * c.Z + k[h]));
        }
    } else {
#pragma unroll
        for (int h = 0; h < R; ++h) {
#pragma unroll
            for (int q = 0; q < D; ++q) mr[h][q] = S(0);
        }
    }
    layer_update<M, S, ALGO, D, CACHE, R>(c, lc, q0, k, sraw, e, jc, idx, lr, mr);
}

// The same for any degree d <= MAXD (one row, masked).  With WU the block row
// (q0, d) is wave-uniform; without, each lane reads its own table entries.
template <typename M, typename S, int ALGO, int MAXD, bool CACHE, bool WU = true>
__device__ __forceinline__ void layer_row_any(const FrameCtx<M, S>& c, const LayerCtx& lc, int q0, int d, int k,
                                              int sraw)
{
    int32_t e[MAXD], jc[MAXD], idx[MAXD];
    M lr[MAXD], x[MAXD], nl[MAXD];
    S mr[MAXD];
#pragma unroll
    for (int q = 0; q < MAXD; ++q) {
        e[q] = (q < d) ? uni<WU>(c.s_row[q0 + q]) : 0;
        jc[q] = (q < d) ? uni<WU>(lc.s_lcol[q0 + q]) : 0;
        lr[q] = M(0);
        mr[q] = S(0);
        idx[q] = 0;
        nl[q] = M(0);
        if (q < d) {
            int p = k + (e[q] & 0xffff);
            p = p >= c.Z ? p - c.Z : p;
            idx[q] = p;
            const int at_loc = ((e[q] >> 16) & 0x1ff) * c.Z + p;
            if (CACHE && (e[q] & kCached)) lr[q] = lds_read(c.s_post + at_loc);
            else lr[q] = at(c.Lp, uint32_t(at_loc));
            if (c.t > 0) mr[q] = at(c.msg, uint32_t((q0 + q) * c.Z + k));
        }
    }
#pragma unroll
    for (int q = 0; q < MAXD; ++q) x[q] = (q < d) ? lr[q] - M(StoreT<S>::get(opaque(mr[q]))) : M(0);
    auto weight = [&](int q) -> M { return c.weighted ? M(c.s_w[(e[q] >> 25) & 0xf]) : M(c.alpha); };
    auto emit = [&](int q, M v) {
        const S sv = StoreT<S>::put(v);
        at(c.msg, uint32_t((q0 + q) * c.Z + k)) = sv;
        nl[q] = x[q] + M(StoreT<S>::get(sv));
    };
    check_rule<M, ALGO, MAXD>(x, d, sraw & 1, M(c.clamp), weight, emit);
    bool nan = false;
#pragma unroll
    for (int q = 0; q < MAXD; ++q) {
        if (q < d) {
            const int at_loc = ((e[q] >> 16) & 0x1ff) * c.Z + idx[q];
            if (CACHE && (e[q] & kCached)) c.s_post[at_loc] = nl[q];
            else at(c.Lp, uint32_t(at_loc)) = nl[q];
            nan |= nl[q] != nl[q];
            if ((lr[q] < M(0)) != (nl[q] < M(0))) {
                const uint32_t b = uint32_t(jc[q] * c.Z + idx[q]);
                atomicXor(lc.s_hard + (b >> 5), 1u << (b & 31));
            }
        }
    }
    if (nan) *lc.s_nan = 1;
}

// Rows k[0..R) of one block row with d edges: the exact-degree body.
template <typename M, typename S, int ALGO, int MAXD, bool CACHE, int R>
__device__ __forceinline__ void layer_rows_d(const FrameCtx<M, S>& c, const LayerCtx& lc, int q0, int d,
                                             const int (&k)[R], const int (&ss)[R])
{
    switch (d) {
    case 1: layer_rows<M, S, ALGO, 1, CACHE, R>(c, lc, q0, k, ss); break;
    case 2: layer_rows<M, S, ALGO, 2, CACHE, R>(c, lc, q0, k, ss); break;
    case 3: layer_rows<M, S, ALGO, 3, CACHE, R>(c, lc, q0, k, ss); break;
    case 4: layer_rows<M, S, ALGO, 4, CACHE, R>(c, lc, q0, k, ss); break;
    case 5: layer_rows<M, S, ALGO, 5, CACHE, R>(c, lc, q0, k, ss); break;
    case 6: layer_rows<M, S, ALGO, 6, CACHE, R>(c, lc, q0, k, ss); break;
    case 7: layer_rows<M, S, ALGO, 7, CACHE, R>(c, lc, q0, k, ss); break;
    case 8: layer_rows<M, S, ALGO, 8, CACHE, R>(c, lc, q0, k, ss); break;
    default:
        if constexpr (MAXD > 8) {
#pragma unroll
            for (int h = 0; h < R; ++h) layer_row_any<M, S, ALGO, MAXD, CACHE>(c, lc, q0, d, k[h], ss[h]);
        }
        break;
    }
}

// One frame, all iterations, on the layered schedule.  SYNL: Bob's syndrome
// bits in LDS (else in the workspace, when LDS is short).
template <typename M, typename S, int ALGO, int MAXD, int NT, bool SYNL>
__device__ __forceinline__ void decode_frame_layered(const DecArgs& a, const LdsMap& lm, int32_t* dsm,
                                                     int32_t (&s_unsat)[2], int32_t& s_nan, float (&s_w)[kMaxTypes],
                                                     int f, const DevFrame& fr, const DevCode& cd)
{
    constexpr bool CACHE = true;
    const int tid = int(threadIdx.x);
    const int Z = cd.Z;
    const int m = cd.mb * Z, n = cd.nb * Z;
    const int zsh = (Z & (Z - 1)) == 0 ? __ffs(Z) - 1 : -1;
    const int32_t* s_rptr = dsm + lm.rptr;
    FrameCtx<M, S> c;
    c.Lp = static_cast<M*>(a.post) + fr.vn_off;
    c.Lc = static_cast<const M*>(a.llr) + fr.vn_off;
    c.msg = static_cast<S*>(a.c2v) + fr.msg_off;
    c.s_row = dsm + lm.row;
    c.s_col = nullptr;
    c.s_cslot = dsm + lm.cslot;
    c.s_post = reinterpret_cast<M*>(dsm + lm.cache);
    c.s_w = s_w;
    c.Z = Z;
    c.T = a.T;
    c.weighted = a.weights != nullptr;
    c.alpha = a.alpha;
    c.clamp = a.clamp;
    LayerCtx lc{dsm + lm.col, reinterpret_cast<uint32_t*>(dsm + lm.hard), &s_nan};
    // Bob's syndrome bits: in LDS, or in the workspace when LDS is short
    uint32_t* s_synb = SYNL ? reinterpret_cast<uint32_t*>(dsm + lm.synb) : a.synw + ((fr.chk_off >> 5) + f);
    auto syn_word = [&](int w) -> uint32_t {
        if constexpr (SYNL) return lds_read(s_synb + w);
        else return *(const __attribute__((address_space(1))) uint32_t*)(s_synb + w);
    };
    const uint8_t* syn = a.syn ? a.syn + fr.chk_off : nullptr;
    M* tr = a.trace ? static_cast<M*>(a.trace) + fr.vn_off : nullptr;
    auto column = [&](int v) { return zsh >= 0 ? (v >> zsh) : v / Z; };
    auto slot_of = [&](int j) { return CACHE ? c.s_cslot[j] : -1; };
    auto post_at = [&](int v) -> M {
        const int j = column(v);
        const int slot = slot_of(j);
        return slot >= 0 ? c.s_post[slot * Z + (v - j * Z)] : at(c.Lp, v);
    };
    auto syn_bit = [&](int r) -> int { return int(syn_word(r >> 5) >> (r & 31)) & 1; };
    for (int w = tid; w < (n + 31) / 32; w += NT) lc.s_hard[w] = 0u;
    // Bob's syndrome of the frame as a bit array (read once)
    for (int w = tid; w < (m + 31) / 32; w += NT) {
        uint32_t bits = 0u;
        if (syn) {
            const int r0 = w * 32;
            for (int b = 0; b < 32 && r0 + b < m; ++b) bits |= uint32_t(at(syn, r0 + b) & 1) << b;
        }
        s_synb[w] = bits;
    }
    if (tid == 0) {
        s_unsat[0] = 0;
        s_unsat[1] = 0;
        s_nan = 0;
    }
    __syncthreads();
    for (int v = tid; v < n; v += NT) {
        const int j = column(v);
        const int slot = slot_of(j);
        const M l = at(c.Lc, v);
        if (slot >= 0) c.s_post[slot * Z + (v - j * Z)] = l;
        else at(c.Lp, v) = l;
        if (tr) tr[v] = l;
        if (l < M(0)) atomicOr(lc.s_hard + (v >> 5), 1u << (v & 31));
        if (l != l) s_nan = 1;
    }
    const int32_t* s_grp = dsm + lm.grp;
    const int ng = s_grp[kMaxLdsDim + 1];
    for (int t = 0;; ++t) {
        c.t = t;
        // the weights of iteration t (every read of the previous ones ended at
        // the barrier after the last layer)
        if (a.weights && t < a.T && tid < a.n_types) s_w[tid] = a.weights[int64_t(t) * a.n_types + tid];
        __syncthreads();
        // syndrome test of the hard decisions of L
        int bad = 0;
        if (Z % 32 == 0) {
            // 32 rows k0 .. k0 + 31 of a block row per thread: an edge with
            // shift s reads the decision bits of variables k0 + s .. k0 + s + 31
            // (mod Z) of its column as one rotated 32-bit window
            const int W = Z >> 5;
            for (int u = tid; u < (m >> 5); u += NT) {
                const int i = zsh >= 0 ? (u >> (zsh - 5)) : u / W;
                const int k0 = (u - i * W) << 5;
                const int q1 = s_rptr[i + 1];
                uint32_t par = syn_word(u);
                for (int q = s_rptr[i]; q < q1; ++q) {
                    int st = k0 + (c.s_row[q] & 0xffff);
                    st = st >= Z ? st - Z : st;
                    const uint32_t* colw = lc.s_hard + lc.s_lcol[q] * W;
                    const int w = st >> 5, off = st & 31;
                    const uint32_t lo = colw[w];
                    const uint32_t hi = colw[w + 1 == W ? 0 : w + 1];
                    par ^= off ? (lo >> off) | (hi << (32 - off)) : lo;
                }
                bad += __popc(par);
            }
        } else {
            for (int r = tid; r < m; r += NT) {
                const int i = zsh >= 0 ? (r >> zsh) : r / Z;
                const int k = r - i * Z;
                const int q1 = s_rptr[i + 1];
                int par = syn_bit(r);
                for (int q = s_rptr[i]; q < q1; ++q) {
                    int p = k + (c.s_row[q] & 0xffff);
                    p = p >= Z ? p - Z : p;
                    const uint32_t b = uint32_t(lc.s_lcol[q] * Z + p);
                    par ^= int(lc.s_hard[b >> 5] >> (b & 31)) & 1;
                }
                bad += par;
            }
        }
        if (bad) atomicAdd(&s_unsat[t & 1], bad);
        __syncthreads();
        const int u = s_unsat[t & 1] + (s_nan ? 1 : 0);
        if ((a.early_stop && u == 0) || t >= a.T) {
            if (tid == 0) {
                a.iters[f] = t;
                a.ok[f] = uint8_t(u == 0);
            }
            break;
        }
        if (tid == 0) s_unsat[(t + 1) & 1] = 0;
        // the layer groups in order; the rows of a group in one step
        for (int g = 0; g < ng; ++g) {
            const int i0 = s_grp[g];
            const int rows = (s_grp[g + 1] - i0) * Z;
            for (int r = tid; r < rows; r += NT) {
                const int di = zsh >= 0 ? (r >> zsh) : r / Z;
                const int k = r - di * Z;
                const int i = i0 + di;
                if (Z % 64 == 0) {
                    // a wavefront's 64 rows lie in one block row: exact-degree bodies
                    const int q0 = __builtin_amdgcn_readfirstlane(s_rptr[i]);
                    const int d = __builtin_amdgcn_readfirstlane(s_rptr[i + 1]) - q0;
                    const int kk[1] = {k}, ss[1] = {syn_bit(i * Z + k)};
                    layer_rows_d<M, S, ALGO, MAXD, CACHE, 1>(c, lc, q0, d, kk, ss);
                } else {
                    // a wavefront spans block rows: the masked body, per-lane tables
                    const int q0 = s_rptr[i];
                    layer_row_any<M, S, ALGO, MAXD, CACHE, false>(c, lc, q0, s_rptr[i + 1] - q0, k, syn_bit(i * Z + k));
                }
            }
            __syncthreads();
        }
        if (tr)
            for (int v = tid; v < n; v += NT) tr[int64_t(t + 1) * a.total_n + v] = post_at(v);
    }
    // hard decisions; cached posteriors go back to HBM
    for (int v = tid; v < n; v += NT) {
        const int j = column(v);
        const int slot = slot_of(j);
        M l;
        if (slot >= 0) {
            l = c.s_post[slot * Z + (v - j * Z)];
            at(c.Lp, v) = l;
        } else {
            l = at(c.Lp, v);
        }
        a.bits[fr.vn_off + v] = l < M(0) ? 1 : 0;
    }
}

template <typename M, typename S, int ALGO, int MAXD, int NT, bool SYNL>
__global__ __launch_bounds__(NT, MAXD <= 8 ? 4 : 1) void k_layered_qc(DecArgs a, LdsMap lm, int32_t* queue, int32_t F,
                                                   const int32_t* order)
{
    extern __shared__ __align__(16) int32_t dsm[];
    __shared__ int32_t s_frame;
    __shared__ int32_t s_unsat[2];
    __shared__ int32_t s_nan;
    __shared__ float s_w[kMaxTypes];
    const int tid = int(threadIdx.x);
    int cur = -1;
    for (;;) {
        if (tid == 0) {
            const int slot = atomicAdd(queue, 1);
            s_frame = slot < F ? order[slot] : F;
        }
        __syncthreads();
        const int f = __builtin_amdgcn_readfirstlane(s_frame);
        if (f >= F) break;
        const DevFrame fr = a.frames[f];
        const DevCode& cd = a.codes[fr.code];
        if (fr.code != cur) {
            load_layer_tables<M, NT>(lm, dsm, cd);
            cur = fr.code;
        }
        decode_frame_layered<M, S, ALGO, MAXD, NT, SYNL>(a, lm, dsm, s_unsat, s_nan, s_w, f, fr, cd);
        __syncthreads();
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
// Every code of the batch has Z % 64 == 0: each wavefront stays inside one
// block row / column, and the wave-uniform kernel applies.
static inline bool wave_uniform(const cvr_batch_s* b)
{
    for (const cvr_code_t c : b->codes)
        if (c->dev.Z % 64) return false;
    return true;
}

template <typename M, typename S, int ALGO, int MAXD>
static cvr_status run_decode(const cvr_batch_s* b, DecArgs a, hipStream_t s, bool qc)
{
    const int64_t nvt = b->n_vn_tiles;
    bool packed = qc;
    for (const cvr_code_t c : b->codes) packed = packed && c->dev.qrow_pk && c->dev.qcol_pk;
    const bool wu = packed && wave_uniform(b);
    a.tiles = b->d_vn_tiles;
    {
        ProfScope prof(CVR_PROF_DEC_SETUP, s);
        hipLaunchKernelGGL(k_dec_init<M>, dim3(nvt), dim3(kTile), 0, s, a);
    }
    if (cvr_status st = check_launch("decode init")) return st;
    for (int t = 0; t <= a.T; ++t) {
        a.t = t;
        if (qc && packed) {
            a.tiles = b->d_qcn_tiles;
            {
                ProfScope prof(CVR_PROF_CHECK, s);
                if (wu) hipLaunchKernelGGL((k_check_qc_pk<M, S, ALGO, MAXD, true>), dim3(b->n_qcn_tiles), dim3(kTile), 0, s, a);
                else hipLaunchKernelGGL((k_check_qc_pk<M, S, ALGO, MAXD, false>), dim3(b->n_qcn_tiles), dim3(kTile), 0, s, a);
            }
            a.tiles = b->d_qvn_tiles;
            {
                ProfScope prof(CVR_PROF_VAR, s);
                if (wu) hipLaunchKernelGGL((k_var_qc_pk<M, S, true>), dim3(b->n_qvn_tiles), dim3(kTile), 0, s, a);
                else hipLaunchKernelGGL((k_var_qc_pk<M, S, false>), dim3(b->n_qvn_tiles), dim3(kTile), 0, s, a);
            }
        } else if (qc) {
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

static inline int device_attr(hipDeviceAttribute_t attr, int fallback)
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, attr, dev) == hipSuccess && v > 0) return v;
    return fallback;
}

// LDS map of a batch: the tables of its largest code, then the posterior cache.
static inline LdsMap lds_map(const cvr_batch_s* b, int cache_bytes)
{
    LdsMap lm{};
    lm.rptr = 0;
    lm.cptr = lm.rptr + b->max_mb + 1;
    lm.row = lm.cptr + b->max_nb + 1;
    lm.col = lm.row + b->max_NB;
    lm.cslot = lm.col + b->max_NB;
    lm.cache = (lm.cslot + b->max_nb + 3) / 4 * 4;     // 16-byte aligned
    lm.cache_bytes = cache_bytes;
    return lm;
}

// lds_kb < 0: no posterior cache; 0: the largest cache that keeps the
// register-limited number of resident workgroups per CU; > 0: that many KiB
// (occupancy follows).
template <typename M, typename S, int ALGO, int MAXD, int NT, bool WU, int MINW, bool CACHE>
static cvr_status launch_frames(const cvr_batch_s* b, DecArgs a, int32_t* queue, hipStream_t s, int lds_kb)
{
    auto kern = k_frames_qc<M, S, ALGO, MAXD, NT, WU, MINW, CACHE>;
    static int lds_blk = 0, lds_cu = 0, static_lds = 0;
    if (lds_blk == 0) {
        lds_cu = device_attr(hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, 65536);
        lds_blk = std::min(lds_cu, device_attr(hipDeviceAttributeMaxSharedMemoryPerBlock, 65536));
        hipFuncAttributes fa{};
        static_lds = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)) == hipSuccess
                         ? int(fa.sharedSizeBytes) : 1024;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  lds_blk - static_lds);
    }
    const int tab = lds_map(b, 0).cache * 4;
    const int room = lds_blk - static_lds - tab;
    if (room < 0) return fail(CVR_EUNSUPPORTED, "decode (persistent): code tables exceed LDS");
    auto occupancy = [&](int dyn) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, NT, size_t(dyn)) != hipSuccess || v < 1) v = 1;
        return v;
    };
    int cache = 0;
    if (!CACHE) {
        cache = 0;
    } else if (lds_kb > 0) {
        cache = std::min(room, lds_kb * 1024);
    } else if (lds_kb == 0) {
        const int want = occupancy(tab);                 // workgroups per CU without a cache
        cache = std::min(room, lds_cu / want - static_lds - tab - 512);
        while (cache > 0 && occupancy(tab + cache) < want) cache -= 2048;
    }
    cache = std::max(0, cache) / 256 * 256;
    const LdsMap lm = lds_map(b, cache);
    const int dyn = tab + cache;
    const int per_cu = occupancy(dyn);
    const int grid = int(std::min<int64_t>(b->F, int64_t(device_cus()) * per_cu));
    ProfScope prof(CVR_PROF_FRAMES, s);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), size_t(dyn), s, a, lm, queue, b->F, b->d_order);
    return check_launch("decode (persistent)");
}


template <typename M, typename S, int ALGO, int MAXD, bool CACHE>
static cvr_status run_shape(const cvr_batch_s* b, DecArgs a, int32_t* queue, hipStream_t s, const LaunchShape& sh)
{
    if (sh.min_waves == 8) {
        if (sh.wg == 1024) return launch_frames<M, S, ALGO, MAXD, 1024, true, 8, CACHE>(b, a, queue, s, sh.lds_kb);
        return launch_frames<M, S, ALGO, MAXD, 512, true, 8, CACHE>(b, a, queue, s, sh.lds_kb);
    }
    if (sh.wg == 1024) return launch_frames<M, S, ALGO, MAXD, 1024, true, 1, CACHE>(b, a, queue, s, sh.lds_kb);
    return launch_frames<M, S, ALGO, MAXD, 512, true, 1, CACHE>(b, a, queue, s, sh.lds_kb);
}

template <typename M, typename S, int ALGO, int MAXD>
static cvr_status run_frames(const cvr_batch_s* b, DecArgs a, int32_t* queue, hipStream_t s, const LaunchShape& sh)
{
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, s, queue, int64_t(1));
    if (cvr_status st = check_launch("decode queue reset")) return st;
    if (!wave_uniform(b)) return launch_frames<M, S, ALGO, MAXD, 512, false, 1, false>(b, a, queue, s, -1);
    if constexpr (MAXD > 8 || sizeof(M) == 8) {
        // binary64, and rows of more than 8 edges, need more registers than
        // the other shapes leave: 512 threads, no posterior cache
        return launch_frames<M, S, ALGO, MAXD, 512, true, 1, false>(b, a, queue, s, -1);
    } else {
        // the cache costs a wave-uniform branch per edge: separate kernels
        if (sh.lds_kb >= 0) return run_shape<M, S, ALGO, MAXD, true>(b, a, queue, s, sh);
        return run_shape<M, S, ALGO, MAXD, false>(b, a, queue, s, sh);
    }
}

// Group schedule (QC codes whose tables fit in LDS): the workgroups per CU
// that the launch bounds guarantee, G per frame (group_wgs, or as many as the
// frames per XCD leave), at most one group per frame of the XCD.
template <typename M, typename S, int ALGO, int MAXD, int NT, bool WU, int MINW>
static cvr_status launch_group(const cvr_batch_s* b, DecArgs a, hipStream_t s, int32_t* ws, int group_wgs)
{
    auto kern = k_group_qc<M, S, ALGO, MAXD, NT, WU, MINW>;
    static int lds_blk = 0, static_lds = 0;
    if (lds_blk == 0) {
        lds_blk = std::min(device_attr(hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, 65536),
                           device_attr(hipDeviceAttributeMaxSharedMemoryPerBlock, 65536));
        hipFuncAttributes fa{};
        static_lds = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)) == hipSuccess
                         ? int(fa.sharedSizeBytes) : 1024;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  lds_blk - static_lds);
    }
    const LdsMap lm = lds_map(b, 0);
    const int dyn = lm.cache * 4;
    if (dyn > lds_blk - static_lds) return fail(CVR_EUNSUPPORTED, "decode (group): code tables exceed LDS");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, size_t(dyn)) != hipSuccess || per_cu < 1)
        return fail(CVR_EUNSUPPORTED, "decode (group): a workgroup does not fit on a CU");
    // the runtime's count can exceed what fits (it does not see the scalar
    // register limit); the launch bounds guarantee MINW waves on each of the 4 SIMDs
    per_cu = std::min(per_cu, std::max(1, MINW * 4 * 64 / NT));
    const int cap = std::max(1, device_cus() / kXcds) * per_cu;  // places per XCD
    const int fx = (b->F + kXcds - 1) / kXcds;                   // frames per XCD
    const int G = group_wgs > 0 ? std::min(group_wgs, cap) : std::max(1, cap / std::min(fx, cap));
    const int NG = std::min(cap / G, fx);
    if (NG * kXcds > kMaxGroups) return fail(CVR_EUNSUPPORTED, "decode (group): too many groups");
    {
        ProfScope prof(CVR_PROF_DEC_SETUP, s);
        hipLaunchKernelGGL(k_group_init, dim3(1), dim3(256), 0, s, ws, int32_t(kGwGroups + NG * kXcds * kGwGroupWords));
    }
    if (cvr_status st = check_launch("decode (group) init")) return st;
    const GroupArgs g{b->d_order, ws, b->F, G, NG, group_wait_ticks()};
    {
        ProfScope prof(CVR_PROF_FRAMES, s);
        hipLaunchKernelGGL(kern, dim3(kXcds * NG * G), dim3(NT), size_t(dyn), s, a, lm, g);
    }
    if (cvr_status st = check_launch("decode (group)")) return st;
    {
        ProfScope prof(CVR_PROF_DEC_SETUP, s);
        hipLaunchKernelGGL(k_group_final, dim3((b->F + 255) / 256), dim3(256), 0, s, a.ok, a.iters, ws, b->F);
    }
    return check_launch("decode (group) final");
}

template <typename M, typename S, int ALGO, int MAXD>
static cvr_status run_group(const cvr_batch_s* b, DecArgs a, hipStream_t s, int32_t* ws, const LaunchShape& sh)
{
    const bool wu = wave_uniform(b);
    if constexpr (MAXD > 8 || sizeof(M) == 8) {
        if (wu) return launch_group<M, S, ALGO, MAXD, 512, true, 1>(b, a, s, ws, sh.group_wgs);
        return launch_group<M, S, ALGO, MAXD, 512, false, 1>(b, a, s, ws, sh.group_wgs);
    } else {
        if (!wu) return launch_group<M, S, ALGO, MAXD, 512, false, 1>(b, a, s, ws, sh.group_wgs);
        if (sh.min_waves == 8) return launch_group<M, S, ALGO, MAXD, 1024, true, 8>(b, a, s, ws, sh.group_wgs);
        return launch_group<M, S, ALGO, MAXD, 1024, true, 1>(b, a, s, ws, sh.group_wgs);
    }
}

// Layered schedule (QC codes whose tables fit in LDS): one workgroup per frame
// from the frame queue; NT threads (256, 512 or 1024); the LDS left after the
// tables and the decision bits (and the syndrome bits when they fit as well)
// caches posteriors (lds_kb as for the persistent decoder).
template <typename M, typename S, int ALGO, int MAXD, int NT, bool SYNL>
static cvr_status launch_layered_as(const cvr_batch_s* b, DecArgs a, int32_t* queue, hipStream_t s, int lds_kb,
                                    int64_t max_n, int64_t max_m)
{
    auto kern = k_layered_qc<M, S, ALGO, MAXD, NT, SYNL>;
    static int lds_blk = 0, lds_cu = 0, static_lds = 0;
    if (lds_blk == 0) {
        lds_cu = device_attr(hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, 65536);
        lds_blk = std::min(lds_cu, device_attr(hipDeviceAttributeMaxSharedMemoryPerBlock, 65536));
        hipFuncAttributes fa{};
        static_lds = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)) == hipSuccess
                         ? int(fa.sharedSizeBytes) : 1024;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  lds_blk - static_lds);
    }
    auto map = [&](int cache_bytes) {
        LdsMap lm = lds_map(b, cache_bytes);
        lm.hard = lm.cache;
        lm.synb = SYNL ? int32_t(lm.hard + (max_n + 31) / 32) : -1;
        lm.grp = int32_t(lm.hard + (max_n + 31) / 32 + (SYNL ? (max_m + 31) / 32 : 0));
        lm.cache = int32_t((lm.grp + kMaxLdsDim + 2 + 3) / 4 * 4);
        return lm;
    };
    const int tab = map(0).cache * 4;
    const int room = lds_blk - static_lds - tab;
    if (room < 0) {
        if constexpr (SYNL)   // the syndrome bits go to the workspace
            return launch_layered_as<M, S, ALGO, MAXD, NT, false>(b, a, queue, s, lds_kb, max_n, max_m);
        return fail(CVR_EUNSUPPORTED, "decode (layered): code tables and decision bits exceed LDS");
    }
    auto occupancy = [&](int dyn) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, NT, size_t(dyn)) != hipSuccess || v < 1) v = 1;
        return v;
    };
    int cache = 0;
    if (lds_kb > 0) {
        cache = std::min(room, lds_kb * 1024);
    } else if (lds_kb == 0) {
        const int want = occupancy(tab);
        cache = std::min(room, lds_cu / want - static_lds - tab - 512);
        while (cache > 0 && occupancy(tab + cache) < want) cache -= 2048;
    }
    cache = std::max(0, cache) / 256 * 256;
    const LdsMap lm = map(cache);
    const int dyn = tab + cache;
    const int per_cu = occupancy(dyn);
    const int grid = int(std::min<int64_t>(b->F, int64_t(device_cus()) * per_cu));
    ProfScope prof(CVR_PROF_FRAMES, s);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), size_t(dyn), s, a, lm, queue, b->F, b->d_order);
    return check_launch("decode (layered)");
}

template <typename M, typename S, int ALGO, int MAXD, int NT>
static cvr_status launch_layered(const cvr_batch_s* b, DecArgs a, int32_t* queue, hipStream_t s, int lds_kb)
{
    int64_t max_n = 0, max_m = 0;
    for (const cvr_code_t c : b->codes) {
        max_n = std::max<int64_t>(max_n, c->dev.n);
        max_m = std::max<int64_t>(max_m, int64_t(c->dev.mb) * c->dev.Z);
    }
    return launch_layered_as<M, S, ALGO, MAXD, NT, true>(b, a, queue, s, lds_kb, max_n, max_m);
}

template <typename M, typename S, int ALGO, int MAXD>
static cvr_status run_layered(const cvr_batch_s* b, DecArgs a, int32_t* queue, hipStream_t s, const LaunchShape& sh)
{
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, s, queue, int64_t(1));
    if (cvr_status st = check_launch("decode queue reset")) return st;
    if constexpr (sizeof(M) == 8 || MAXD > 8) {
        return launch_layered<M, S, ALGO, MAXD, 512>(b, a, queue, s, sh.lds_kb);
    } else {
        if (sh.wg == 256) return launch_layered<M, S, ALGO, MAXD, 256>(b, a, queue, s, sh.lds_kb);
        if (sh.wg == 1024) return launch_layered<M, S, ALGO, MAXD, 1024>(b, a, queue, s, sh.lds_kb);
        return launch_layered<M, S, ALGO, MAXD, 512>(b, a, queue, s, sh.lds_kb);
    }
}

// mode: 0 per-pass launches, 1 persistent frame-per-workgroup, 2 frame groups,
// 3 layered schedule (one workgroup per frame)
template <typename M, typename S, int ALGO>
static cvr_status dispatch_deg(const cvr_batch_s* b, DecArgs a, hipStream_t s, bool qc, int mode, int32_t* queue,
                               int32_t* gridws, const LaunchShape& sh)
{
    if (mode == 1) {
        if (b->max_row_deg <= 8) return run_frames<M, S, ALGO, 8>(b, a, queue, s, sh);
        if (b->max_row_deg <= 16) return run_frames<M, S, ALGO, 16>(b, a, queue, s, sh);
        return run_frames<M, S, ALGO, 32>(b, a, queue, s, sh);
    }
    if (mode == 3) {
        if (b->max_row_deg <= 8) return run_layered<M, S, ALGO, 8>(b, a, queue, s, sh);
        return run_layered<M, S, ALGO, 32>(b, a, queue, s, sh);
    }
    if (mode == 2) {
        if (b->max_row_deg <= 8) return run_group<M, S, ALGO, 8>(b, a, s, gridws, sh);
        if (b->max_row_deg <= 16) return run_group<M, S, ALGO, 16>(b, a, s, gridws, sh);
        return run_group<M, S, ALGO, 32>(b, a, s, gridws, sh);
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
    size_t c2v, post, active, unsat, queue, grid, synw, total;
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
    w.queue = off;              // persistent decoder's frame queue
    off = align256(off + 4);
    w.grid = off;               // group schedule: see k_group_qc
    off = align256(off + kGroupWsBytes);
    w.synw = off;               // layered schedule: syndrome bits of frames whose bits exceed LDS
    if (p->schedule == CVR_SCHED_LAYERED) off = align256(off + size_t((b->total_m + 31) / 32 + b->F + 1) * 4);
    w.total = off;
    return w;
}

// The persistent and group paths need a quasi-cyclic batch whose protograph tables fit in LDS.
static inline bool frames_fit(const cvr_batch_s* b)
{
    if (!b->all_qc) return false;
    for (const cvr_code_t c : b->codes)
        if (c->dev.NB > kMaxLdsBlocks || c->dev.mb > kMaxLdsDim || c->dev.nb > kMaxLdsDim || c->dev.Z > kMaxLdsZ)
            return false;
    return true;
}


// One instantiation per (math, store, rule); each lives in its own translation unit.
#define CVR_DECL_DISPATCH(NAME)                                                                      \
    cvr_status NAME(const cvr_batch_s* b, DecArgs a, hipStream_t s, bool qc, int mode, int32_t* queue, \
                    int32_t* gridws, const LaunchShape& sh)
CVR_DECL_DISPATCH(decode_f64_sp);
CVR_DECL_DISPATCH(decode_f64_nms);
CVR_DECL_DISPATCH(decode_f32_sp);
CVR_DECL_DISPATCH(decode_f32_nms);
CVR_DECL_DISPATCH(decode_f16_sp);
CVR_DECL_DISPATCH(decode_f16_nms);
}  // namespace cvr
