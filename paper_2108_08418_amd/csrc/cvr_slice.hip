// Bob's quantiser/slicer and Alice's slice LLRs (Sec. III-B steps 1, 2 and 4),
// with two other forms of Alice's soft information: lower slices entered as
// soft priors (the decoder's final LLRs, Sec. III-B step 4) and the hard
// binary-symmetric-channel LLR from her own quantised bits and the bit error
// ratio p_j of Sec. II Step 4.
//
// All kernels are streaming passes over the quadratures: one fp64 load per
// sample plus m_bits slice bytes (quantiser) or the known slice bytes, the
// prior rows and one output (LLR).  The thresholds travel by value in the
// kernel arguments.
#include "cvr_internal.h"

#include <cmath>

namespace cvr {

constexpr int kMaxThr = 255;

struct QuantArgs {
    const double* y;
    uint8_t* slices;
    int64_t n;
    int32_t m_bits;
    int32_t nthr;
    int32_t gray;
    int32_t vec;           // 1: n % 4 == 0 and y/slices aligned for the 4-wide path
    double t[kMaxThr];
};

struct LlrArgs {
    const double* x;
    const uint8_t* slices;
    void* out;
    int64_t n;
    double sigma;
    int32_t m_bits;
    int32_t nthr;
    int32_t gray;
    int32_t j;
    uint32_t known;
    int32_t out_f64;
    const float* prior;    // [m_bits][n]; rows in prior_mask read (prior form only)
    uint32_t prior_mask;
    void* next0;           // LLR of slice j+1 given bit j = 0 / 1 (next form only)
    void* next1;
    double t[kMaxThr];
};

struct ChooseArgs {
    const void* l0;
    const void* l1;
    const uint8_t* bits;
    void* out;
    int64_t n;
    int32_t f64;
};

struct BscArgs {
    const double* x;
    void* out;
    int64_t n;
    double p;
    int32_t nthr;
    int32_t gray;
    int32_t j;
    int32_t out_f64;
    double t[kMaxThr];
};

__device__ __forceinline__ int interval_label(const QuantArgs& a, double y)
{
    int k = 0;
    for (int q = 0; q < a.nthr; ++q) k += (a.t[q] <= y) ? 1 : 0;   // #{i : t_i <= y}
    return a.gray ? (k ^ (k >> 1)) : k;
}

// Four consecutive samples per thread: two 16-byte loads of y and one 4-byte
// store per slice row.
__global__ __launch_bounds__(256) void k_quantize(QuantArgs a)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x * 4;
    for (int64_t i0 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4; i0 < a.n; i0 += stride) {
        if (a.vec) {
            const double4 yv = *reinterpret_cast<const double4*>(a.y + i0);
            const int g0 = interval_label(a, yv.x), g1 = interval_label(a, yv.y);
            const int g2 = interval_label(a, yv.z), g3 = interval_label(a, yv.w);
            for (int j = 0; j < a.m_bits; ++j) {
                uint32_t w = uint32_t((g0 >> j) & 1) | (uint32_t((g1 >> j) & 1) << 8) |
                             (uint32_t((g2 >> j) & 1) << 16) | (uint32_t((g3 >> j) & 1) << 24);
                *reinterpret_cast<uint32_t*>(a.slices + int64_t(j) * a.n + i0) = w;
            }
        } else {
            for (int64_t i = i0; i < i0 + 4 && i < a.n; ++i) {
                const int g = interval_label(a, a.y[i]);
                for (int j = 0; j < a.m_bits; ++j) a.slices[int64_t(j) * a.n + i] = uint8_t((g >> j) & 1);
            }
        }
    }
}

// ln Q(z) for z >= 0 (z may be +inf), Q(z) = 1 - Phi(z) the normal upper tail,
// through the scaled complementary error function erfcx(w) = exp(w^2) erfc(w):
// ln Q(z) = ln(erfcx(z / sqrt 2) / 2) - z^2 / 2, finite far into the tail.
__device__ __forceinline__ double ln_q(double z)
{
    if (z == INFINITY) return -INFINITY;
    const double w = z * M_SQRT1_2;
    return log(0.5 * erfcx(w)) - w * w;
}

// ln Pr(lo <= Z < hi) for a standard normal Z and lo < hi (either may be
// infinite).  A lower-tail interval is mirrored onto the upper tail (same
// probability), so only two cases remain: both ends above the mean, where
// P = Q(lo) - Q(hi) = Q(lo) (1 - Q(hi)/Q(lo)), and an interval containing the
// mean, where P = 1 - Q(-lo) - Q(hi).  Both need ln Q at |lo| and hi only.
__device__ __forceinline__ double ln_interval(double lo, double hi)
{
    if (hi <= 0.0) {
        const double t = lo;
        lo = -hi;
        hi = -t;
    }
    const double A = ln_q(fabs(lo));
    const double B = ln_q(hi);
    if (lo >= 0.0) return A + log(-expm1(B - A));
    return log1p(-(exp(A) + exp(B)));
}

__device__ __forceinline__ void lse_push(double& mx, double& s, double v)
{
    if (v == -INFINITY) return;
    if (v > mx) {
        s = s * exp(mx - v) + 1.0;
        mx = v;
    } else {
        s += exp(v - mx);
    }
}

// Pr(lo <= Z < hi) for a standard normal Z in the same mirrored form as
// ln_interval, from the complementary error function: the upper-tail case is
// (erfc(lo/sqrt 2) - erfc(hi/sqrt 2)) / 2, the case containing the mean
// 1 - (erfc(|lo|/sqrt 2) + erfc(hi/sqrt 2)) / 2.  erfc keeps its relative
// accuracy down to about 1e-300, i.e. |z| up to about 37.
__device__ __forceinline__ double interval_prob(double lo, double hi)
{
    if (hi <= 0.0) {
        const double t = lo;
        lo = -hi;
        hi = -t;
    }
    const double ea = erfc(fabs(lo) * M_SQRT1_2);
    const double eb = erfc(hi * M_SQRT1_2);
    return (lo >= 0.0) ? 0.5 * (ea - eb) : 1.0 - 0.5 * (ea + eb);
}

// ln(1 + e^z) without overflow; +inf at z = +inf, 0 at z = -inf.
__device__ __forceinline__ double softplus(double z)
{
    return fmax(z, 0.0) + log1p(exp(-fabs(z)));
}

// One thread per sample.  Only the 2^(m - |known|) labels that agree with the
// sample's known slice bits are visited (a uniform trip count: the free bit
// positions are the same for every sample), so wavefronts do not diverge over
// interval membership.  Interval bounds come from an LDS copy of the
// thresholds with t_0 = -inf and t_{2^m} = +inf.
// The two sums of interval probabilities are formed in linear fp64 (two erfc
// per interval, one log per sample); a sample whose smaller sum falls below
// 1e-290, where erfc would lose relative accuracy or underflow, is redone in
// the log domain (ln_interval and a running log-sum-exp).
// NEXT: the same pass also yields the LLR of slice j+1 given bit j = 0 and
// given bit j = 1 (the interval probabilities it needs are among those
// visited).  Each is summed over its labels in the order slice j+1's own pass
// would visit them, so both equal that pass bit for bit.
// PRIOR: each label is also weighted by prod_i Pr(S_i = bit i of the label)
// over the slices i in prior_mask, with Pr(S_i = 0) = 1 / (1 + e^-lambda_i),
// Pr(S_i = 1) = 1 / (1 + e^lambda_i) from the prior LLR lambda_i of the sample
// (ln of the logistic factor, -softplus, in the log-domain pass).
// Four waves per SIMD (at most 128 VGPRs) pays for the prior form only:
// 5.5 vs 6.9 ms at 2^27 samples; the one-pass form is 2.6 % slower with it.
template <bool PRIOR, bool NEXT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PRIOR ? 4 : 1))) void k_slice_llr(LlrArgs a)
{
    __shared__ double bnd[kMaxThr + 2];
    const int K = 1 << a.m_bits;
    for (int q = threadIdx.x; q <= K; q += blockDim.x)
        bnd[q] = (q == 0) ? -INFINITY : (q == K ? INFINITY : a.t[q - 1]);
    __syncthreads();
    const uint32_t freemask = uint32_t(K - 1) & ~a.known;
    const int nfree = __popc(freemask);
    const double inv_sigma = 1.0 / a.sigma;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const double x = a.x[i];
        uint32_t kb = 0;
        for (int q = 0; q < a.m_bits; ++q)
            if ((a.known >> q) & 1u) kb |= uint32_t(a.slices[int64_t(q) * a.n + i] & 1) << q;
        // interval index and bit j of the c-th label consistent with the known bits
        // (g is the label's bit pattern, k its interval)
        auto label = [&](int c, uint32_t& k, uint32_t& g) {
            uint32_t fm = freemask;
            g = kb;
            for (int b = 0; b < nfree; ++b) {
                const uint32_t low = fm & (~fm + 1u);
                if ((c >> b) & 1) g |= low;
                fm &= fm - 1u;
            }
            k = g;
            if (a.gray)
                for (uint32_t sh = 1; sh < 8; sh <<= 1) k ^= k >> sh;
            return (g >> a.j) & 1u;
        };
        // prior LLR of each slice in prior_mask (PRIOR only), by slice index, and
        // its two logistic factors Pr(S_q = 0), Pr(S_q = 1) for the linear pass
        double lam[8], pr0[8], pr1[8];
        if constexpr (PRIOR) {
            for (int q = 0; q < 8; ++q) {
                const bool on = q < a.m_bits && ((a.prior_mask >> q) & 1u);
                lam[q] = on ? double(a.prior[int64_t(q) * a.n + i]) : 0.0;
                pr0[q] = on ? 1.0 / (1.0 + exp(-lam[q])) : 1.0;
                pr1[q] = on ? 1.0 / (1.0 + exp(lam[q])) : 1.0;
            }
        }
        // the label's prior weight, linear or logarithmic
        auto prior_w = [&](uint32_t g) {
            double w = 1.0;
            for (int q = 0; q < 8; ++q)
                if ((a.prior_mask >> q) & 1u) w *= ((g >> q) & 1u) ? pr1[q] : pr0[q];
            return w;
        };
        auto prior_lnw = [&](uint32_t g) {
            double w = 0.0;
            for (int q = 0; q < 8; ++q)
                if ((a.prior_mask >> q) & 1u) w -= softplus(((g >> q) & 1u) ? lam[q] : -lam[q]);
            return w;
        };
        double p0 = 0.0, p1 = 0.0;
        double q00 = 0.0, q01 = 0.0, q10 = 0.0, q11 = 0.0;   // NEXT: (bit j, bit j+1)
        for (int c = 0; c < (1 << nfree); ++c) {
            uint32_t k, g;
            const uint32_t bit = label(c, k, g);
            double p = interval_prob((bnd[k] - x) * inv_sigma, (bnd[k + 1] - x) * inv_sigma);
            if constexpr (PRIOR) p *= prior_w(g);
            if (bit) p1 += p;
            else p0 += p;
            if constexpr (NEXT) {
                const uint32_t up = (g >> (a.j + 1)) & 1u;
                if (bit) (up ? q11 : q10) += p;
                else (up ? q01 : q00) += p;
            }
        }
        double L;
        if (p0 > 1e-290 && p1 > 1e-290) {
            L = log(p0 / p1);
        } else {
            double m0 = -INFINITY, s0 = 0.0, m1 = -INFINITY, s1 = 0.0;
            for (int c = 0; c < (1 << nfree); ++c) {
                uint32_t k, g;
                const uint32_t bit = label(c, k, g);
                double lp = ln_interval((bnd[k] - x) / a.sigma, (bnd[k + 1] - x) / a.sigma);
                if constexpr (PRIOR) lp += prior_lnw(g);
                if (bit) lse_push(m1, s1, lp);
                else lse_push(m0, s0, lp);
            }
            L = (m0 + log(s0)) - (m1 + log(s1));
        }
        if (a.out_f64) static_cast<double*>(a.out)[i] = L;
        else static_cast<float*>(a.out)[i] = float(L);
        if constexpr (NEXT) {
            for (uint32_t b = 0; b < 2; ++b) {
                const double s0 = b ? q10 : q00, s1 = b ? q11 : q01;
                double Ln;
                if (s0 > 1e-290 && s1 > 1e-290) {
                    Ln = log(s0 / s1);
                } else {
                    double m0 = -INFINITY, t0 = 0.0, m1 = -INFINITY, t1 = 0.0;
                    for (int c = 0; c < (1 << nfree); ++c) {
                        uint32_t k, g;
                        const uint32_t bit = label(c, k, g);
                        if (bit != b) continue;
                        const double lp = ln_interval((bnd[k] - x) / a.sigma, (bnd[k + 1] - x) / a.sigma);
                        if ((g >> (a.j + 1)) & 1u) lse_push(m1, t1, lp);
                        else lse_push(m0, t0, lp);
                    }
                    Ln = (m0 + log(t0)) - (m1 + log(t1));
                }
                void* dst = b ? a.next1 : a.next0;
                if (a.out_f64) static_cast<double*>(dst)[i] = Ln;
                else static_cast<float*>(dst)[i] = float(Ln);
            }
        }
    }
}

// out = bits & 1 ? l1 : l0, one sample per thread and stride.
__global__ __launch_bounds__(256) void k_llr_choose(ChooseArgs a)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const bool one = a.bits[i] & 1;
        if (a.f64) static_cast<double*>(a.out)[i] = one ? static_cast<const double*>(a.l1)[i]
                                                        : static_cast<const double*>(a.l0)[i];
        else static_cast<float*>(a.out)[i] = one ? static_cast<const float*>(a.l1)[i]
                                                 : static_cast<const float*>(a.l0)[i];
    }
}

// Hard LLR of a binary symmetric channel with crossover p: Alice quantises
// her own x with the same thresholds and labelling, takes bit j of the label
// (a_j), and outputs (1 - 2 a_j) ln((1 - p) / p).  One thread per sample.
__global__ __launch_bounds__(256) void k_slice_llr_bsc(BscArgs a)
{
    const double mag = log1p(-a.p) - log(a.p);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const double x = a.x[i];
        int k = 0;
        for (int q = 0; q < a.nthr; ++q) k += (a.t[q] <= x) ? 1 : 0;
        const int g = a.gray ? (k ^ (k >> 1)) : k;
        const double L = ((g >> a.j) & 1) ? -mag : mag;
        if (a.out_f64) static_cast<double*>(a.out)[i] = L;
        else static_cast<float*>(a.out)[i] = float(L);
    }
}

static int grid_for(int64_t items, int per_block)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return int(g);
}

static cvr_status check_thresholds(const char* fn, const double* t, int32_t m_bits)
{
    if (m_bits < 1 || m_bits > 8) return fail(CVR_EINVAL, std::string(fn) + ": m_bits must be in [1, 8]");
    if (!t) return fail(CVR_EINVAL, std::string(fn) + ": thresholds is NULL");
    const int nthr = (1 << m_bits) - 1;
    for (int q = 0; q < nthr; ++q) {
        if (!std::isfinite(t[q])) return fail(CVR_EINVAL, std::string(fn) + ": non-finite threshold");
        if (q > 0 && !(t[q] > t[q - 1])) return fail(CVR_EINVAL, std::string(fn) + ": thresholds not strictly ascending");
    }
    return CVR_OK;
}

}  // namespace cvr

using namespace cvr;

extern "C" cvr_status slice_quantize(const double* y, int64_t n, const double* thresholds, int32_t m_bits,
                                     int32_t labelling, uint8_t* slices, void* stream)
{
    if (n < 0) return fail(CVR_EINVAL, "slice_quantize: n < 0");
    if (labelling != CVR_GRAY && labelling != CVR_BINARY) return fail(CVR_EINVAL, "slice_quantize: bad labelling");
    if (cvr_status st = check_thresholds("slice_quantize", thresholds, m_bits)) return st;
    if (n == 0) return CVR_OK;
    if (!y || !slices) return fail(CVR_EINVAL, "slice_quantize: NULL y or slices");
    QuantArgs a{};
    a.y = y;
    a.slices = slices;
    a.n = n;
    a.m_bits = m_bits;
    a.nthr = (1 << m_bits) - 1;
    a.gray = labelling == CVR_GRAY;
    for (int q = 0; q < a.nthr; ++q) a.t[q] = thresholds[q];
    a.vec = (n % 4 == 0) && (reinterpret_cast<uintptr_t>(y) % 32 == 0) &&
            (reinterpret_cast<uintptr_t>(slices) % 4 == 0);
    ProfScope prof(CVR_PROF_QUANTIZE, hipStream_t(stream));
    hipLaunchKernelGGL(k_quantize, dim3(grid_for((n + 3) / 4, 256)), dim3(256), 0, hipStream_t(stream), a);
    return check_launch("slice_quantize");
}

extern "C" cvr_status slice_llr(const double* x, int64_t n, double sigma_n, const double* thresholds, int32_t m_bits,
                                int32_t labelling, int32_t j, uint32_t known_mask, const uint8_t* slices,
                                int32_t out_dtype, void* llr_out, void* stream)
{
    if (n < 0) return fail(CVR_EINVAL, "slice_llr: n < 0");
    if (labelling != CVR_GRAY && labelling != CVR_BINARY) return fail(CVR_EINVAL, "slice_llr: bad labelling");
    if (cvr_status st = check_thresholds("slice_llr", thresholds, m_bits)) return st;
    if (!(sigma_n > 0.0) || !std::isfinite(sigma_n)) return fail(CVR_EINVAL, "slice_llr: sigma_n must be finite and > 0");
    if (j < 0 || j >= m_bits) return fail(CVR_EINVAL, "slice_llr: j out of range");
    if ((known_mask >> j) & 1u) return fail(CVR_EINVAL, "slice_llr: slice j is already in known_mask");
    if (known_mask >> m_bits) return fail(CVR_EINVAL, "slice_llr: known_mask has bits >= m_bits");
    if (out_dtype != CVR_F32 && out_dtype != CVR_F64) return fail(CVR_EINVAL, "slice_llr: out_dtype must be F32 or F64");
    if (n == 0) return CVR_OK;
    if (!x || !llr_out) return fail(CVR_EINVAL, "slice_llr: NULL x or llr_out");
    if (known_mask && !slices) return fail(CVR_EINVAL, "slice_llr: known_mask set but slices is NULL");
    LlrArgs a{};
    a.x = x;
    a.slices = slices;
    a.out = llr_out;
    a.n = n;
    a.sigma = sigma_n;
    a.m_bits = m_bits;
    a.nthr = (1 << m_bits) - 1;
    a.gray = labelling == CVR_GRAY;
    a.j = j;
    a.known = known_mask;
    a.out_f64 = out_dtype == CVR_F64;
    for (int q = 0; q < a.nthr; ++q) a.t[q] = thresholds[q];
    ProfScope prof(CVR_PROF_LLR, hipStream_t(stream));
    hipLaunchKernelGGL((k_slice_llr<false, false>), dim3(grid_for(n, 256)), dim3(256), 0, hipStream_t(stream), a);
    return check_launch("slice_llr");
}

extern "C" cvr_status slice_llr_next(const double* x, int64_t n, double sigma_n, const double* thresholds,
                                     int32_t m_bits, int32_t labelling, int32_t j, uint32_t known_mask,
                                     const uint8_t* slices, int32_t out_dtype, void* llr_out, void* next_if0,
                                     void* next_if1, void* stream)
{
    if (n < 0) return fail(CVR_EINVAL, "slice_llr_next: n < 0");
    if (labelling != CVR_GRAY && labelling != CVR_BINARY) return fail(CVR_EINVAL, "slice_llr_next: bad labelling");
    if (cvr_status st = check_thresholds("slice_llr_next", thresholds, m_bits)) return st;
    if (!(sigma_n > 0.0) || !std::isfinite(sigma_n))
        return fail(CVR_EINVAL, "slice_llr_next: sigma_n must be finite and > 0");
    if (j < 0 || j + 1 >= m_bits) return fail(CVR_EINVAL, "slice_llr_next: need 0 <= j and j + 1 < m_bits");
    if ((known_mask >> j) & 3u) return fail(CVR_EINVAL, "slice_llr_next: slice j or j + 1 is in known_mask");
    if (known_mask >> m_bits) return fail(CVR_EINVAL, "slice_llr_next: known_mask has bits >= m_bits");
    if (out_dtype != CVR_F32 && out_dtype != CVR_F64)
        return fail(CVR_EINVAL, "slice_llr_next: out_dtype must be F32 or F64");
    if (n == 0) return CVR_OK;
    if (!x || !llr_out || !next_if0 || !next_if1) return fail(CVR_EINVAL, "slice_llr_next: NULL x or output");
    if (known_mask && !slices) return fail(CVR_EINVAL, "slice_llr_next: known_mask set but slices is NULL");
    LlrArgs a{};
    a.x = x;
    a.slices = slices;
    a.out = llr_out;
    a.n = n;
    a.sigma = sigma_n;
    a.m_bits = m_bits;
    a.nthr = (1 << m_bits) - 1;
    a.gray = labelling == CVR_GRAY;
    a.j = j;
    a.known = known_mask;
    a.out_f64 = out_dtype == CVR_F64;
    a.next0 = next_if0;
    a.next1 = next_if1;
    for (int q = 0; q < a.nthr; ++q) a.t[q] = thresholds[q];
    ProfScope prof(CVR_PROF_LLR, hipStream_t(stream));
    hipLaunchKernelGGL((k_slice_llr<false, true>), dim3(grid_for(n, 256)), dim3(256), 0, hipStream_t(stream), a);
    return check_launch("slice_llr_next");
}

extern "C" cvr_status slice_llr_choose(const void* llr_if0, const void* llr_if1, const uint8_t* bits, int64_t n,
                                       int32_t dtype, void* llr_out, void* stream)
{
    if (n < 0) return fail(CVR_EINVAL, "slice_llr_choose: n < 0");
    if (dtype != CVR_F32 && dtype != CVR_F64) return fail(CVR_EINVAL, "slice_llr_choose: dtype must be F32 or F64");
    if (n == 0) return CVR_OK;
    if (!llr_if0 || !llr_if1 || !bits || !llr_out) return fail(CVR_EINVAL, "slice_llr_choose: NULL argument");
    ChooseArgs a{llr_if0, llr_if1, bits, llr_out, n, dtype == CVR_F64};
    ProfScope prof(CVR_PROF_LLR, hipStream_t(stream));
    hipLaunchKernelGGL(k_llr_choose, dim3(grid_for(n, 256)), dim3(256), 0, hipStream_t(stream), a);
    return check_launch("slice_llr_choose");
}

extern "C" cvr_status slice_llr_prior(const double* x, int64_t n, double sigma_n, const double* thresholds,
                                      int32_t m_bits, int32_t labelling, int32_t j, uint32_t known_mask,
                                      const uint8_t* slices, uint32_t prior_mask, const float* prior_llr,
                                      int32_t out_dtype, void* llr_out, void* stream)
{
    if (n < 0) return fail(CVR_EINVAL, "slice_llr_prior: n < 0");
    if (labelling != CVR_GRAY && labelling != CVR_BINARY) return fail(CVR_EINVAL, "slice_llr_prior: bad labelling");
    if (cvr_status st = check_thresholds("slice_llr_prior", thresholds, m_bits)) return st;
    if (!(sigma_n > 0.0) || !std::isfinite(sigma_n))
        return fail(CVR_EINVAL, "slice_llr_prior: sigma_n must be finite and > 0");
    if (j < 0 || j >= m_bits) return fail(CVR_EINVAL, "slice_llr_prior: j out of range");
    if ((known_mask >> m_bits) || (prior_mask >> m_bits))
        return fail(CVR_EINVAL, "slice_llr_prior: known_mask or prior_mask has bits >= m_bits");
    if (((known_mask | prior_mask) >> j) & 1u)
        return fail(CVR_EINVAL, "slice_llr_prior: slice j is in known_mask or prior_mask");
    if (known_mask & prior_mask) return fail(CVR_EINVAL, "slice_llr_prior: known_mask and prior_mask overlap");
    if (out_dtype != CVR_F32 && out_dtype != CVR_F64)
        return fail(CVR_EINVAL, "slice_llr_prior: out_dtype must be F32 or F64");
    if (n == 0) return CVR_OK;
    if (!x || !llr_out) return fail(CVR_EINVAL, "slice_llr_prior: NULL x or llr_out");
    if (known_mask && !slices) return fail(CVR_EINVAL, "slice_llr_prior: known_mask set but slices is NULL");
    if (prior_mask && !prior_llr) return fail(CVR_EINVAL, "slice_llr_prior: prior_mask set but prior_llr is NULL");
    LlrArgs a{};
    a.x = x;
    a.slices = slices;
    a.out = llr_out;
    a.n = n;
    a.sigma = sigma_n;
    a.m_bits = m_bits;
    a.nthr = (1 << m_bits) - 1;
    a.gray = labelling == CVR_GRAY;
    a.j = j;
    a.known = known_mask;
    a.out_f64 = out_dtype == CVR_F64;
    a.prior = prior_llr;
    a.prior_mask = prior_mask;
    for (int q = 0; q < a.nthr; ++q) a.t[q] = thresholds[q];
    ProfScope prof(CVR_PROF_LLR, hipStream_t(stream));
    hipLaunchKernelGGL((k_slice_llr<true, false>), dim3(grid_for(n, 256)), dim3(256), 0, hipStream_t(stream), a);
    return check_launch("slice_llr_prior");
}

extern "C" cvr_status slice_llr_bsc(const double* x, int64_t n, const double* thresholds, int32_t m_bits,
                                    int32_t labelling, int32_t j, double p, int32_t out_dtype, void* llr_out,
                                    void* stream)
{
    if (n < 0) return fail(CVR_EINVAL, "slice_llr_bsc: n < 0");
    if (labelling != CVR_GRAY && labelling != CVR_BINARY) return fail(CVR_EINVAL, "slice_llr_bsc: bad labelling");
    if (cvr_status st = check_thresholds("slice_llr_bsc", thresholds, m_bits)) return st;
    if (j < 0 || j >= m_bits) return fail(CVR_EINVAL, "slice_llr_bsc: j out of range");
    if (!(p > 0.0 && p < 1.0)) return fail(CVR_EINVAL, "slice_llr_bsc: p must be in (0, 1)");
    if (out_dtype != CVR_F32 && out_dtype != CVR_F64)
        return fail(CVR_EINVAL, "slice_llr_bsc: out_dtype must be F32 or F64");
    if (n == 0) return CVR_OK;
    if (!x || !llr_out) return fail(CVR_EINVAL, "slice_llr_bsc: NULL x or llr_out");
    BscArgs a{};
    a.x = x;
    a.out = llr_out;
    a.n = n;
    a.p = p;
    a.nthr = (1 << m_bits) - 1;
    a.gray = labelling == CVR_GRAY;
    a.j = j;
    a.out_f64 = out_dtype == CVR_F64;
    for (int q = 0; q < a.nthr; ++q) a.t[q] = thresholds[q];
    ProfScope prof(CVR_PROF_LLR, hipStream_t(stream));
    hipLaunchKernelGGL(k_slice_llr_bsc, dim3(grid_for(n, 256)), dim3(256), 0, hipStream_t(stream), a);
    return check_launch("slice_llr_bsc");
}
