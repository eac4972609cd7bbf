// Batched belief-propagation decoding of sub-blocks (Sec. III-A, Sec. III-C),
// flooding or layered, and syndrome checks (Sec. II Step 5).
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
#include "cvr_decode_impl.h"

#include <atomic>
#include <mutex>

namespace cvr {

// ---------------------------------------------------------------------------
// syndrome check over F frames of one code
// ---------------------------------------------------------------------------
struct SynArgs {
    DevCode code;
    const uint8_t* bits;
    const uint8_t* ref;
    uint8_t* out;
    int32_t* n_unsat;
    int32_t F;
    int32_t fpt;              // frames per thread (k_syndrome_qc)
};

__global__ __launch_bounds__(256) void k_syndrome(SynArgs a)
{
    const int f = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const DevCode& cd = a.code;
    int bad = 0;
    if (r < cd.m) {
        const uint8_t* b = a.bits + int64_t(f) * cd.n;
        int par = 0;
        for (int e = cd.row_ptr[r]; e < cd.row_ptr[r + 1]; ++e) par ^= b[cd.col_idx[e]] & 1;
        const int ref = a.ref ? (a.ref[int64_t(f) * cd.m + r] & 1) : 0;
        if (a.out) a.out[int64_t(f) * cd.m + r] = uint8_t(par);
        bad = par != ref;
    }
    if (a.n_unsat) add_unsat(&a.n_unsat[f], bad);
}

// Quasi-cyclic codes: row i Z + k XORs the bits (k + shift) mod Z of its block
// columns, so a wavefront's 64 rows read 64 consecutive bits of each block (no
// index array); the packed row table gives shift | block column << 16.  A
// thread takes its row in a.fpt <= kSynFrames frames, with all of their bits
// of one table entry loaded before they are combined (with one row per thread,
// a launch over thousands of frames was mostly workgroup dispatch).
constexpr int kSynFrames = 8;

__global__ __launch_bounds__(256) void k_syndrome_qc(SynArgs a)
{
    const int f0 = blockIdx.y * a.fpt;
    const int nf = min(a.fpt, a.F - f0);                     // block-uniform, <= kSynFrames
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const DevCode& cd = a.code;
    int par[kSynFrames];
#pragma unroll
    for (int h = 0; h < kSynFrames; ++h) par[h] = 0;
    if (r < cd.m) {
        const int Z = cd.Z;
        const int i = r / Z;
        const int k = r - i * Z;
        const int q1 = cd.qrow_ptr[i + 1];
        for (int q = cd.qrow_ptr[i]; q < q1; ++q) {
            const int32_t e = cd.qrow_pk[q];
            int u = k + (e & 0xffff);
            u = u >= Z ? u - Z : u;
            const uint8_t* b = a.bits + int64_t(f0) * cd.n + ((e >> 16) & 0x1ff) * Z + u;
            uint8_t v[kSynFrames];
#pragma unroll
            for (int h = 0; h < kSynFrames; ++h) v[h] = (h < nf) ? b[int64_t(h) * cd.n] : uint8_t(0);
#pragma unroll
            for (int h = 0; h < kSynFrames; ++h) par[h] ^= v[h] & 1;
        }
    }
#pragma unroll
    for (int h = 0; h < kSynFrames; ++h) {
        if (h >= nf) break;
        const int64_t f = f0 + h;
        int bad = 0;
        if (r < cd.m) {
            const int ref = a.ref ? (a.ref[f * cd.m + r] & 1) : 0;
            if (a.out) a.out[f * cd.m + r] = uint8_t(par[h]);
            bad = par[h] != ref;
        }
        if (a.n_unsat) add_unsat(&a.n_unsat[f], bad);
    }
}

static cvr_status check_params(const cvr_batch_s* b, const cvr_decode_params* p)
{
    if (!b) return fail(CVR_EINVAL, "decode: NULL batch");
    if (!p) return fail(CVR_EINVAL, "decode: NULL params");
    if (p->algo != CVR_SP && p->algo != CVR_NMS) return fail(CVR_EINVAL, "decode: bad algo");
    if (p->max_iter < 0 || p->max_iter > 100000) return fail(CVR_EINVAL, "decode: max_iter out of range");
    if (p->math != CVR_F32 && p->math != CVR_F64) return fail(CVR_EINVAL, "decode: math must be F32 or F64");
    if (p->store != CVR_F64 && p->store != CVR_F32 && p->store != CVR_F16) return fail(CVR_EINVAL, "decode: bad store");
    if (p->store == CVR_F64 && p->math != CVR_F64) return fail(CVR_EINVAL, "decode: F64 storage needs F64 math");
    if (p->math == CVR_F64 && p->store != CVR_F64)
        return fail(CVR_EUNSUPPORTED, "decode: F64 math is implemented with F64 storage only");
    if (p->algo == CVR_SP && !(p->msg_clamp > 0.0f)) return fail(CVR_EINVAL, "decode: msg_clamp must be > 0");
    if (p->schedule < CVR_SCHED_AUTO || p->schedule > CVR_SCHED_LAYERED) return fail(CVR_EINVAL, "decode: bad schedule");
    if (p->schedule == CVR_SCHED_LAYERED) {
        if (p->wg_threads != 0 && p->wg_threads != 256 && p->wg_threads != 512 && p->wg_threads != 1024)
            return fail(CVR_EINVAL, "decode: wg_threads must be 0, 256, 512 or 1024");
    } else if (p->wg_threads != 0 && p->wg_threads != 512 && p->wg_threads != 1024) {
        return fail(CVR_EINVAL, "decode: wg_threads must be 0, 512 or 1024");
    }
    if (p->min_waves != 0 && p->min_waves != 8) return fail(CVR_EINVAL, "decode: min_waves must be 0 or 8");
    if (p->lds_cache_kb < -1 || p->lds_cache_kb > 1024) return fail(CVR_EINVAL, "decode: lds_cache_kb must be in [-1, 1024]");
    if (p->group_wgs < 0 || p->group_wgs > 1024) return fail(CVR_EINVAL, "decode: group_wgs must be in [0, 1024]");
    return CVR_OK;
}

}  // namespace cvr

namespace cvr {
static std::atomic<uint64_t> g_group_wait_ticks{kGroupWaitTicks};
uint64_t group_wait_ticks() { return g_group_wait_ticks.load(std::memory_order_relaxed); }
}  // namespace cvr

using namespace cvr;

extern "C" cvr_status cvr_debug_group_wait_ticks(uint64_t ticks)
{
    if (ticks > 10000000000ull) return fail(CVR_EINVAL, "cvr_debug_group_wait_ticks: ticks > 1e10");
    g_group_wait_ticks.store(ticks, std::memory_order_relaxed);
    return CVR_OK;
}

extern "C" cvr_status cvr_decode_workspace_size(cvr_batch_t batch, const cvr_decode_params* params, size_t* bytes)
{
    if (cvr_status st = check_params(batch, params)) return st;
    if (!bytes) return fail(CVR_EINVAL, "cvr_decode_workspace_size: bytes is NULL");
    *bytes = layout(batch, params).total;
    return CVR_OK;
}

extern "C" cvr_status ldpc_decode_batch(cvr_batch_t batch, const cvr_decode_params* params, const void* llr,
                                        const uint8_t* syndrome, uint8_t* bits_out, void* llr_post_out,
                                        int32_t* iters_out, uint8_t* ok_out, void* workspace, size_t ws_bytes,
                                        void* stream)
{
    if (cvr_status st = check_params(batch, params)) return st;
    if (batch->F == 0) return CVR_OK;
    if (!llr || !bits_out || !iters_out || !ok_out) return fail(CVR_EINVAL, "ldpc_decode_batch: NULL input/output");
    const WsLayout w = layout(batch, params);
    if (!workspace || ws_bytes < w.total) return fail(CVR_ENOMEM, "ldpc_decode_batch: workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(CVR_EINVAL, "ldpc_decode_batch: workspace not 256-byte aligned");
    if (params->weights && batch->max_types > kMaxTypes) return fail(CVR_EINVAL, "ldpc_decode_batch: too many edge types");
    char* ws = static_cast<char*>(workspace);
    DecArgs a{};
    a.codes = batch->d_codes;
    a.frames = batch->d_frames;
    a.llr = llr;
    a.syn = syndrome;
    a.c2v = ws + w.c2v;
    a.post = llr_post_out ? llr_post_out : static_cast<void*>(ws + w.post);
    a.trace = params->trace;
    a.bits = bits_out;
    a.iters = iters_out;
    a.ok = ok_out;
    a.active = reinterpret_cast<int32_t*>(ws + w.active);
    a.unsat = reinterpret_cast<int32_t*>(ws + w.unsat);
    a.synw = reinterpret_cast<uint32_t*>(ws + w.synw);
    a.weights = params->weights;
    a.total_n = batch->total_n;
    a.alpha = params->alpha;
    a.clamp = params->msg_clamp;
    a.T = params->max_iter;
    a.early_stop = params->early_stop ? 1 : 0;
    a.n_types = batch->max_types;
    const hipStream_t s = hipStream_t(stream);
    const bool qc = batch->all_qc;
    int mode = 0;
    if (params->schedule == CVR_SCHED_PERSISTENT) {
        if (!frames_fit(batch))
            return fail(CVR_EUNSUPPORTED, "ldpc_decode_batch: the persistent schedule needs QC codes with <= 2048 "
                                          "circulants, <= 512 block rows/columns and Z <= 65535");
        mode = 1;
    } else if (params->schedule == CVR_SCHED_GROUP) {
        if (!frames_fit(batch))
            return fail(CVR_EUNSUPPORTED, "ldpc_decode_batch: the group schedule needs QC codes with <= 2048 "
                                          "circulants, <= 512 block rows/columns and Z <= 65535");
        mode = 2;
    } else if (params->schedule == CVR_SCHED_LAYERED) {
        if (!frames_fit(batch))
            return fail(CVR_EUNSUPPORTED, "ldpc_decode_batch: the layered schedule needs QC codes with <= 2048 "
                                          "circulants, <= 512 block rows/columns and Z <= 65535");
        mode = 3;
    } else if (params->schedule == CVR_SCHED_AUTO) {
        // a workgroup per frame leaves compute units idle below one frame per
        // CU; then groups of workgroups share each frame (16 frames of 2^16:
        // 1.1 ms for both coded slices, against 5.9 ms of per-pass launches)
        if (frames_fit(batch)) mode = batch->F >= device_cus() ? 1 : 2;
    }
    int32_t* queue = reinterpret_cast<int32_t*>(ws + w.queue);
    int32_t* gridws = reinterpret_cast<int32_t*>(ws + w.grid);
    const LaunchShape sh{params->wg_threads, params->min_waves, params->lds_cache_kb, params->group_wgs};
    const bool sp = params->algo == CVR_SP;
    if (params->math == CVR_F64)
        return sp ? decode_f64_sp(batch, a, s, qc, mode, queue, gridws, sh) : decode_f64_nms(batch, a, s, qc, mode, queue, gridws, sh);
    if (params->store == CVR_F32)
        return sp ? decode_f32_sp(batch, a, s, qc, mode, queue, gridws, sh) : decode_f32_nms(batch, a, s, qc, mode, queue, gridws, sh);
    return sp ? decode_f16_sp(batch, a, s, qc, mode, queue, gridws, sh) : decode_f16_nms(batch, a, s, qc, mode, queue, gridws, sh);
}

// ---------------------------------------------------------------------------
// Decoding without allocation: the workspace is a static device array
// ---------------------------------------------------------------------------
// Every GPU the library runs on holds its own copy of `scratch` until the
// process ends.  Host code never names the array as an address (on the host
// it is only a stand-in symbol): its device address is looked up once per
// device, with that device current, and kept here.
namespace cvr {
static __device__ __align__(256) char scratch[CVR_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices];

static cvr_status scratch_for_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CVR_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(CVR_EUNSUPPORTED, "ldpc_decode_batch_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CVR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CVR_OK;
}
}  // namespace cvr

extern "C" cvr_status ldpc_decode_batch_noalloc(cvr_batch_t batch, const cvr_decode_params* params,
                                                const void* llr, const uint8_t* syndrome, uint8_t* bits_out,
                                                void* llr_post_out, int32_t* iters_out, uint8_t* ok_out,
                                                void* stream)
{
    if (cvr_status st = check_params(batch, params)) return st;
    if (batch->F == 0) return CVR_OK;
    const size_t need = layout(batch, params).total;
    if (need > size_t(CVR_NOALLOC_SCRATCH_BYTES))
        return fail(CVR_ENOMEM, "ldpc_decode_batch_noalloc: the batch needs " + std::to_string(need) +
                                    " bytes of workspace, more than the static " +
                                    std::to_string(size_t(CVR_NOALLOC_SCRATCH_BYTES)) + "; use ldpc_decode_batch");
    void* ws = nullptr;
    if (cvr_status st = scratch_for_current_device(&ws)) return st;
    return ldpc_decode_batch(batch, params, llr, syndrome, bits_out, llr_post_out, iters_out, ok_out, ws,
                             size_t(CVR_NOALLOC_SCRATCH_BYTES), stream);
}

extern "C" cvr_status syndrome_check(cvr_code_t code, int32_t F, const uint8_t* bits, const uint8_t* syndrome,
                                     uint8_t* syndrome_out, int32_t* n_unsat, void* stream)
{
    if (!code) return fail(CVR_EINVAL, "syndrome_check: NULL code");
    if (F < 0) return fail(CVR_EINVAL, "syndrome_check: F < 0");
    if (F == 0) return CVR_OK;
    if (F > 65535) return fail(CVR_EINVAL, "syndrome_check: F > 65535");
    if (!bits) return fail(CVR_EINVAL, "syndrome_check: bits is NULL");
    const hipStream_t s = hipStream_t(stream);
    ProfScope prof(CVR_PROF_SYNDROME, s);
    if (n_unsat) {
        hipLaunchKernelGGL(k_zero_i32, dim3((F + 255) / 256), dim3(256), 0, s, n_unsat, int64_t(F));
        if (cvr_status st = check_launch("syndrome_check zero")) return st;
    }
    SynArgs a{};
    a.code = code->dev;
    a.bits = bits;
    a.ref = syndrome;
    a.out = syndrome_out;
    a.n_unsat = n_unsat;
    a.F = F;
    // several frames per thread only when the frames alone fill the chip
    a.fpt = F >= 64 ? kSynFrames : 1;
    if (code->dev.is_qc && code->dev.qrow_pk)
        hipLaunchKernelGGL(k_syndrome_qc, dim3((code->dev.m + 255) / 256, (F + a.fpt - 1) / a.fpt), dim3(256), 0,
                           s, a);
    else
        hipLaunchKernelGGL(k_syndrome, dim3((code->dev.m + 255) / 256, F), dim3(256), 0, s, a);
    return check_launch("syndrome_check");
}
