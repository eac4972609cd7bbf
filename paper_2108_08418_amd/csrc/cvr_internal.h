// Internal declarations shared by the translation units of libcvqkd_recon.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cvqkd_recon.h"

namespace cvr {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
cvr_status fail(cvr_status st, const std::string& msg);
cvr_status check_launch(const char* what);

#define CVR_HIP_TRY(expr)                                                        \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess)                                                    \
            return ::cvr::fail(CVR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Opt-in launch timing (cvr_profile_enable): brackets the launches made in its
// scope with HIP events on stream s.
constexpr int kProfKinds = 8;   // CVR_PROF_* kinds
class ProfScope {
public:
    ProfScope(int kind, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

private:
    int kind_;
    hipStream_t s_;
    void* a_ = nullptr;
};

constexpr int kMaxRowDeg = 32;
constexpr int kMaxTypes = 16;
constexpr int kTile = 256;          // threads per work tile

// ---------------------------------------------------------------------------
// device-side views (plain structs copied to device memory)
// ---------------------------------------------------------------------------
struct QcBlock {          // one nonzero circulant of a QC code
    int32_t other;        // block column (row table) or block row (column table)
    int32_t shift;
    int32_t blk;          // index of the block: messages of block b live at [b*Z, b*Z+Z)
    int32_t type;         // edge class
};

struct DevCode {
    int32_t n, m;
    int64_t E;
    int32_t max_row_deg, max_col_deg, n_types, is_qc;
    int32_t min_row_deg, pad0;
    int32_t nb, mb, Z, NB;
    // CSR (always present): row c -> edges row_ptr[c]..row_ptr[c+1]-1
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const uint8_t* edge_type;
    // column view: variable v -> CSR edge ids col_edge[col_ptr[v]..col_ptr[v+1]-1], checks ascending
    const int32_t* col_ptr;
    const int32_t* col_edge;
    // QC tables (is_qc only): per block row / block column, blocks in ascending order
    const int32_t* qrow_ptr;
    const QcBlock* qrow;
    const int32_t* qcol_ptr;
    const QcBlock* qcol;
    const int32_t* qcol_rank;   // block columns by degree, descending (ties: lower index first)
    // one word per table entry (NULL unless Z <= 65535 and nb <= 512):
    // row: shift | block column << 16 | type << 25; column: shift | block id << 16
    const int32_t* qrow_pk;
    const int32_t* qcol_pk;
};

struct DevFrame {
    int32_t code;
    int32_t n;
    int32_t m;
    int32_t pad;
    int64_t vn_off;
    int64_t chk_off;
    int64_t msg_off;       // offset of the frame's messages in the workspace message array
};

// A unit of work of <= kTile consecutive rows or variables of one frame.
struct Tile {
    int32_t frame;
    int32_t a;             // generic: first row/variable; QC: block row/column
    int32_t b;             // QC: first k / u inside the circulant; generic: unused
    int32_t count;         // bit 31: first variable tile of its frame; low bits: item count
};
constexpr int32_t kFirstTile = int32_t(0x80000000u);

}  // namespace cvr

// ---------------------------------------------------------------------------
// host-side handles
// ---------------------------------------------------------------------------
struct cvr_code_s {
    cvr::DevCode dev;          // device pointers inside
    std::vector<void*> allocations;
    int64_t E = 0;
};

struct cvr_batch_s {
    int32_t F = 0;
    int64_t total_n = 0, total_m = 0, total_E = 0;
    int32_t max_row_deg = 0;
    int32_t max_types = 1;
    int32_t max_mb = 0, max_nb = 0, max_NB = 0;   // largest QC protograph dimensions of the batch
    bool all_qc = false;
    std::vector<cvr_code_t> codes;
    std::vector<cvr::DevFrame> frames_host;
    cvr::DevCode* d_codes = nullptr;
    cvr::DevFrame* d_frames = nullptr;
    int32_t* d_order = nullptr;           // processing order of the persistent decoder: largest frames first
    cvr::Tile* d_cn_tiles = nullptr;     // generic rows
    cvr::Tile* d_vn_tiles = nullptr;     // generic variables
    cvr::Tile* d_qcn_tiles = nullptr;    // QC rows (within a block row)
    cvr::Tile* d_qvn_tiles = nullptr;    // QC variables (within a block column)
    int64_t n_cn_tiles = 0, n_vn_tiles = 0, n_qcn_tiles = 0, n_qvn_tiles = 0;
};
