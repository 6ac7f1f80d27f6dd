// Host-side plan object of the FRAM-RIR library (opaque behind framrir.h).
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/framrir.h"
#include "framrir_internal.h"

// gfx950 LDS per compute unit, and the largest dynamic LDS of one workgroup
// (accumulator tile plus compacted image list), leaving room for the kernels'
// static scratch.
constexpr int kLdsPerCu = 163840;
constexpr int kMaxDynLdsBytes = 160000;
// Compute units of an MI355X (gfx950): only the order in which the
// preparation takes the sources depends on it.
constexpr int kCus = 256;

// Compiled (threads per workgroup, waves per SIMD) shapes of the render and
// backward kernels.
#define FR_KERNEL_SHAPES(X) X(256, 4) X(256, 8) X(512, 4) X(512, 8) X(1024, 4) X(1024, 8)
// Workspace header: work-queue and completion counters of the persistent grid.
constexpr int64_t kWsCounterBytes = 256;

// Render by bin moments (render_path 1): per microphone 7 rows (six moments
// and the direct row of the centre taps) of R = 256 nblk + 80 bins for a tile
// of at most 256 nblk samples.  Bin e sits in word e + 4 (e / 32) of its row
// (4 pad words after every 32 bins, so that the 16 columns of a matrix-core
// operand read, 16 bins apart, fall on distinct LDS banks); a row takes
// mom_row_words(R) words.  Static LDS of that kernel: mic positions and the
// item slot.
constexpr int kMomRows = 7;
constexpr int kMomBlock = 256;
constexpr int kMomMaxBlocks = 31;   // tiles of at most 7936 samples
constexpr int kMomStaticLds = 1024;
constexpr int mom_row_words(int r) { return r + 4 * ((r + 31) / 32); }
// Longest tile of a group of mg microphones within lds_bytes (a multiple of
// 256 samples), or 0 when not even one block fits.
constexpr int moment_tile_cap(int lds_bytes, int mg) {
    int nblk = 0;
    while (nblk < kMomMaxBlocks &&
           static_cast<int64_t>(4) * kMomRows * mg * mom_row_words((nblk + 1) * kMomBlock + 80) <= lds_bytes)
        ++nblk;
    return nblk * kMomBlock;
}

struct framrir_plan {
    framrir_params prm;
    framrir_launch launch;
    framrir::DescHeader header;
    std::vector<framrir::RoomDesc> rooms;
    std::vector<framrir::SrcDesc> srcs;
    std::vector<framrir::WorkItem> items;
    std::vector<int32_t> room_items;
    std::vector<char> blob;
    int64_t ws_bytes = 0;
    int64_t ws_bwd_bytes = 0;
    int32_t grid = 1;       // render workgroups
    int32_t bwd_grid = 1;   // backward workgroups
    // workspace layout: counters | per-source scale | bucket offsets | slot of
    // row 0 | per-room completion counts | delay-ordered rows (ws_bytes: the
    // render) | per-item partials (ws_bwd_bytes: the backward)
    int64_t ws_scale_off = 0, ws_bucket_off = 0, ws_row0_off = 0, ws_room_off = 0, ws_rows_off = 0,
            ws_part_off = 0;
    // multi-rate workspace (ws_mr_bytes): the render workspace, then per
    // high-pass chunk its partial end deviation and its initial deviation, per
    // sub-chunk the chunk's partial deviation at its start, and per r_l the
    // decimation filter's matrix-core fragments
    int64_t ws_zend_off = 0, ws_init_off = 0, ws_sub_off = 0, ws_taps_off = 0, ws_mr_bytes = 0;
};

int fr_fail(int code, const char* fmt, ...);
