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

// Compiled (threads per workgroup, waves per SIMD) shapes of the render and
// backward kernels.
#define FR_KERNEL_SHAPES(X) X(256, 4) X(256, 8) X(512, 4) X(512, 8) X(1024, 4) X(1024, 8)
// Workspace header: work-queue and completion counters of the persistent grid.
constexpr int64_t kWsCounterBytes = 256;

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
    // high-pass chunk its partial end deviation and its initial deviation, per room the
    // high-pass unforced responses over a chunk and the decimation taps
    int64_t ws_zend_off = 0, ws_init_off = 0, ws_basis_off = 0, ws_taps_off = 0, ws_mr_bytes = 0;
};

int fr_fail(int code, const char* fmt, ...);
