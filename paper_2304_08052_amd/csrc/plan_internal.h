// Host-side plan object of the FRAM-RIR library (opaque behind framrir.h).
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/framrir.h"
#include "framrir_internal.h"

// Largest LDS accumulator budget per workgroup: 160 000 B of gfx950 LDS minus
// the compacted image list, the bound reduction and small scratch.
constexpr int kMaxAccLdsBytes = 160000 - 4 * framrir::kListCap - 6144;
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
    int32_t grid = 1;
};

int fr_fail(int code, const char* fmt, ...);
