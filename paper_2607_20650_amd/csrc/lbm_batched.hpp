// lbm_batched.hpp -- device descriptors of the serving engine.
#pragma once

#include "lbm_common.hpp"

namespace lbm {

constexpr int BATCH_TILE_X = 64; // one wavefront per tile row
constexpr int BATCH_TILE_Y = 4;

// One resident request, as the batched kernel sees it.
struct SlotDesc {
    void* lat[2];         // two lattices (pull state in lat[steps_done & 1])
    const uint8_t* types; // node types [ny][px]
    const uint32_t* links; // link words [ny][px] (KParams::links)
    float* rin2;          // Neumann inlet densities, 2 x ny (by update parity), or null
    Geometry g;
    Physics ph;
    int64_t steps_done;   // updates done before the current bundle
    int64_t steps_left;   // updates still to do at the start of the bundle
};

struct WorkItem {
    int32_t slot;
    int32_t x0, y0; // first node of the tile
};

hipError_t launch_batched(int layout, int prec, const SlotDesc* slots, const WorkItem* work, const int32_t* n_work,
                          int k, int blocks, hipStream_t s);

// Persistent grid size of the batched kernel: resident blocks on the device.
int batched_blocks(int layout, int prec);

} // namespace lbm
