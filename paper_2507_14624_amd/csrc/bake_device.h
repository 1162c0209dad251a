// Device side of probe baking from a point cloud (Implementation Details, Probe Data
// Generation): every point is taken into the probe's frame and projected onto the
// probe's octahedral map, and each texel keeps the point nearest to the probe.
//
// A workgroup owns one tile (up to 128 x 128 texels) of one probe's map and keeps, in
// LDS, one 64-bit key per texel: the FP32 bits of the squared distance (non-negative, so
// the bits order like the values) above the point index.  Every point of the cloud is
// projected and an LDS atomic min keeps the nearest (ties to the smaller index); the
// tile is then resolved into the distance, normal and radiance maps.  The nearest point
// is an integer decision taken in FP32 with the operations spelled out below, uncontracted
// (the file is compiled with -ffp-contract=off), division and square root correctly
// rounded.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

constexpr int kBakeTile = 128;  // LDS: 128 * 128 keys * 8 B = 128 KiB per workgroup
constexpr int kBakeThreads = 1024;

struct BakeGrid {
    int n[3];
    float org[3], spc[3];
    int N;
    int tiles;  // tiles per map side (N / tile side)
    int ts;     // tile side: min(N, kBakeTile)
};

// Octahedral (u, v) of a direction, z fold axis, with the correctly rounded division:
// q = d / (|dx| + |dy| + |dz|); lower hemisphere folded over the diagonals.
__device__ __forceinline__ void bake_oct(float x, float y, float z, float &u, float &v) {
    float L = (fabsf(x) + fabsf(y)) + fabsf(z);
    float qx = x / L, qy = y / L, qz = z / L;
    float sx = qx >= 0.0f ? 1.0f : -1.0f, sy = qy >= 0.0f ? 1.0f : -1.0f;
    u = qz >= 0.0f ? qx : (1.0f - fabsf(qy)) * sx;
    v = qz >= 0.0f ? qy : (1.0f - fabsf(qx)) * sy;
}

}  // namespace pt
