// Measurement probe: the throughput of float atomics in the access pattern
// of the render backward's gradient flush, so that the backward's atomic
// rate can be set against what the memory system sustains for that pattern.
//
// Each wave64 issues `iters` atomic add instructions without return value.
// In each, lanes 0-7 add to the 8 corner gradients of one voxel (a 32-byte
// row) and lanes 8-10 to its 3 colour gradients (a 12-byte row), as the
// backward does after its wave reduction; the voxel is drawn per instruction
// from a per-wave linear congruential sequence, uniform over n_rows.
#include "svr_internal.h"

namespace svr {

__global__ __launch_bounds__(kBlock) void k_atomic_probe(float* __restrict__ corner,
                                                         float* __restrict__ colour,
                                                         uint32_t n_rows, int iters) {
  const uint32_t wave = (blockIdx.x * (uint32_t)kBlock + threadIdx.x) >> 6;
  const int lane = (int)(threadIdx.x & 63u);
  uint32_t h = wave * 2654435761u + 0x9e3779b9u;
  for (int it = 0; it < iters; ++it) {
    h = h * 1664525u + 1013904223u;
    const uint32_t v = (uint32_t)(((uint64_t)h * n_rows) >> 32);
    float* p = lane < 8 ? corner + (size_t)v * 8 + lane : colour + (size_t)v * 3 + (lane - 8);
    if (lane < 11) atomicAdd(p, 1.0f);
  }
}

hipError_t launch_atomic_probe(float* corner, float* colour, int64_t n_rows, int64_t n_waves,
                               int iters, hipStream_t s) {
  const int64_t blocks = (n_waves * 64 + kBlock - 1) / kBlock;
  SVR_LAUNCH("atomic_probe", k_atomic_probe, dim3((unsigned)blocks), dim3(kBlock), 0, s, corner,
             colour, (uint32_t)n_rows, iters);
  return hipGetLastError();
}

}  // namespace svr
