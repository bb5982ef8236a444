// D3Q19 velocity set and small device helpers of the gfx950 library.
//
// Velocities (Sec. 2.1 uses D3Q19: 19 discrete velocities on a cubic
// lattice): rest, the 6 face neighbours, the 12 edge neighbours; the
// opposite of odd i is i+1.  Rest weights 1/3, 1/18, 1/36.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;

__host__ __device__ constexpr int cx(int i) {
    constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

template <class R>
__host__ __device__ constexpr R wgt(int i) {
    return i == 0 ? R(1) / R(3) : (i <= 6 ? R(1) / R(18) : R(1) / R(36));
}

// Workgroups are handed to the 8 XCDs round-robin (workgroup b runs on XCD
// b % 8).  Renumber them so each XCD walks one contiguous range of tiles:
// neighbouring tiles then share an L2 (their partial-line stores of the
// x-shifted populations merge there) and each L2 sees a compact footprint.
// Where a workgroup holds whole x rows the natural order is faster (one
// compact address range for the whole chip), and the collide-stream passes
// skip the renumbering.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, k = b & 7, i = b >> 3;
    return (k < r) ? k * (q + 1) + i : r * (q + 1) + (k - r) * q + i;
}

__device__ __forceinline__ int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Wave-level (64 lanes) then block-level sum of doubles, fixed order so the
// result does not depend on scheduling.  `red` holds nwaves*K doubles.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *red) {
#pragma unroll
    for (int k = 0; k < K; k++) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    }
    const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) red[wave * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) {
        double s = 0.0;
        for (int w = 0; w < nw; w++) s += red[w * K + k];
        v[k] = s;
    }
    __syncthreads();
}

}  // namespace lbm
