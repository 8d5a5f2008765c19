// Frame scheduling of the persistent decode grids (device code only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fwbf {

// Workgroups are dispatched to the 8 XCDs of the device round-robin, so
// workgroup b runs on XCD b % 8.  XCD x owns the contiguous frame range
// [x*Fx, (x+1)*Fx) and its workgroups stride through it: neighbouring frames,
// which share cache lines whenever a frame row is not a multiple of the line
// size, are then read (and their outputs written) through one L2 instead of
// two.  Falls back to a plain grid stride when the grid is not a multiple of 8.
struct FrameRange {
    int64_t first, end, step;
};

__device__ __forceinline__ FrameRange xcd_frames(int64_t F)
{
    constexpr int NX = 8;
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (G % NX != 0 || F < G) return FrameRange{b, F, G};
    const int64_t x = b % NX, per = G / NX;
    const int64_t Fx = (F + NX - 1) / NX;
    const int64_t end = (x + 1) * Fx < F ? (x + 1) * Fx : F;
    return FrameRange{x * Fx + b / NX, end, per};
}

}  // namespace fwbf

namespace fwbf {

// The same ranges when every workgroup runs W independent wavefronts, each
// decoding its own frames: wavefront w of workgroup b is worker b*W + w
// (all W on the XCD of b).
__device__ __forceinline__ FrameRange xcd_frames_waves(int64_t F, int W, int w)
{
    constexpr int NX = 8;
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (G % NX != 0 || F < G * W) return FrameRange{b * W + w, F, G * W};
    const int64_t x = b % NX, per = G / NX;
    const int64_t Fx = (F + NX - 1) / NX;
    const int64_t end = (x + 1) * Fx < F ? (x + 1) * Fx : F;
    return FrameRange{x * Fx + (b / NX) * W + w, end, per * W};
}

}  // namespace fwbf

namespace fwbf {

// A uniform value the compiler must take as defined here: tests of kernel
// arguments made inside a loop from such a copy stay scalar compares at
// their use, instead of being hoisted out of the loop as 64-bit lane masks
// that stay live (and, with enough of them, spill) for the whole loop.
__device__ __forceinline__ int fresh(int v)
{
    asm volatile("" : "+s"(v));
    return v;
}
__device__ __forceinline__ float fresh(float v)
{
    asm volatile("" : "+s"(v));
    return v;
}
template <typename T>
__device__ __forceinline__ T *fresh(T *v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// Product of the low 24 bits of a and b (v_mul_u32_u24, full rate), as an
// unsigned 32-bit value: HIP's __umul24 returns int, which would turn a
// product at or above 2^31 negative under shifts and comparisons.
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) { return (uint32_t)__umul24(a, b); }

}  // namespace fwbf
