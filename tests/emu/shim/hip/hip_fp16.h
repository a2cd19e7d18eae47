// FP16 pairs for the CPU emulation of the amqft kernels (test infrastructure).
#pragma once
#include "hip_runtime.h"
struct alignas(4) __half2 {
    _Float16 x, y;
};
inline float2 __half22float2(__half2 h) { return {(float)h.x, (float)h.y}; }
inline __half2 __float22half2_rn(float2 f) { return {(_Float16)f.x, (_Float16)f.y}; }
