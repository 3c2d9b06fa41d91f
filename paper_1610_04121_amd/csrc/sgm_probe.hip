// Measurement helper behind sgm_debug_valu_probe.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "sgm_plan.h"

namespace sgm {
namespace {

// Packed-u16 VALU throughput probe (a measurement of the ALU peak the
// aggregation's instruction counts are compared with): every lane runs
// `iters` rounds of 8 independent (v_pk_add_u16, v_pk_min_u16) pairs, so a
// wave issues 16 VALU instructions per round with no dependent pair closer
// than 8 instructions.  The result only reaches memory in the (never taken)
// case that it equals a constant, so the stores cost nothing but keep the
// work.
typedef unsigned short valu_u16x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void valu_probe_kernel(int iters, uint32_t* sink) {
    valu_u16x2 a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        a[j] = valu_u16x2{(unsigned short)(threadIdx.x + j), (unsigned short)(blockIdx.x + 3 * j)};
    const valu_u16x2 inc = {1, 3}, cap = {0x7FF0, 0x7FE0};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = __builtin_elementwise_min(a[j] + inc, cap);
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r ^= (uint32_t)a[j].x | ((uint32_t)a[j].y << 16);
    if (r == 0x9E3779B9u) sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// Latency probes: one dependent chain per lane, 16 instructions per round.
// MODE 1: packed u16 add then min (VALU to VALU); MODE 2: u32 min whose
// operand comes through a DPP row_mirror (VALU to DPP); MODE 3: a
// permlane16 swap and a min (the cross-row step of a 32-lane group
// minimum, 8 rounds of the pair per round of 16).
template <int MODE>
__global__ __launch_bounds__(256) void valu_latency_kernel(int iters, uint32_t* sink) {
    uint32_t v = threadIdx.x * 2654435761u + blockIdx.x;
    const valu_u16x2 inc = {1, 3}, cap = {0x7FF0, 0x7FE0};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if constexpr (MODE == 1) {
                const valu_u16x2 a = __builtin_bit_cast(valu_u16x2, v) + inc;
                v = __builtin_bit_cast(uint32_t, __builtin_elementwise_min(a, cap));
            } else if constexpr (MODE == 2) {
                v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true)) + 1u;
            } else {
                const auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);
                v = min((uint32_t)sw[0], (uint32_t)sw[1]) + 1u;
            }
        }
    }
    if (v == 0x9E3779B9u) sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = v;
}

}  // namespace

hipError_t launch_valu_probe(int blocks, int iters, uint32_t* sink, hipStream_t stream) {
    hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(256), 0, stream, iters, sink);
    return hipGetLastError();
}

hipError_t launch_valu_latency_probe(int mode, int blocks, int iters, uint32_t* sink, hipStream_t stream) {
    auto k = mode == 1 ? valu_latency_kernel<1> : (mode == 2 ? valu_latency_kernel<2> : valu_latency_kernel<3>);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, stream, iters, sink);
    return hipGetLastError();
}

}  // namespace sgm
