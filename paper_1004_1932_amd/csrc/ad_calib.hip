/*
 * Measurement support: the vector-ALU issue rate of the FP32 Oseen pair
 * term's own instruction mix, and the shader clock under that load (the
 * longest work-group life in shader cycles over the kernel's duration).
 *
 * Every lane evaluates pair terms of one target against 8 sources held in
 * registers (no memory traffic inside the loop), exactly as the pair loops
 * do (difference, r^2 by FMA, hardware reciprocal square root, then the
 * three-component Oseen term accumulated with FMAs; with hi/lo positions the
 * difference takes the second three subtractions and three additions). The
 * target (with hi/lo positions, its lo part too) moves by a tiny step after
 * every 8 terms so that nothing is loop invariant. kind 1 replaces the term by 8 independent FMA chains, the plain
 * FMA issue rate. No packed FP32 instructions are used (the build forbids
 * them), so the rates are those of the single-issue FP32 path.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ad.h"

namespace {

__device__ __forceinline__ void term(float hx, float hy, float hz, float lx, float ly, float lz, float sx, float sy,
                                     float sz, float tx, float ty, float tz, float fx, float fy, float fz, bool hilo,
                                     float& px, float& py, float& pz) {
    float rx, ry, rz;
    if (hilo) {
        rx = (hx - sx) + (lx - tx);
        ry = (hy - sy) + (ly - ty);
        rz = (hz - sz) + (lz - tz);
    } else {
        rx = hx - sx;
        ry = hy - sy;
        rz = hz - sz;
    }
    const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
    const float ir = __builtin_amdgcn_rsqf(r2);
    const float fr = __builtin_fmaf(rz, fz, __builtin_fmaf(ry, fy, rx * fx));
    const float ir2 = ir * ir;
    const float tt = fr * ir2;
    px = __builtin_fmaf(ir, __builtin_fmaf(tt, rx, fx), px);
    py = __builtin_fmaf(ir, __builtin_fmaf(tt, ry, fy), py);
    pz = __builtin_fmaf(ir, __builtin_fmaf(tt, rz, fz), pz);
}

template <int KIND>
__global__ __launch_bounds__(256) void k_valu_rate(int iters, float seed, float* __restrict__ sink,
                                                   long long* __restrict__ clk) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const long long c0 = clock64();
    const float b = seed + 1e-3f * (float)(threadIdx.x & 63);
    float sx[8], sy[8], sz[8], fx[8], fy[8], fz[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        sx[k] = b + 3.0f * k;
        sy[k] = b - 2.0f * k;
        sz[k] = 0.5f * b + k;
        fx[k] = 0.1f * k;
        fy[k] = -0.2f * k + b;
        fz[k] = 0.3f;
    }
    float hx = 100.f + b, hy = -50.f + b, hz = 25.f;
    float lx = 1e-6f * b, ly = -1e-6f, lz = 2e-6f;
    float px = 0.f, py = 0.f, pz = 0.f;
    float qx[4] = {0.f, 0.f, 0.f, 0.f}, qy[4] = {0.f, 0.f, 0.f, 0.f}, qz[4] = {0.f, 0.f, 0.f, 0.f};
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = b + k;
    for (int it = 0; it < iters; ++it) {
        if (KIND == 1) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = __builtin_fmaf(a[k], 0.999f, 1e-3f);
        } else if (KIND == 3) {
            /* the same terms into four independent accumulators */
#pragma unroll
            for (int k = 0; k < 8; ++k)
                term(hx, hy, hz, lx, ly, lz, sx[k], sy[k], sz[k], 0.f, 0.f, 0.f, fx[k], fy[k], fz[k], false,
                     qx[k & 3], qy[k & 3], qz[k & 3]);
            hx += 1e-4f;
            hy += 1e-4f;
            hz += 1e-4f;
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                term(hx, hy, hz, lx, ly, lz, sx[k], sy[k], sz[k], 1e-7f * k, -2e-7f, 3e-7f * k, fx[k], fy[k], fz[k], KIND == 2, px,
                     py, pz);
            hx += 1e-4f;
            hy += 1e-4f;
            hz += 1e-4f;
            if (KIND == 2) { /* the lo parts move too, so no difference is loop invariant */
                lx += 1e-12f;
                ly += 1e-12f;
                lz += 1e-12f;
            }
        }
    }
    float out = px + py + pz;
#pragma unroll
    for (int k = 0; k < 4; ++k) out += qx[k] + qy[k] + qz[k];
#pragma unroll
    for (int k = 0; k < 8; ++k) out += a[k];
    sink[g] = out;
    __syncthreads();
    if (threadIdx.x == 0) {
        /* shader cycles of this work-group's life: the longest, and the sum */
        const unsigned long long cyc = (unsigned long long)(clock64() - c0);
        atomicMax(reinterpret_cast<unsigned long long*>(&clk[0]), cyc);
        atomicAdd(reinterpret_cast<unsigned long long*>(&clk[1]), cyc);
    }
}

}  // namespace

/* kind 0: Oseen term with single-float positions, 1: FMA chains, 2: Oseen
 * term with hi/lo positions, 3: kind 0 with four accumulators. blocks
 * work-groups of 256 threads, iters loop trips of 8 terms (or 8 FMAs) per
 * thread; sink: device [blocks*256] floats; clk: device [2], zeroed by the
 * caller: the longest life of a work-group in shader cycles, and the sum
 * over work-groups. Asynchronous. */
extern "C" int ad_valu_probe(int32_t kind, int32_t blocks, int32_t iters, float* sink, long long* clk,
                             void* stream) {
    if (blocks < 1 || iters < 1 || !sink || !clk || kind < 0 || kind > 3) return AD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (kind == 0)
        hipLaunchKernelGGL(k_valu_rate<0>, dim3(blocks), dim3(256), 0, s, iters, 0.25f, sink, clk);
    else if (kind == 1)
        hipLaunchKernelGGL(k_valu_rate<1>, dim3(blocks), dim3(256), 0, s, iters, 0.25f, sink, clk);
    else if (kind == 2)
        hipLaunchKernelGGL(k_valu_rate<2>, dim3(blocks), dim3(256), 0, s, iters, 0.25f, sink, clk);
    else
        hipLaunchKernelGGL(k_valu_rate<3>, dim3(blocks), dim3(256), 0, s, iters, 0.25f, sink, clk);
    return hipGetLastError() == hipSuccess ? AD_OK : AD_EDEVICE;
}
