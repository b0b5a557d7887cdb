// Measurement aid: kernels that run one kind of arithmetic at full rate, so
// the achievable peaks of this GPU can be measured beside the path's kernels
// (FP32 and FP64 vector fused multiply-adds, BF16 matrix-core products).
// They compute nothing of the method.
#include "md_common.h"

namespace md {

constexpr int kProbeChains = 8;   // independent dependency chains per thread

__device__ __forceinline__ float fma_t(float v, float a, float b) { return __builtin_fmaf(v, a, b); }
__device__ __forceinline__ double fma_t(double v, double a, double b) { return __builtin_fma(v, a, b); }

template <typename T>
__global__ __launch_bounds__(kBlock) void k_probe_fma(int64_t iters, T a, T b, T *out)
{
    T v[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) v[c] = T(threadIdx.x + c);
    for (int64_t k = 0; k < iters; ++k)
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) v[c] = fma_t(v[c], a, b);
    T s = 0;
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) s += v[c];
    if (s == T(-1.2345)) out[0] = s;   // keeps the chains alive; never true for these inputs
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_probe_mfma(int64_t iters, float *out)
{
    const float base = float(threadIdx.x % 7) * 0.125f;
    const bf16x8_t a = __builtin_convertvector(
        (f32x4_t{base, 0.5f, 0.25f, 1.0f}).xyzwxyzw, bf16x8_t);
    f32x4_t acc[4] = {};
    for (int64_t k = 0; k < iters; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, acc[c], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (s == -1.2345f) out[0] = s;
}

int probe(int32_t kind, int64_t iters, int32_t blocks, void *out, hipStream_t s)
{
    switch (kind) {
    case MD_PROBE_FMA_F32:
        hipLaunchKernelGGL(k_probe_fma<float>, dim3(blocks), dim3(kBlock), 0, s, iters, 0.999f, 1e-3f,
                           static_cast<float *>(out));
        break;
    case MD_PROBE_FMA_F64:
        hipLaunchKernelGGL(k_probe_fma<double>, dim3(blocks), dim3(kBlock), 0, s, iters, 0.999, 1e-3,
                           static_cast<double *>(out));
        break;
    case MD_PROBE_MFMA_BF16:
        hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(kBlock), 0, s, iters, static_cast<float *>(out));
        break;
    default:
        return MD_ERR_ARG;
    }
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

}  // namespace md

extern "C" int md_probe(int32_t kind, int64_t iters, int32_t blocks, void *out, void *stream)
{
    if (iters < 1 || blocks < 1 || !out) return MD_ERR_ARG;
    return md::probe(kind, iters, blocks, out, static_cast<hipStream_t>(stream));
}
