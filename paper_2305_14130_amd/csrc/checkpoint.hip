// 16-bit wavefield checkpoints with per-field max-abs scaling.
//
// A checkpoint holds one shot's forward state block (2D: the five padded wavefields and the
// eight CPML strip arrays; 3D: nine and eighteen). Each field gets one FP32 scale per
// snapshot:
//   FP16: codes x / s, s = max|x| / 2^14 (largest code 16384 < 65504; values down to
//         max|x| 2^-28 stay normal),
//   BF16: codes x / s, s = max|x| (BF16 keeps FP32's exponent range).
// Both round to nearest even; a zero field keeps s = 0 and decodes to zeros.
// Slot layout: CKPT_HEADER bytes of scales (one float per field, padded), then one 16-bit
// code per element of the state block, in the block's element order.
#include <hip/hip_fp16.h>

#include "efwi_internal.h"

namespace efwi {
namespace {

constexpr int CB = 256;

__device__ __forceinline__ float field_scale(unsigned int maxbits, int codec) {
  const float mx = __uint_as_float(maxbits);
  return codec == CKPT_CODEC_FP16 ? mx * (1.0f / 16384.0f) : mx;
}

// Max |x| of each field: block reduction, then an integer atomic max on the bit pattern of
// the (non-negative) float, which orders like the value and makes the result exact and
// independent of the reduction order.
__global__ __launch_bounds__(CB) void k_maxabs(const float* __restrict__ state, CkptFields f,
                                              unsigned int* __restrict__ maxbits) {
  __shared__ float sh[CB];
  const int fld = blockIdx.y;
  const float* p = state + f.off[fld];
  const long len = f.len[fld];
  float m = 0.0f;
  for (long e = (long)blockIdx.x * CB + threadIdx.x; e < len; e += (long)gridDim.x * CB) m = fmaxf(m, fabsf(p[e]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = CB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0] > 0.0f) atomicMax(maxbits + fld, __float_as_uint(sh[0]));
}

__device__ __forceinline__ unsigned short to_bf16(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  return (unsigned short)(u >> 16);
}

__global__ __launch_bounds__(CB) void k_encode(const float* __restrict__ state, CkptFields f,
                                              const unsigned int* __restrict__ maxbits, float* __restrict__ scales,
                                              unsigned short* __restrict__ codes, int codec) {
  const int fld = blockIdx.y;
  const float s = field_scale(maxbits[fld], codec);
  if (blockIdx.x == 0 && threadIdx.x == 0) scales[fld] = s;
  const float* p = state + f.off[fld];
  unsigned short* q = codes + f.off[fld];
  const long len = f.len[fld];
  for (long e = (long)blockIdx.x * CB + threadIdx.x; e < len; e += (long)gridDim.x * CB) {
    const float v = s > 0.0f ? p[e] / s : 0.0f;
    q[e] = codec == CKPT_CODEC_FP16 ? __half_as_ushort(__float2half_rn(v)) : to_bf16(v);
  }
}

__global__ __launch_bounds__(CB) void k_decode(float* __restrict__ state, CkptFields f,
                                              const float* __restrict__ scales,
                                              const unsigned short* __restrict__ codes, int codec) {
  const int fld = blockIdx.y;
  const float s = scales[fld];
  float* p = state + f.off[fld];
  const unsigned short* q = codes + f.off[fld];
  const long len = f.len[fld];
  for (long e = (long)blockIdx.x * CB + threadIdx.x; e < len; e += (long)gridDim.x * CB) {
    const unsigned short c = q[e];
    const float v = codec == CKPT_CODEC_FP16 ? __half2float(__ushort_as_half(c)) : __uint_as_float((unsigned int)c << 16);
    p[e] = v * s;
  }
}

dim3 grid_for(const CkptFields& f) {
  long mx = 1;
  for (int k = 0; k < f.n; ++k) mx = f.len[k] > mx ? f.len[k] : mx;
  long nb = (mx + 4L * CB - 1) / (4L * CB);
  if (nb > 2048) nb = 2048;
  return dim3((unsigned)nb, (unsigned)f.n);
}

}  // namespace

hipError_t launch_ckpt_encode(const float* state, const CkptFields& f, unsigned int* maxbits, void* slot, int codec,
                              hipStream_t st) {
  hipError_t e = hipMemsetAsync(maxbits, 0, f.n * sizeof(unsigned int), st);
  if (e != hipSuccess) return e;
  const dim3 g = grid_for(f);
  k_maxabs<<<g, CB, 0, st>>>(state, f, maxbits);
  float* scales = static_cast<float*>(slot);
  unsigned short* codes = reinterpret_cast<unsigned short*>(static_cast<unsigned char*>(slot) + CKPT_HEADER);
  k_encode<<<g, CB, 0, st>>>(state, f, maxbits, scales, codes, codec);
  return hipGetLastError();
}

hipError_t launch_ckpt_decode(float* state, const CkptFields& f, const void* slot, int codec, hipStream_t st) {
  const float* scales = static_cast<const float*>(slot);
  const unsigned short* codes =
      reinterpret_cast<const unsigned short*>(static_cast<const unsigned char*>(slot) + CKPT_HEADER);
  k_decode<<<grid_for(f), CB, 0, st>>>(state, f, scales, codes, codec);
  return hipGetLastError();
}

}  // namespace efwi
