// Consistency regularizer of the extended misfit (Model extension, eq.(8) second term;
// Source zone of influence, eqs.(11)-(12)), value and gradient, pointwise in space.
//
// At one point with per-shot values m_s, weights b_s and sinkhole flags k_s:
//   B_s   = sum_{i != s} b_i                         (eq.(11) denominator)
//   (Wm)_s = b_s m_s + (1 - b_s)(sum_i b_i m_i - b_s m_s) / B_s   if k_s and B_s > 0
//          = m_s                                                   otherwise
//   b'_s  = 1 if k_s else b_s;  mbar = sum b'_s (Wm)_s / sum b'_s  (eq.(12), S_w)
//   y_s   = (Wm)_s - mbar                            ((I - S^T S_w) W m)
//   phi  += 1/2 eta^2 sum_s y_s^2
//   z_s   = y_s - b'_s / (sum b') * sum_i y_i        ((I - S^T S_w)^T y)
//   (W^T z)_i = W_ii z_i + b_i (T - [k_i, B_i > 0] (1 - b_i) z_i / B_i),
//               T = sum_{s: k_s, B_s > 0} (1 - b_s) z_s / B_s
//   g_i  += eta^2 (W^T z)_i
// W is never formed: each of the five passes is O(Ns). The arithmetic is FP64 because
// y_s is a small difference of O(1e3) model values; the kernel is bound by the Ns-fold
// reads of m~, b and the sinkhole flags, not by the FP64 rate.
#include "efwi_internal.h"

namespace efwi {
namespace {

constexpr int RB = 256;

__global__ __launch_bounds__(RB) void k_regularizer(int ns, long npts, long plane, const float* __restrict__ m,
                                                    const float* __restrict__ b,
                                                    const unsigned char* __restrict__ sink, double eta2,
                                                    float* __restrict__ g, double* __restrict__ partial) {
  __shared__ double sh[RB];
  double phi = 0.0;
  for (long p = blockIdx.x * (long)RB + threadIdx.x; p < npts; p += (long)gridDim.x * RB) {
    double bsum = 0.0;
    for (int s = 0; s < ns; ++s) bsum += b[(long)s * npts + p];
    double bpsum = 0.0;
    for (int s = 0; s < ns; ++s) bpsum += sink[(long)s * npts + p] ? 1.0 : (double)b[(long)s * npts + p];
    if (!(bpsum > 0.0)) continue;
    for (int k = 0; k < 3; ++k) {
      auto mv = [&](int s) { return (double)m[((long)s * 3 + k) * plane + p]; };
      double A = 0.0;
      for (int s = 0; s < ns; ++s) A += (double)b[(long)s * npts + p] * mv(s);
      auto wm = [&](int s) {
        const double bs = b[(long)s * npts + p];
        const double Bs = bsum - bs;
        const double ms = mv(s);
        if (sink[(long)s * npts + p] && Bs > 0.0) return bs * ms + (1.0 - bs) * (A - bs * ms) / Bs;
        return ms;
      };
      double num = 0.0;
      for (int s = 0; s < ns; ++s) {
        const double bp = sink[(long)s * npts + p] ? 1.0 : (double)b[(long)s * npts + p];
        num += bp * wm(s);
      }
      const double mbar = num / bpsum;
      double Y = 0.0;
      for (int s = 0; s < ns; ++s) {
        const double y = wm(s) - mbar;
        Y += y;
        phi += y * y;
      }
      auto zf = [&](int s) {
        const double bp = sink[(long)s * npts + p] ? 1.0 : (double)b[(long)s * npts + p];
        return (wm(s) - mbar) - bp / bpsum * Y;
      };
      double T = 0.0;
      for (int s = 0; s < ns; ++s) {
        const double bs = b[(long)s * npts + p];
        const double Bs = bsum - bs;
        if (sink[(long)s * npts + p] && Bs > 0.0) T += (1.0 - bs) * zf(s) / Bs;
      }
      for (int s = 0; s < ns; ++s) {
        const double bs = b[(long)s * npts + p];
        const double Bs = bsum - bs;
        const double z = zf(s);
        const bool in = sink[(long)s * npts + p] && Bs > 0.0;
        const double wz = (in ? bs : 1.0) * z + bs * (T - (in ? (1.0 - bs) * z / Bs : 0.0));
        float* gp = g + ((long)s * 3 + k) * plane + p;
        *gp = (float)((double)*gp + eta2 * wz);
      }
    }
  }
  sh[threadIdx.x] = phi;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_sum_partials(const double* partial, int n, double scale, double* out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) a += partial[k];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = scale * sh[0];
}

}  // namespace

int regularizer_blocks(long npts) {
  long nb = (npts + RB - 1) / RB;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  return (int)nb;
}

hipError_t launch_regularizer(int ns, long npts, long plane, const float* m_ext, const float* b,
                              const unsigned char* sink, float eta, float* g_ext, double* partial, int nblocks,
                              double* phi, hipStream_t st) {
  const double eta2 = (double)eta * (double)eta;
  k_regularizer<<<nblocks, RB, 0, st>>>(ns, npts, plane, m_ext, b, sink, eta2, g_ext, partial);
  k_sum_partials<<<1, 256, 0, st>>>(partial, nblocks, 0.5 * eta2, phi);
  return hipGetLastError();
}

}  // namespace efwi
