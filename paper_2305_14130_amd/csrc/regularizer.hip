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
    // Passes over the sources with the three parameters together; per source the sinkhole
    // mix (in s's sinkhole and other weights present) and 1 / B_s are formed once a pass.
    // (W m)_s,k = mix ? b_s m_s,k + (1 - b_s)(A_k - b_s m_s,k) / B_s : m_s,k
    auto mv = [&](int s, int k) { return (double)m[((long)s * 3 + k) * plane + p]; };
    double bsum = 0.0, bpsum = 0.0, A[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < ns; ++s) {
      const double bs = b[(long)s * npts + p];
      bsum += bs;
      bpsum += sink[(long)s * npts + p] ? 1.0 : bs;
      for (int k = 0; k < 3; ++k) A[k] += bs * mv(s, k);
    }
    if (!(bpsum > 0.0)) continue;
    struct Src {
      double bs, bp, inv;
      bool mix;
    };
    auto src = [&](int s) {
      Src r;
      r.bs = b[(long)s * npts + p];
      const double Bs = bsum - r.bs;
      const bool in = sink[(long)s * npts + p] != 0;
      r.mix = in && Bs > 0.0;
      r.bp = in ? 1.0 : r.bs;
      r.inv = r.mix ? 1.0 / Bs : 0.0;
      return r;
    };
    auto wm = [&](const Src& q, int s, int k) {
      const double ms = mv(s, k);
      return q.mix ? q.bs * ms + (1.0 - q.bs) * (A[k] - q.bs * ms) * q.inv : ms;
    };
    // mean over the useful components: mbar_k = sum_s b'_s (W m)_s,k / sum b'
    double mbar[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < ns; ++s) {
      const Src q = src(s);
      for (int k = 0; k < 3; ++k) mbar[k] += q.bp * wm(q, s, k);
    }
    for (int k = 0; k < 3; ++k) mbar[k] /= bpsum;
    // y = W m - mbar: its sum over sources and the penalty
    double Y[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < ns; ++s) {
      const Src q = src(s);
      for (int k = 0; k < 3; ++k) {
        const double y = wm(q, s, k) - mbar[k];
        Y[k] += y;
        phi += y * y;
      }
    }
    // z_s = y_s - b'_s / sum b' * sum y; T_k = sum over mixing sources of (1 - b_s) z_s / B_s
    auto zf = [&](const Src& q, int s, int k) { return (wm(q, s, k) - mbar[k]) - q.bp / bpsum * Y[k]; };
    double T[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < ns; ++s) {
      const Src q = src(s);
      if (!q.mix) continue;
      for (int k = 0; k < 3; ++k) T[k] += (1.0 - q.bs) * zf(q, s, k) * q.inv;
    }
    // g_s += eta^2 W^T z
    for (int s = 0; s < ns; ++s) {
      const Src q = src(s);
      for (int k = 0; k < 3; ++k) {
        const double z = zf(q, s, k);
        const double wz = (q.mix ? q.bs : 1.0) * z + q.bs * (T[k] - (q.mix ? (1.0 - q.bs) * z * q.inv : 0.0));
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

// ---------------------------------------------------------------------------------------
// Zone of influence of one source (Source zone of influence, eq.(10)), pointwise:
//   b = (cos^n(pi r / 2) - ln nu) / (1 - ln nu),  r = max(r_out, r_sink) in [0, 1]
//   r_out  = (Euclidean distance to the active box) / taper, capped at 1 (a step if taper 0)
//   r_sink = 1 - d inside the sinkhole d < 1, d = sqrt(dp^T C^-1 dp) (Mahalanobis distance
//            to the source), 0 outside; sink = (d^2 < 1)
// FP64, with the squared distance summed in a fixed order and no contraction, so that the
// sinkhole flag (an integer decided by floating point) is reproducible.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_zoi(long npts, int ny, int nx, int xblocks, double dz, double dy, double dx,
                                            int three, ZoiBatch zb, float* __restrict__ b,
                                            unsigned char* __restrict__ sink) {
#pragma clang fp contract(off)
  // one zone per blockIdx.y; blockIdx.x = row (i, k) x block of RB columns
  const ZoiArgs& a = zb.z[blockIdx.y];
  const int row = (int)(blockIdx.x / (unsigned)xblocks), j = (int)(blockIdx.x - (unsigned)row * xblocks) * RB + threadIdx.x;
  if (j < nx) {
    const int i = row / ny, k = row - i * ny;
    const long p = (long)row * nx + j;
    const double z = (double)i * dz, y = (double)k * dy, x = (double)j * dx;
    const double ez = fmax(fmax(a.box[0] - z, z - a.box[1]), 0.0);
    const double ex = fmax(fmax(a.box[4] - x, x - a.box[5]), 0.0);
    double e2 = ez * ez + ex * ex;
    if (three) {
      const double ey = fmax(fmax(a.box[2] - y, y - a.box[3]), 0.0);
      e2 = e2 + ey * ey;
    }
    const double e = sqrt(e2);
    const double r_out = a.taper > 0.0 ? fmin(e / a.taper, 1.0) : (e > 0.0 ? 1.0 : 0.0);
    const double pz = z - a.src[0], px = x - a.src[2];
    // icov = (zz, yy, xx, zy, zx, yx)
    double d2 = (a.icov[0] * pz) * pz;
    d2 = d2 + (a.icov[2] * px) * px;
    d2 = d2 + ((2.0 * a.icov[4]) * pz) * px;
    if (three) {
      const double py = y - a.src[1];
      d2 = d2 + (a.icov[1] * py) * py;
      d2 = d2 + ((2.0 * a.icov[3]) * pz) * py;
      d2 = d2 + ((2.0 * a.icov[5]) * py) * px;
    }
    const bool in = d2 < 1.0;
    const double r_sink = in ? 1.0 - sqrt(d2) : 0.0;
    const double r = fmax(r_out, r_sink);
    // r = 0 (the active part) gives exactly 1: skip the transcendental functions there
    const long q = (long)blockIdx.y * npts + p;
    float w = 1.0f;
    if (r > 0.0) {
      const double ln = log(a.nu), den = 1.0 - ln;
      w = (float)((pow(cos(0.5 * M_PI * r), a.n) - ln) / den);
    }
    b[q] = w;
    sink[q] = in ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------------------
// Final physical model m = S_w W m~ (eq.(9)), pointwise, with W and S_w as in k_regularizer
// (0 where sum b' = 0: no source is useful there).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_final_model(int ns, long npts, long plane, const float* __restrict__ m,
                                                    const float* __restrict__ b,
                                                    const unsigned char* __restrict__ sink,
                                                    float* __restrict__ out) {
  for (long p = blockIdx.x * (long)RB + threadIdx.x; p < npts; p += (long)gridDim.x * RB) {
    // first pass: sum b, sum b' and A_k = sum_s b_s m_s,k for the three parameters
    double bsum = 0.0, bpsum = 0.0, A[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < ns; ++s) {
      const double bs = b[(long)s * npts + p];
      bsum += bs;
      bpsum += sink[(long)s * npts + p] ? 1.0 : bs;
      for (int k = 0; k < 3; ++k) A[k] += bs * (double)m[((long)s * 3 + k) * plane + p];
    }
    if (!(bpsum > 0.0)) {
      for (int k = 0; k < 3; ++k) out[(long)k * plane + p] = 0.0f;
      continue;
    }
    // second pass: (W m)_s (one division per source) weighted by b'_s
    double num[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < ns; ++s) {
      const double bs = b[(long)s * npts + p];
      const double Bs = bsum - bs;
      const bool in = sink[(long)s * npts + p] != 0;
      const bool mix = in && Bs > 0.0;
      const double inv = mix ? 1.0 / Bs : 0.0, wp = in ? 1.0 : bs;
      for (int k = 0; k < 3; ++k) {
        const double ms = m[((long)s * 3 + k) * plane + p];
        const double wm = mix ? bs * ms + (1.0 - bs) * (A[k] - bs * ms) * inv : ms;
        num[k] += wp * wm;
      }
    }
    for (int k = 0; k < 3; ++k) out[(long)k * plane + p] = (float)(num[k] / bpsum);
  }
}

// Extension along groups of shots: one shot's FP64 gradient sums G [3][nz][ny][cp] (its
// window) rounded to FP32 and added into its group's component of the extended gradient,
// out [3][...] with the full model's plane, row strides and the window origin.
__global__ __launch_bounds__(RB) void k_add_gradient(const double* __restrict__ G, long cells, int cp, int nz, int ny,
                                                     int nx, float* __restrict__ out, long mplane, long mrow,
                                                     long mslab, int z0, int y0, int x0) {
  const long n = (long)nz * ny * nx;
  for (long q = blockIdx.x * (long)RB + threadIdx.x; q < n; q += (long)gridDim.x * RB) {
    const int j = (int)(q % nx);
    const long r = q / nx;
    const int k = (int)(r % ny), i = (int)(r / ny);
    const long c = ((long)i * ny + k) * cp + j;
    const long o = (long)(z0 + i) * mslab + (long)(y0 + k) * mrow + (x0 + j);
    for (int f = 0; f < 3; ++f) out[f * mplane + o] += (float)G[f * cells + c];
  }
}

}  // namespace

hipError_t launch_zoi(int three, int count, long npts, int nz, int ny, int nx, double dz, double dy, double dx,
                      const ZoiBatch& zb, float* b, unsigned char* sink, hipStream_t st) {
  if (count < 1 || count > ZOI_BATCH || npts <= 0) return count == 0 ? hipSuccess : hipErrorInvalidValue;
  const int xblocks = (nx + RB - 1) / RB;
  if ((long)nz * ny * xblocks > 0x7fffffffL) return hipErrorInvalidValue;
  k_zoi<<<dim3((unsigned)((long)nz * ny * xblocks), (unsigned)count), RB, 0, st>>>(npts, ny, nx, xblocks, dz, dy, dx,
                                                                                   three, zb, b, sink);
  return hipGetLastError();
}

hipError_t launch_final_model(int ns, long npts, const float* m_ext, const float* b, const unsigned char* sink,
                              float* m_out, hipStream_t st) {
  k_final_model<<<regularizer_blocks(npts), RB, 0, st>>>(ns, npts, npts, m_ext, b, sink, m_out);
  return hipGetLastError();
}

hipError_t launch_add_gradient(const double* G, long cells, int cp, int nz, int ny, int nx, float* out, long mplane,
                               long mrow, long mslab, int z0, int y0, int x0, hipStream_t st) {
  const long n = (long)nz * ny * nx;
  if (n <= 0) return hipSuccess;
  k_add_gradient<<<regularizer_blocks(n), RB, 0, st>>>(G, cells, cp, nz, ny, nx, out, mplane, mrow, mslab, z0, y0, x0);
  return hipGetLastError();
}

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
