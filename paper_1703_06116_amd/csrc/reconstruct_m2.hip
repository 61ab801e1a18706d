// Superposition of the beams at evaluation points for phase space m = 2
// (Sec. 2.3 eq. (2.26), Sec. 2.4 step 6):
//   out_i(x) = sum_{k: l_k = i} exp(omega_k) A_k exp(-y^T Z_k y/(2 eps) + i P_k.y/eps + i S_k/eps),
//   y = x - X_k.
// A block owns a tile of points (one per thread, in registers) and a chunk of
// beams; beams pass through LDS in tiles of 256, each beam's coefficients
// formed once per tile (weight exp(omega) A exp(iS/eps), Z/(2 eps), P/eps), and
// every thread evaluates its point against the whole tile (LDS broadcast
// reads).  The component of the current beam is uniform across the block, so
// the accumulator select is a uniform branch.  Chunks write partial sums;
// a second kernel adds them in chunk order (bitwise reproducible).
// A term whose real exponent is below the range of exp (the exponential is
// exactly +0 in the working precision) adds exactly zero when its phase and
// the beam weight are finite, so exp, sincos and the accumulation are
// skipped for it; a wavefront in which every lane is in that case skips the
// whole evaluation (far beams are the common case on a field grid).
#include "device.h"

namespace shgb {

constexpr int kRecThreads = 256;
constexpr int kRecTile = 256;          // beams per LDS tile
constexpr int64_t kRecMaxChunks = 128;
// below these arguments exp (FP64) and the hardware exp2 (FP32) return +0:
// e^x < 2^-1075 for x < -745.14; 2^x < 2^-150 for x < -150
constexpr double kExpZero64 = -745.2;
constexpr float kExp2Zero32 = -151.0f;

struct RecTiling {
  int64_t chunk, n_chunks, pt_tiles;
};

RecTiling rec_tiling_m2(int64_t n, int64_t Q) {
  RecTiling t;
  int64_t nc = (n + kRecTile - 1) / kRecTile;
  if (nc > kRecMaxChunks) nc = kRecMaxChunks;
  if (nc < 1) nc = 1;
  int64_t per = (n + nc - 1) / nc;
  t.chunk = (per + kRecTile - 1) / kRecTile * kRecTile;
  if (t.chunk < kRecTile) t.chunk = kRecTile;
  t.n_chunks = (n + t.chunk - 1) / t.chunk;
  if (t.n_chunks < 1) t.n_chunks = 1;
  t.pt_tiles = (Q + kRecThreads - 1) / kRecThreads;
  return t;
}

// exp(omega) A exp(iS/eps) of beam b, in FP64 (S/eps is a large angle)
__device__ inline void beam_weight_m2(const double *__restrict__ sc, int64_t ld, int64_t b, double inv_eps,
                                      double &wr, double &wi) {
  const double mag = exp(sc[kRowLogw * ld + b] + sc[kRowLam * ld + b]);
  const double pr = sc[kRowPhre * ld + b] * mag, pi = sc[kRowPhim * ld + b] * mag;
  const double ar = sc[kRowAre * ld + b], ai = sc[kRowAim * ld + b];
  double sn, cs;
  sincos(sc[kRowS * ld + b] * inv_eps, &sn, &cs);
  const double wr0 = pr * ar - pi * ai, wi0 = pr * ai + pi * ar;
  wr = wr0 * cs - wi0 * sn;
  wi = wr0 * sn + wi0 * cs;
}

// coefficient record of one beam in LDS (structure of arrays)
enum { RC_X1, RC_X2, RC_R11, RC_R12, RC_R22, RC_I11, RC_I12, RC_I22, RC_P1, RC_P2, RC_WRE, RC_WIM, RC_N };

__global__ void __launch_bounds__(kRecThreads)
recon_m2_kernel(DevModel md, const double *__restrict__ f, const double *__restrict__ sc,
                const int32_t *__restrict__ comp, int64_t n, int64_t ld, const double *__restrict__ pts, int64_t Q,
                int64_t chunk, double *__restrict__ partial) {
  __shared__ double rec[RC_N][kRecTile];
  __shared__ int rcomp[kRecTile];
  const Layout L(2, ld);
  const double inv_eps = 1.0 / md.eps, half_inv_eps = 0.5 / md.eps;
  const int64_t q = (int64_t)blockIdx.x * kRecThreads + threadIdx.x;
  const bool qlive = q < Q;
  const double x1 = qlive ? pts[2 * q] : 0.0, x2 = qlive ? pts[2 * q + 1] : 0.0;
  double acc[SHGB_NCOMP][2];
#pragma unroll
  for (int i = 0; i < SHGB_NCOMP; ++i) acc[i][0] = acc[i][1] = 0.0;
  const int64_t kbeg = (int64_t)blockIdx.y * chunk;
  const int64_t kend = kbeg + chunk < n ? kbeg + chunk : n;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kRecTile) {
    const int nt = (int)(kend - k0 < kRecTile ? kend - k0 : kRecTile);
    __syncthreads();
    if (threadIdx.x < nt) {
      const int64_t b = k0 + threadIdx.x;
      double wr, wi;
      beam_weight_m2(sc, ld, b, inv_eps, wr, wi);
      rec[RC_WRE][threadIdx.x] = wr;
      rec[RC_WIM][threadIdx.x] = wi;
      rec[RC_X1][threadIdx.x] = f[L.X(0) * ld + b];
      rec[RC_X2][threadIdx.x] = f[L.X(1) * ld + b];
      rec[RC_R11][threadIdx.x] = f[L.Zre(0) * ld + b] * half_inv_eps;
      rec[RC_R12][threadIdx.x] = f[L.Zre(1) * ld + b] * inv_eps;
      rec[RC_R22][threadIdx.x] = f[L.Zre(2) * ld + b] * half_inv_eps;
      rec[RC_I11][threadIdx.x] = f[L.Zim(0) * ld + b] * half_inv_eps;
      rec[RC_I12][threadIdx.x] = f[L.Zim(1) * ld + b] * inv_eps;
      rec[RC_I22][threadIdx.x] = f[L.Zim(2) * ld + b] * half_inv_eps;
      rec[RC_P1][threadIdx.x] = f[L.P(0) * ld + b] * inv_eps;
      rec[RC_P2][threadIdx.x] = f[L.P(1) * ld + b] * inv_eps;
      rcomp[threadIdx.x] = comp[b];
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      const double y1 = x1 - rec[RC_X1][t], y2 = x2 - rec[RC_X2][t];
      const double y11 = y1 * y1, y12 = y1 * y2, y22 = y2 * y2;
      const double re = -(rec[RC_R11][t] * y11 + rec[RC_R12][t] * y12 + rec[RC_R22][t] * y22);
      const double im = rec[RC_P1][t] * y1 + rec[RC_P2][t] * y2 -
                        (rec[RC_I11][t] * y11 + rec[RC_I12][t] * y12 + rec[RC_I22][t] * y22);
      const double wr = rec[RC_WRE][t], wi = rec[RC_WIM][t];
      if (re < kExpZero64 && fabs(im) < INFINITY && fabs(wr) < INFINITY && fabs(wi) < INFINITY) continue;
      const double g = exp(re);
      double sn, cs;
      sincos(im, &sn, &cs);
      const double gr = g * cs, gi = g * sn;
      const double vr = wr * gr - wi * gi, vi = wr * gi + wi * gr;
      switch (rcomp[t]) {  // uniform across the block
        case 0: acc[0][0] += vr; acc[0][1] += vi; break;
        case 1: acc[1][0] += vr; acc[1][1] += vi; break;
        case 2: acc[2][0] += vr; acc[2][1] += vi; break;
        default: acc[3][0] += vr; acc[3][1] += vi; break;
      }
    }
  }
  if (qlive) {
    double *dst = partial + (int64_t)blockIdx.y * SHGB_NCOMP * Q * 2;
#pragma unroll
    for (int i = 0; i < SHGB_NCOMP; ++i) {
      dst[(i * Q + q) * 2 + 0] = acc[i][0];
      dst[(i * Q + q) * 2 + 1] = acc[i][1];
    }
  }
}

// Mixed-precision state: y = x - X is formed in FP64 and rounded once; the
// exponent, exp and sincos are FP32 (hardware exp2 / sin / cos after an
// exact-enough reduction of the angle to [-1/2, 1/2] turns); each term is
// added to FP64 accumulators.
__global__ void __launch_bounds__(kRecThreads)
recon_m2_mixed_kernel(DevModel md, const float *__restrict__ f, const double *__restrict__ sc,
                      const int32_t *__restrict__ comp, int64_t n, int64_t ld, const double *__restrict__ pts,
                      int64_t Q, int64_t chunk, double *__restrict__ partial) {
  __shared__ float rec[RC_N][kRecTile];
  __shared__ int rcomp[kRecTile];
  const Layout L(2, ld);
  const double inv_eps = 1.0 / md.eps;
  const float finv_eps = (float)inv_eps, fhalf_inv_eps = (float)(0.5 * inv_eps);
  const float inv_2pi = (float)(0.5 / M_PI), log2e = (float)M_LOG2E;
  const int64_t q = (int64_t)blockIdx.x * kRecThreads + threadIdx.x;
  const bool qlive = q < Q;
  const double x1 = qlive ? pts[2 * q] : 0.0, x2 = qlive ? pts[2 * q + 1] : 0.0;
  double acc[SHGB_NCOMP][2];
#pragma unroll
  for (int i = 0; i < SHGB_NCOMP; ++i) acc[i][0] = acc[i][1] = 0.0;
  const int64_t kbeg = (int64_t)blockIdx.y * chunk;
  const int64_t kend = kbeg + chunk < n ? kbeg + chunk : n;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kRecTile) {
    const int nt = (int)(kend - k0 < kRecTile ? kend - k0 : kRecTile);
    __syncthreads();
    if (threadIdx.x < nt) {
      const int64_t b = k0 + threadIdx.x;
      double wr, wi;
      beam_weight_m2(sc, ld, b, inv_eps, wr, wi);
      rec[RC_WRE][threadIdx.x] = (float)wr;
      rec[RC_WIM][threadIdx.x] = (float)wi;
      rec[RC_X1][threadIdx.x] = f[L.X(0) * ld + b];
      rec[RC_X2][threadIdx.x] = f[L.X(1) * ld + b];
      // the real quadratic form carries log2(e), so that exp is one exp2
      rec[RC_R11][threadIdx.x] = f[L.Zre(0) * ld + b] * (fhalf_inv_eps * log2e);
      rec[RC_R12][threadIdx.x] = f[L.Zre(1) * ld + b] * (finv_eps * log2e);
      rec[RC_R22][threadIdx.x] = f[L.Zre(2) * ld + b] * (fhalf_inv_eps * log2e);
      // the phase in turns
      rec[RC_I11][threadIdx.x] = f[L.Zim(0) * ld + b] * (fhalf_inv_eps * inv_2pi);
      rec[RC_I12][threadIdx.x] = f[L.Zim(1) * ld + b] * (finv_eps * inv_2pi);
      rec[RC_I22][threadIdx.x] = f[L.Zim(2) * ld + b] * (fhalf_inv_eps * inv_2pi);
      rec[RC_P1][threadIdx.x] = f[L.P(0) * ld + b] * (finv_eps * inv_2pi);
      rec[RC_P2][threadIdx.x] = f[L.P(1) * ld + b] * (finv_eps * inv_2pi);
      rcomp[threadIdx.x] = comp[b];
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      const float y1 = (float)(x1 - (double)rec[RC_X1][t]), y2 = (float)(x2 - (double)rec[RC_X2][t]);
      const float y11 = y1 * y1, y12 = y1 * y2, y22 = y2 * y2;
      const float re2 = -(rec[RC_R11][t] * y11 + rec[RC_R12][t] * y12 + rec[RC_R22][t] * y22);
      float turns = rec[RC_P1][t] * y1 + rec[RC_P2][t] * y2 -
                    (rec[RC_I11][t] * y11 + rec[RC_I12][t] * y12 + rec[RC_I22][t] * y22);
      const float wr = rec[RC_WRE][t], wi = rec[RC_WIM][t];
      if (re2 < kExp2Zero32 && fabsf(turns) < INFINITY && fabsf(wr) < INFINITY && fabsf(wi) < INFINITY) continue;
      turns = turns - rintf(turns);
      const float g = __builtin_amdgcn_exp2f(re2);
      const float gr = g * __builtin_amdgcn_cosf(turns), gi = g * __builtin_amdgcn_sinf(turns);
      const double vr = (double)(wr * gr - wi * gi), vi = (double)(wr * gi + wi * gr);
      switch (rcomp[t]) {  // uniform across the block
        case 0: acc[0][0] += vr; acc[0][1] += vi; break;
        case 1: acc[1][0] += vr; acc[1][1] += vi; break;
        case 2: acc[2][0] += vr; acc[2][1] += vi; break;
        default: acc[3][0] += vr; acc[3][1] += vi; break;
      }
    }
  }
  if (qlive) {
    double *dst = partial + (int64_t)blockIdx.y * SHGB_NCOMP * Q * 2;
#pragma unroll
    for (int i = 0; i < SHGB_NCOMP; ++i) {
      dst[(i * Q + q) * 2 + 0] = acc[i][0];
      dst[(i * Q + q) * 2 + 1] = acc[i][1];
    }
  }
}

__global__ void recon_reduce_kernel(const double *__restrict__ partial, int64_t n_chunks, int64_t len,
                                    double *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int64_t c = 0; c < n_chunks; ++c) s += partial[c * len + e];
  out[e] = s;
}

int64_t recon_m2_workspace_bytes(int64_t n, int64_t Q) {
  const RecTiling t = rec_tiling_m2(n, Q);
  return t.n_chunks * SHGB_NCOMP * Q * 2 * (int64_t)sizeof(double);
}

hipError_t launch_recon_m2(const DevModel &md, const shgb_state &st, const double *pts, int64_t Q, double *out,
                           void *work, hipStream_t stream) {
  const int64_t len = SHGB_NCOMP * Q * 2;
  if (Q == 0) return hipSuccess;
  const RecTiling t = rec_tiling_m2(st.n_beams, Q);
  double *partial = (double *)work;
  if (st.n_beams == 0) {  // an empty sum: the reduce kernel over zero chunks writes zeros
    hipLaunchKernelGGL(recon_reduce_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, partial,
                       (int64_t)0, len, out);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)t.pt_tiles, (unsigned)t.n_chunks);
  if (mixed(st))
    hipLaunchKernelGGL(recon_m2_mixed_kernel, grid, dim3(kRecThreads), 0, stream, md, st.f32, scalar_block(st),
                       st.comp, st.n_beams, st.ld, pts, Q, t.chunk, partial);
  else
    hipLaunchKernelGGL(recon_m2_kernel, grid, dim3(kRecThreads), 0, stream, md, st.f64, scalar_block(st), st.comp,
                       st.n_beams, st.ld, pts, Q, t.chunk, partial);
  hipLaunchKernelGGL(recon_reduce_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, partial,
                     t.n_chunks, len, out);
  return hipGetLastError();
}

}  // namespace shgb
