// Superposition of the beams at evaluation points for phase space m = 2
// (Sec. 2.3 eq:shgb, Sec. 2.4 step 6):
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
// skipped for it.  Far beams are the common case on a field grid, so they
// are culled before any per-point work: points are taken in Morton order
// (one sorting workgroup per chunk of points), each wavefront bounds its 64
// points by a box, and each beam gets the box of the ellipse outside which
// its real exponent is below the zero threshold with a margin; a wavefront
// tests 64 beams at once and evaluates only the beams whose box meets its
// own, in ascending order.  Culled terms are exactly the ones the per-point
// test would skip, so every sum is bitwise the one without culling (the
// margin covers the rounding of the box and of the exponent; beams whose
// coefficients are not finite, too large or too ill-conditioned for that
// bound are never culled).
#include "device.h"

namespace shgb {

constexpr int kRecThreads = 256;
constexpr int kRecTile = 256;          // beams per LDS tile
constexpr int64_t kRecMaxChunks = 512;
constexpr int64_t kRecTargetBlocks = 8192;   // 32 workgroups per CU: culled work is uneven across point tiles
// below these arguments exp (FP64) and the hardware exp2 (FP32) return +0:
// e^x < 2^-1075 for x < -745.14; 2^x < 2^-150 for x < -150
constexpr double kExpZero64 = -745.2;
constexpr float kExp2Zero32 = -151.0f;
// culling bounds: the exponent bound with a margin (natural log units for
// the FP64 kernel, log2 units for the FP32 one), the conditioning the
// rounding argument needs, and the magnitude below which every term of a
// non-culled evaluation stays finite
constexpr double kCullT64 = 760.0, kCullCond64 = 1e-6, kCullMax64 = 1e100;
constexpr double kCullT32 = 155.0, kCullCond32 = 1e-3, kCullMax32 = 1e15, kCullMaxX32 = 5e9;
constexpr int kSortN = 4096;           // points per Morton-sorted chunk
constexpr int kSortThreads = 1024;

struct RecTiling {
  int64_t chunk, n_chunks, pt_tiles;
};

// Beam chunks: enough workgroups for about kRecTargetBlocks in all (at most
// kRecMaxChunks chunks, at least a tile of beams each), so that the partial
// sums stay within kRecTargetBlocks x 256 points.
RecTiling rec_tiling_m2(int64_t n, int64_t Q) {
  RecTiling t;
  const int64_t pt_tiles = (Q + kRecThreads - 1) / kRecThreads;
  int64_t nc = (n + kRecTile - 1) / kRecTile;
  if (nc > kRecMaxChunks) nc = kRecMaxChunks;
  const int64_t want = pt_tiles > 0 ? (kRecTargetBlocks + pt_tiles - 1) / pt_tiles : 1;
  if (nc > want) nc = want;
  if (nc < 1) nc = 1;
  int64_t per = (n + nc - 1) / nc;
  t.chunk = (per + kRecTile - 1) / kRecTile * kRecTile;
  if (t.chunk < kRecTile) t.chunk = kRecTile;
  t.n_chunks = (n + t.chunk - 1) / t.chunk;
  if (t.n_chunks < 1) t.n_chunks = 1;
  t.pt_tiles = pt_tiles;
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

// coefficient record of one beam in LDS (structure of arrays); H1, H2: the
// half-widths of its culling box (infinite: never culled)
enum { RC_X1, RC_X2, RC_R11, RC_R12, RC_R22, RC_I11, RC_I12, RC_I22, RC_P1, RC_P2, RC_WRE, RC_WIM, RC_H1, RC_H2, RC_N };

// Half-widths of the bounding box of {y : r11 y1^2 + r12 y1 y2 + r22 y2^2 <=
// T} when the form is positive definite with det >= cond r11 r22 and ok
// (finite, bounded coefficients); else infinite.
__device__ inline void cull_box(double r11, double r12, double r22, bool ok, double T, double cond, double &h1,
                                double &h2) {
  const double det = r11 * r22 - 0.25 * r12 * r12;
  if (ok && r11 > 0.0 && r22 > 0.0 && det >= cond * r11 * r22) {
    h1 = sqrt(T * r22 / det);
    h2 = sqrt(T * r11 / det);
  } else {
    h1 = h2 = INFINITY;
  }
}

// Box of the wavefront's live points; an unbounded box (nothing culled) if
// one of them is not below xmax in magnitude.
struct WaveBox {
  double a1, b1, a2, b2;
};
__device__ inline WaveBox wave_box(bool live, double x1, double x2, double xmax) {
  const bool bad = live && !(fabs(x1) < xmax && fabs(x2) < xmax);
  double a1 = live ? x1 : INFINITY, b1 = live ? x1 : -INFINITY;
  double a2 = live ? x2 : INFINITY, b2 = live ? x2 : -INFINITY;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a1 = fmin(a1, __shfl_xor(a1, off, 64));
    b1 = fmax(b1, __shfl_xor(b1, off, 64));
    a2 = fmin(a2, __shfl_xor(a2, off, 64));
    b2 = fmax(b2, __shfl_xor(b2, off, 64));
  }
  if (__ballot(bad)) return WaveBox{-INFINITY, INFINITY, -INFINITY, INFINITY};
  return WaveBox{a1, b1, a2, b2};
}

// The beam (centre X, half-widths h) cannot reach the box: every point of
// it has |x1 - X1| > h1 or |x2 - X2| > h2 (differences rounded as the
// evaluation rounds them, which is monotone).
__device__ inline bool culled(const WaveBox &w, double X1, double X2, double h1, double h2) {
  return (w.a1 - X1 > h1) || (X1 - w.b1 > h1) || (w.a2 - X2 > h2) || (X2 - w.b2 > h2);
}

__device__ inline uint32_t spread_bits16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__device__ inline uint32_t quant16(double x, double lo, double scale) {
  const double u = (x - lo) * scale;   // NaN and out-of-range values go to the ends
  return u >= 65535.0 ? 65535u : (u > 0.0 ? (uint32_t)u : 0u);
}

// Morton order of each chunk of kSortN points (m = 2): perm[base + i] = the
// index of the point taken at sorted position base + i.  Keys are the
// interleaved 16-bit coordinates within the chunk's bounding box, ties
// broken by index; one bitonic sort in LDS per chunk.
__global__ void __launch_bounds__(kSortThreads)
rec_sort_m2_kernel(const double *__restrict__ pts, int64_t Q, int32_t *__restrict__ perm) {
  __shared__ uint64_t key[kSortN];
  __shared__ double red[4][kSortThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kSortN;
  const int n = (int)(Q - base < kSortN ? Q - base : kSortN);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double lo1 = INFINITY, hi1 = -INFINITY, lo2 = INFINITY, hi2 = -INFINITY;
  for (int i = tid; i < n; i += kSortThreads) {
    const double x1 = pts[2 * (base + i)], x2 = pts[2 * (base + i) + 1];
    if (fabs(x1) < INFINITY) { lo1 = fmin(lo1, x1); hi1 = fmax(hi1, x1); }
    if (fabs(x2) < INFINITY) { lo2 = fmin(lo2, x2); hi2 = fmax(hi2, x2); }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo1 = fmin(lo1, __shfl_xor(lo1, off, 64));
    hi1 = fmax(hi1, __shfl_xor(hi1, off, 64));
    lo2 = fmin(lo2, __shfl_xor(lo2, off, 64));
    hi2 = fmax(hi2, __shfl_xor(hi2, off, 64));
  }
  if (lane == 0) { red[0][wid] = lo1; red[1][wid] = hi1; red[2][wid] = lo2; red[3][wid] = hi2; }
  __syncthreads();
  lo1 = red[0][0]; hi1 = red[1][0]; lo2 = red[2][0]; hi2 = red[3][0];
  for (int w = 1; w < kSortThreads / 64; ++w) {
    lo1 = fmin(lo1, red[0][w]); hi1 = fmax(hi1, red[1][w]);
    lo2 = fmin(lo2, red[2][w]); hi2 = fmax(hi2, red[3][w]);
  }
  const double s1 = hi1 > lo1 && hi1 - lo1 < INFINITY ? 65535.0 / (hi1 - lo1) : 0.0;
  const double s2 = hi2 > lo2 && hi2 - lo2 < INFINITY ? 65535.0 / (hi2 - lo2) : 0.0;
  for (int i = tid; i < kSortN; i += kSortThreads) {
    uint64_t k = ~0ull;
    if (i < n) {
      const double x1 = pts[2 * (base + i)], x2 = pts[2 * (base + i) + 1];
      const uint32_t code = spread_bits16(quant16(x1, lo1, s1)) | (spread_bits16(quant16(x2, lo2, s2)) << 1);
      k = ((uint64_t)code << 32) | (uint32_t)i;
    }
    key[i] = k;
  }
  __syncthreads();
  for (int k = 2; k <= kSortN; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < kSortN; i += kSortThreads) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t ki = key[i], kl = key[l];
          const bool up = (i & k) == 0;
          if ((ki > kl) == up) { key[i] = kl; key[l] = ki; }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += kSortThreads) perm[base + i] = (int32_t)(base + (int64_t)(key[i] & 0xffffffffu));
}

__global__ void __launch_bounds__(kRecThreads) __attribute__((amdgpu_waves_per_eu(4)))
recon_m2_kernel(DevModel md, const double *__restrict__ f, const double *__restrict__ sc,
                const int32_t *__restrict__ comp, int64_t n, int64_t ld, const double *__restrict__ pts,
                const int32_t *__restrict__ perm, int64_t Q, int64_t chunk, double *__restrict__ partial) {
  __shared__ double rec[RC_N][kRecTile];
  __shared__ int rcomp[kRecTile];
  const Layout L(2, ld);
  const double inv_eps = 1.0 / md.eps, half_inv_eps = 0.5 / md.eps;
  const int lane = threadIdx.x & 63;
  // point tile: rotated by the chunk, so that the workgroups that launch
  // round-robin over the 8 XCDs do not give one XCD the same tiles (the
  // dense ones) in every chunk
  const int64_t tile = ((int64_t)blockIdx.x + blockIdx.y) % gridDim.x;
  const int64_t qs = tile * kRecThreads + threadIdx.x;   // position in Morton order
  const bool qlive = qs < Q;
  const int64_t q = qlive ? perm[qs] : 0;
  const double x1 = qlive ? pts[2 * q] : 0.0, x2 = qlive ? pts[2 * q + 1] : 0.0;
  const WaveBox box = wave_box(qlive, x1, x2, kCullMax64);
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
      double v[RC_H1];
      v[RC_WRE] = wr;
      v[RC_WIM] = wi;
      v[RC_X1] = f[L.X(0) * ld + b];
      v[RC_X2] = f[L.X(1) * ld + b];
      v[RC_R11] = f[L.Zre(0) * ld + b] * half_inv_eps;
      v[RC_R12] = f[L.Zre(1) * ld + b] * inv_eps;
      v[RC_R22] = f[L.Zre(2) * ld + b] * half_inv_eps;
      v[RC_I11] = f[L.Zim(0) * ld + b] * half_inv_eps;
      v[RC_I12] = f[L.Zim(1) * ld + b] * inv_eps;
      v[RC_I22] = f[L.Zim(2) * ld + b] * half_inv_eps;
      v[RC_P1] = f[L.P(0) * ld + b] * inv_eps;
      v[RC_P2] = f[L.P(1) * ld + b] * inv_eps;
      bool ok = fabs(wr) < INFINITY && fabs(wi) < INFINITY;
#pragma unroll
      for (int j = RC_X1; j <= RC_P2; ++j) ok = ok && fabs(v[j]) < kCullMax64;
      double h1, h2;
      cull_box(v[RC_R11], v[RC_R12], v[RC_R22], ok, kCullT64, kCullCond64, h1, h2);
#pragma unroll
      for (int j = 0; j < RC_H1; ++j) rec[j][threadIdx.x] = v[j];
      rec[RC_H1][threadIdx.x] = h1;
      rec[RC_H2][threadIdx.x] = h2;
      rcomp[threadIdx.x] = comp[b];
    }
    __syncthreads();
    for (int g = 0; g < nt; g += 64) {
      // 64 beams tested at once; the survivors are evaluated in ascending order
      const int jl = g + lane;
      const bool keep = jl < nt && !culled(box, rec[RC_X1][jl], rec[RC_X2][jl], rec[RC_H1][jl], rec[RC_H2][jl]);
      uint64_t mask = __ballot(keep);
      while (mask) {
        const int t = g + __builtin_ctzll(mask);
        mask &= mask - 1;
        const double y1 = x1 - rec[RC_X1][t], y2 = x2 - rec[RC_X2][t];
        const double y11 = y1 * y1, y12 = y1 * y2, y22 = y2 * y2;
        const double re = -(rec[RC_R11][t] * y11 + rec[RC_R12][t] * y12 + rec[RC_R22][t] * y22);
        const double im = rec[RC_P1][t] * y1 + rec[RC_P2][t] * y2 -
                          (rec[RC_I11][t] * y11 + rec[RC_I12][t] * y12 + rec[RC_I22][t] * y22);
        const double wr = rec[RC_WRE][t], wi = rec[RC_WIM][t];
        if (re < kExpZero64 && fabs(im) < INFINITY && fabs(wr) < INFINITY && fabs(wi) < INFINITY) continue;
        const double e = exp(re);
        double sn, cs;
        sincos(im, &sn, &cs);
        const double gr = e * cs, gi = e * sn;
        const double vr = wr * gr - wi * gi, vi = wr * gi + wi * gr;
        switch (rcomp[t]) {  // uniform across the block
          case 0: acc[0][0] += vr; acc[0][1] += vi; break;
          case 1: acc[1][0] += vr; acc[1][1] += vi; break;
          case 2: acc[2][0] += vr; acc[2][1] += vi; break;
          default: acc[3][0] += vr; acc[3][1] += vi; break;
        }
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
__global__ void __launch_bounds__(kRecThreads) __attribute__((amdgpu_waves_per_eu(4)))
recon_m2_mixed_kernel(DevModel md, const float *__restrict__ f, const double *__restrict__ sc,
                      const int32_t *__restrict__ comp, int64_t n, int64_t ld, const double *__restrict__ pts,
                      const int32_t *__restrict__ perm, int64_t Q, int64_t chunk, double *__restrict__ partial) {
  __shared__ float rec[RC_N][kRecTile];
  __shared__ int rcomp[kRecTile];
  const Layout L(2, ld);
  const double inv_eps = 1.0 / md.eps;
  const float finv_eps = (float)inv_eps, fhalf_inv_eps = (float)(0.5 * inv_eps);
  const float inv_2pi = (float)(0.5 / M_PI), log2e = (float)M_LOG2E;
  const int lane = threadIdx.x & 63;
  // point tile: rotated by the chunk, so that the workgroups that launch
  // round-robin over the 8 XCDs do not give one XCD the same tiles (the
  // dense ones) in every chunk
  const int64_t tile = ((int64_t)blockIdx.x + blockIdx.y) % gridDim.x;
  const int64_t qs = tile * kRecThreads + threadIdx.x;   // position in Morton order
  const bool qlive = qs < Q;
  const int64_t q = qlive ? perm[qs] : 0;
  const double x1 = qlive ? pts[2 * q] : 0.0, x2 = qlive ? pts[2 * q + 1] : 0.0;
  const WaveBox box = wave_box(qlive, x1, x2, kCullMaxX32);
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
      float v[RC_H1];
      v[RC_WRE] = (float)wr;
      v[RC_WIM] = (float)wi;
      v[RC_X1] = f[L.X(0) * ld + b];
      v[RC_X2] = f[L.X(1) * ld + b];
      // the real quadratic form carries log2(e), so that exp is one exp2
      v[RC_R11] = f[L.Zre(0) * ld + b] * (fhalf_inv_eps * log2e);
      v[RC_R12] = f[L.Zre(1) * ld + b] * (finv_eps * log2e);
      v[RC_R22] = f[L.Zre(2) * ld + b] * (fhalf_inv_eps * log2e);
      // the phase in turns
      v[RC_I11] = f[L.Zim(0) * ld + b] * (fhalf_inv_eps * inv_2pi);
      v[RC_I12] = f[L.Zim(1) * ld + b] * (finv_eps * inv_2pi);
      v[RC_I22] = f[L.Zim(2) * ld + b] * (fhalf_inv_eps * inv_2pi);
      v[RC_P1] = f[L.P(0) * ld + b] * (finv_eps * inv_2pi);
      v[RC_P2] = f[L.P(1) * ld + b] * (finv_eps * inv_2pi);
      bool ok = fabsf(v[RC_WRE]) < INFINITY && fabsf(v[RC_WIM]) < INFINITY && fabsf(v[RC_X1]) < kCullMaxX32 &&
                fabsf(v[RC_X2]) < kCullMaxX32;
#pragma unroll
      for (int j = RC_R11; j <= RC_P2; ++j) ok = ok && fabsf(v[j]) < kCullMax32;
      double h1, h2;
      cull_box(v[RC_R11], v[RC_R12], v[RC_R22], ok, kCullT32, kCullCond32, h1, h2);
#pragma unroll
      for (int j = 0; j < RC_H1; ++j) rec[j][threadIdx.x] = v[j];
      rec[RC_H1][threadIdx.x] = (float)h1;
      rec[RC_H2][threadIdx.x] = (float)h2;
      rcomp[threadIdx.x] = comp[b];
    }
    __syncthreads();
    for (int g = 0; g < nt; g += 64) {
      // 64 beams tested at once; the survivors are evaluated in ascending order
      const int jl = g + lane;
      const bool keep = jl < nt && !culled(box, rec[RC_X1][jl], rec[RC_X2][jl], rec[RC_H1][jl], rec[RC_H2][jl]);
      uint64_t mask = __ballot(keep);
      while (mask) {
        const int t = g + __builtin_ctzll(mask);
        mask &= mask - 1;
        const float y1 = (float)(x1 - (double)rec[RC_X1][t]), y2 = (float)(x2 - (double)rec[RC_X2][t]);
        const float y11 = y1 * y1, y12 = y1 * y2, y22 = y2 * y2;
        const float re2 = -(rec[RC_R11][t] * y11 + rec[RC_R12][t] * y12 + rec[RC_R22][t] * y22);
        float turns = rec[RC_P1][t] * y1 + rec[RC_P2][t] * y2 -
                      (rec[RC_I11][t] * y11 + rec[RC_I12][t] * y12 + rec[RC_I22][t] * y22);
        const float wr = rec[RC_WRE][t], wi = rec[RC_WIM][t];
        if (re2 < kExp2Zero32 && fabsf(turns) < INFINITY && fabsf(wr) < INFINITY && fabsf(wi) < INFINITY) continue;
        turns = turns - rintf(turns);
        const float e = __builtin_amdgcn_exp2f(re2);
        const float gr = e * __builtin_amdgcn_cosf(turns), gi = e * __builtin_amdgcn_sinf(turns);
        const double vr = (double)(wr * gr - wi * gi), vi = (double)(wr * gi + wi * gr);
        switch (rcomp[t]) {  // uniform across the block
          case 0: acc[0][0] += vr; acc[0][1] += vi; break;
          case 1: acc[1][0] += vr; acc[1][1] += vi; break;
          case 2: acc[2][0] += vr; acc[2][1] += vi; break;
          default: acc[3][0] += vr; acc[3][1] += vi; break;
        }
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

// workspace: the per-chunk partial sums, then the point permutation
static int64_t partial_bytes_m2(int64_t n, int64_t Q) {
  const RecTiling t = rec_tiling_m2(n, Q);
  return (t.n_chunks * SHGB_NCOMP * Q * 2 * (int64_t)sizeof(double) + 255) / 256 * 256;
}

int64_t recon_m2_workspace_bytes(int64_t n, int64_t Q) { return partial_bytes_m2(n, Q) + Q * (int64_t)sizeof(int32_t); }

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
  int32_t *perm = (int32_t *)((char *)work + partial_bytes_m2(st.n_beams, Q));
  hipLaunchKernelGGL(rec_sort_m2_kernel, dim3((unsigned)((Q + kSortN - 1) / kSortN)), dim3(kSortThreads), 0, stream,
                     pts, Q, perm);
  const dim3 grid((unsigned)t.pt_tiles, (unsigned)t.n_chunks);
  if (mixed(st))
    hipLaunchKernelGGL(recon_m2_mixed_kernel, grid, dim3(kRecThreads), 0, stream, md, st.f32, scalar_block(st),
                       st.comp, st.n_beams, st.ld, pts, perm, Q, t.chunk, partial);
  else
    hipLaunchKernelGGL(recon_m2_kernel, grid, dim3(kRecThreads), 0, stream, md, st.f64, scalar_block(st), st.comp,
                       st.n_beams, st.ld, pts, perm, Q, t.chunk, partial);
  hipLaunchKernelGGL(recon_reduce_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, partial,
                     t.n_chunks, len, out);
  return hipGetLastError();
}

}  // namespace shgb
