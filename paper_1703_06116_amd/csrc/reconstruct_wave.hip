// Superposition at evaluation points for phase space m = 4, 6, 8, FP64 on
// the vector ALU (Sec. 2.3 eq:shgb, Sec. 2.4 step 6).  A block owns 256
// points (one per thread, kept in registers) and a chunk of beams; beams pass
// through LDS in tiles whose coefficients are formed once per tile:
//   weight w = exp(logw + Lam) phase A exp(iS/eps),  P/eps,  and the packed
//   quadratic form Q_ij = Z_ij / (2 eps) (diagonal), Z_ij / eps (i < j),
// so that the exponent is -sum_{i<=j} Q_ij y_i y_j + i P.y/eps with y = x - X
// formed in FP64 first.  Chunks write partial sums; a second kernel adds them
// in chunk order.
#include "device.h"

namespace shgb {

constexpr int kRwThreads = 256;
constexpr int kRwTile = 8;             // beams per LDS tile
constexpr int64_t kRwMaxChunks = 64;

struct RwTiling {
  int64_t chunk, n_chunks, pt_tiles;
};

RwTiling rw_tiling(int64_t n, int64_t Q) {
  RwTiling t;
  int64_t nc = (n + 255) / 256;
  if (nc > kRwMaxChunks) nc = kRwMaxChunks;
  if (nc < 1) nc = 1;
  const int64_t per = (n + nc - 1) / nc;
  t.chunk = (per + kRwTile - 1) / kRwTile * kRwTile;
  if (t.chunk < kRwTile) t.chunk = kRwTile;
  t.n_chunks = (n + t.chunk - 1) / t.chunk;
  if (t.n_chunks < 1) t.n_chunks = 1;
  t.pt_tiles = (Q + kRwThreads - 1) / kRwThreads;
  return t;
}

template <int M>
struct RwBeam {
  static constexpr int T = M * (M + 1) / 2;
  double X[M], Pe[M], Qr[T], Qi[T];
  double wr, wi;
  int comp;
};

// TS: element type of the stored trajectory rows; the arithmetic is FP64.
template <int M, typename TS>
__global__ void __launch_bounds__(kRwThreads)
recon_wave_kernel(DevModel md, const TS *__restrict__ f, const double *__restrict__ sc,
                  const int32_t *__restrict__ cmp, int64_t n, int64_t ld, const double *__restrict__ pts, int64_t Q,
                  int64_t chunk, double *__restrict__ partial) {
  constexpr int T = M * (M + 1) / 2;
  __shared__ RwBeam<M> tile[kRwTile];
  const Layout L(M, ld);
  const double inv_eps = 1.0 / md.eps, half_inv_eps = 0.5 / md.eps;
  const int64_t q = (int64_t)blockIdx.x * kRwThreads + threadIdx.x;
  const bool qlive = q < Q;
  double x[M];
#pragma unroll
  for (int i = 0; i < M; ++i) x[i] = qlive ? pts[q * M + i] : 0.0;
  double acc[SHGB_NCOMP][2];
#pragma unroll
  for (int i = 0; i < SHGB_NCOMP; ++i) acc[i][0] = acc[i][1] = 0.0;
  const int64_t kbeg = (int64_t)blockIdx.y * chunk;
  const int64_t kend = kbeg + chunk < n ? kbeg + chunk : n;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kRwTile) {
    const int nt = (int)(kend - k0 < kRwTile ? kend - k0 : kRwTile);
    __syncthreads();
    // cooperative fill: every thread handles some (beam, field) pairs
    for (int u = threadIdx.x; u < nt * (T + 2 * M); u += kRwThreads) {
      const int bt = u / (T + 2 * M), r = u % (T + 2 * M);
      const int64_t b = k0 + bt;
      if (r < T) {
        int a = 0, rem = r;
        while (rem >= M - a) { rem -= M - a; ++a; }
        const double s = (rem == 0) ? half_inv_eps : inv_eps;  // rem == 0: diagonal entry
        tile[bt].Qr[r] = (double)f[L.Zre(r) * ld + b] * s;
        tile[bt].Qi[r] = (double)f[L.Zim(r) * ld + b] * s;
      } else if (r < T + M) {
        tile[bt].X[r - T] = (double)f[L.X(r - T) * ld + b];
      } else {
        tile[bt].Pe[r - T - M] = (double)f[L.P(r - T - M) * ld + b] * inv_eps;
      }
    }
    if (threadIdx.x < nt) {
      const int64_t b = k0 + threadIdx.x;
      const double mag = exp(sc[kRowLogw * ld + b] + sc[kRowLam * ld + b]);
      const double pr = sc[kRowPhre * ld + b] * mag, pim = sc[kRowPhim * ld + b] * mag;
      const double ar = sc[kRowAre * ld + b], ai = sc[kRowAim * ld + b];
      double sn, cs;
      sincos(sc[kRowS * ld + b] * inv_eps, &sn, &cs);
      const double wr0 = pr * ar - pim * ai, wi0 = pr * ai + pim * ar;
      tile[threadIdx.x].wr = wr0 * cs - wi0 * sn;
      tile[threadIdx.x].wi = wr0 * sn + wi0 * cs;
      tile[threadIdx.x].comp = cmp[b];
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      const RwBeam<M> &bm = tile[t];
      double y[M];
#pragma unroll
      for (int i = 0; i < M; ++i) y[i] = x[i] - bm.X[i];
      double re = 0.0, im = 0.0;
      int idx = 0;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int j = i; j < M; ++j) {
          sr += bm.Qr[idx] * y[j];
          si += bm.Qi[idx] * y[j];
          ++idx;
        }
        re -= sr * y[i];
        im += bm.Pe[i] * y[i] - si * y[i];
      }
      const double g = exp(re);
      double sn, cs;
      sincos(im, &sn, &cs);
      const double gr = g * cs, gi = g * sn;
      const double vr = bm.wr * gr - bm.wi * gi, vi = bm.wr * gi + bm.wi * gr;
      switch (bm.comp) {  // uniform across the block
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

__global__ void recon_wave_reduce(const double *__restrict__ partial, int64_t n_chunks, int64_t len,
                                  double *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int64_t c = 0; c < n_chunks; ++c) s += partial[c * len + e];
  out[e] = s;
}

bool recon_wave_supported(int m) { return m == 4 || m == 6 || m == 8; }

int64_t recon_wave_workspace_bytes(int64_t n, int, int64_t Q) {
  const RwTiling t = rw_tiling(n, Q);
  return t.n_chunks * SHGB_NCOMP * Q * 2 * (int64_t)sizeof(double);
}

hipError_t launch_recon_wave(const DevModel &md, const shgb_state &st, const double *pts, int64_t Q, double *out,
                             void *work, hipStream_t stream) {
  if (Q == 0) return hipSuccess;
  const int64_t len = SHGB_NCOMP * Q * 2;
  const RwTiling t = rw_tiling(st.n_beams, Q);
  double *partial = (double *)work;
  if (st.n_beams == 0) {
    hipLaunchKernelGGL(recon_wave_reduce, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, partial,
                       (int64_t)0, len, out);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)t.pt_tiles, (unsigned)t.n_chunks);
  const double *sc = scalar_block(st);
#define SHGB_RW_CASE(MM)                                                                                  \
  case MM:                                                                                                \
    if (mixed(st))                                                                                        \
      hipLaunchKernelGGL((recon_wave_kernel<MM, float>), grid, dim3(kRwThreads), 0, stream, md, st.f32, sc, \
                         st.comp, st.n_beams, st.ld, pts, Q, t.chunk, partial);                           \
    else                                                                                                  \
      hipLaunchKernelGGL((recon_wave_kernel<MM, double>), grid, dim3(kRwThreads), 0, stream, md, st.f64,   \
                         sc, st.comp, st.n_beams, st.ld, pts, Q, t.chunk, partial);                       \
    break;
  switch (st.m) {
    SHGB_RW_CASE(4)
    SHGB_RW_CASE(6)
    SHGB_RW_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef SHGB_RW_CASE
  hipLaunchKernelGGL(recon_wave_reduce, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, partial,
                     t.n_chunks, len, out);
  return hipGetLastError();
}

}  // namespace shgb
