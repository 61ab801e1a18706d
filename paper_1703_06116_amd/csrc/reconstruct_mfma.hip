// Superposition at evaluation points for phase space m = 24 on the FP64
// matrix cores (Sec. 2.3 eq. (2.26), Sec. 2.4 step 6).
//
// The exponent of beam k at point x is a fixed quadratic polynomial in x.
// With x~ = x - c and X~ = X - c (c the mean of the points, to keep the terms
// small) and Z = M + iN:
//   -(x~ - X~)^T Z (x~ - X~)/(2 eps) + i P.(x~ - X~)/eps
//     = sum_f W[k][f] Phi[f][x],
//   Phi = ( x~_i x~_j (i <= j, 300), x~_i (24), 1 ),
//   W   = ( -Z_ij/(2 eps) (i = j) or -Z_ij/eps (i < j),
//           (Z X~)_i/eps + i P_i/eps,
//           -X~^T Z X~/(2 eps) - i P.X~/eps ),
// so all exponents of a beam tile and a point tile form one dense real
// GEMM [beams x 328] x [328 x points] for Re and for Im (F = 325 padded to
// 328).  It runs on v_mfma_f64_16x16x4_f64; the epilogue multiplies
// exp(Re) (cos Im + i sin Im) by the beam weight exp(omega) A exp(iS/eps)
// and sums per component and point.  Blocks own 128 points and a chunk of
// beams (64 per tile); partial sums per chunk are added in chunk order.
#include "device.h"

namespace shgb {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int RM = 24;
constexpr int RT = RM * (RM + 1) / 2;  // 300 quadratic features
constexpr int RF = RT + RM + 1;        // 325
constexpr int RFP = 328;               // padded to a multiple of the slab
constexpr int RBK = 64;                // beams per block tile
constexpr int RBQ = 128;               // points per block tile
constexpr int RKS = 8;                 // features per LDS slab (two MFMA k-steps)
constexpr int RNSLAB = RFP / RKS;      // 41
constexpr int RTHREADS = 256;
constexpr int64_t RMAXCHUNK = 8;

struct RmLayout {
  int64_t NB, QP, n_chunks, tiles_per_chunk, pt_tiles;
  int64_t off_c, off_phi, off_wr, off_wi, off_wk, off_cmp, off_partial, total;  // in doubles
};

RmLayout rm_layout(int64_t n, int64_t Q) {
  RmLayout L;
  L.NB = (n + RBK - 1) / RBK * RBK;
  if (L.NB == 0) L.NB = RBK;
  L.QP = (Q + RBQ - 1) / RBQ * RBQ;
  if (L.QP == 0) L.QP = RBQ;
  L.pt_tiles = L.QP / RBQ;
  const int64_t beam_tiles = L.NB / RBK;
  // enough blocks to fill the chip: at least ~1024 (4 per CU) when the work allows
  int64_t nc = (1024 + L.pt_tiles - 1) / L.pt_tiles;
  if (nc > RMAXCHUNK * 64) nc = RMAXCHUNK * 64;
  if (nc > beam_tiles) nc = beam_tiles;
  if (nc < 1) nc = 1;
  L.tiles_per_chunk = (beam_tiles + nc - 1) / nc;
  L.n_chunks = (beam_tiles + L.tiles_per_chunk - 1) / L.tiles_per_chunk;
  L.off_c = 0;
  L.off_phi = 32;
  L.off_wr = L.off_phi + (int64_t)RFP * L.QP;
  L.off_wi = L.off_wr + (int64_t)RFP * L.NB;
  L.off_wk = L.off_wi + (int64_t)RFP * L.NB;
  L.off_cmp = L.off_wk + 2 * L.NB;
  L.off_partial = L.off_cmp + L.NB;
  L.total = L.off_partial + L.n_chunks * SHGB_NCOMP * Q * 2;
  return L;
}

// Mean of the points (one block, fixed order).
__global__ void __launch_bounds__(RTHREADS) rm_center_kernel(const double *__restrict__ pts, int64_t Q,
                                                              double *__restrict__ c) {
  __shared__ double red[RTHREADS / 64][RM];
  double s[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) s[i] = 0.0;
  for (int64_t q = threadIdx.x; q < Q; q += RTHREADS)
#pragma unroll
    for (int i = 0; i < RM; ++i) s[i] += pts[q * RM + i];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    double x = s[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[wid][i] = x;
  }
  __syncthreads();
  if (threadIdx.x < RM) {
    double x = 0.0;
    for (int w = 0; w < RTHREADS / 64; ++w) x += red[w][threadIdx.x];
    c[threadIdx.x] = Q > 0 ? x / (double)Q : 0.0;
  }
}

// Point features Phi[f][q] (feature-major), zero for padded points.
__global__ void __launch_bounds__(RTHREADS) rm_points_kernel(const double *__restrict__ pts, int64_t Q, int64_t QP,
                                                              const double *__restrict__ c, double *__restrict__ phi) {
  const int64_t q = (int64_t)blockIdx.x * RTHREADS + threadIdx.x;
  if (q >= QP) return;
  double x[RM];
  const bool live = q < Q;
#pragma unroll
  for (int i = 0; i < RM; ++i) x[i] = live ? pts[q * RM + i] - c[i] : 0.0;
  int f = 0;
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = i; j < RM; ++j) phi[(int64_t)(f++) * QP + q] = x[i] * x[j];
#pragma unroll
  for (int i = 0; i < RM; ++i) phi[(int64_t)(f++) * QP + q] = x[i];
  phi[(int64_t)(f++) * QP + q] = live ? 1.0 : 0.0;
  for (; f < RFP; ++f) phi[(int64_t)f * QP + q] = 0.0;
}

// Beam feature weights W[f][k] (feature-major, Re and Im), weight and
// component, in FP64 from trajectory rows of element type TS.
template <typename TS>
__global__ void __launch_bounds__(RTHREADS)
rm_beams_kernel(DevModel md, const TS *__restrict__ fs, const double *__restrict__ sc,
                const int32_t *__restrict__ comp, int64_t n, int64_t ld, int64_t NB, const double *__restrict__ c,
                double *__restrict__ wr, double *__restrict__ wi, double *__restrict__ wk, double *__restrict__ wc) {
  const int64_t k = (int64_t)blockIdx.x * RTHREADS + threadIdx.x;
  if (k >= NB) return;
  if (k >= n) {
    for (int f = 0; f < RFP; ++f) { wr[(int64_t)f * NB + k] = 0.0; wi[(int64_t)f * NB + k] = 0.0; }
    wk[2 * k] = wk[2 * k + 1] = 0.0;
    wc[k] = 0.0;
    return;
  }
  const Layout L(RM, ld);
  const double ie = 1.0 / md.eps, h2e = 0.5 / md.eps;
  double xt[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) xt[i] = (double)fs[L.X(i) * ld + k] - c[i];
  // quadratic weights
  for (int t = 0, i = 0; i < RM; ++i)
    for (int j = i; j < RM; ++j, ++t) {
      const double s = (i == j) ? -h2e : -ie;
      wr[(int64_t)t * NB + k] = s * (double)fs[L.Zre(t) * ld + k];
      wi[(int64_t)t * NB + k] = s * (double)fs[L.Zim(t) * ld + k];
    }
  // Z X~, linear and constant weights
  double cr = 0.0, ci = 0.0, px = 0.0;
  for (int i = 0; i < RM; ++i) {
    double zr = 0.0, zi = 0.0;
    for (int j = 0; j < RM; ++j) {
      const int t = i <= j ? Layout::tri(RM, i, j) : Layout::tri(RM, j, i);
      zr += (double)fs[L.Zre(t) * ld + k] * xt[j];
      zi += (double)fs[L.Zim(t) * ld + k] * xt[j];
    }
    const double Pi = (double)fs[L.P(i) * ld + k];
    wr[(int64_t)(RT + i) * NB + k] = zr * ie;
    wi[(int64_t)(RT + i) * NB + k] = (zi + Pi) * ie;
    cr += xt[i] * zr;
    ci += xt[i] * zi;
    px += Pi * xt[i];
  }
  wr[(int64_t)(RF - 1) * NB + k] = -cr * h2e;
  wi[(int64_t)(RF - 1) * NB + k] = -ci * h2e - px * ie;
  for (int f = RF; f < RFP; ++f) { wr[(int64_t)f * NB + k] = 0.0; wi[(int64_t)f * NB + k] = 0.0; }
  // exp(omega) A exp(iS/eps)
  const double mag = exp(sc[kRowLogw * ld + k] + sc[kRowLam * ld + k]);
  const double pr = sc[kRowPhre * ld + k] * mag, pim = sc[kRowPhim * ld + k] * mag;
  const double ar = sc[kRowAre * ld + k], ai = sc[kRowAim * ld + k];
  double sn, cs;
  sincos(sc[kRowS * ld + k] * ie, &sn, &cs);
  const double w0r = pr * ar - pim * ai, w0i = pr * ai + pim * ar;
  wk[2 * k] = w0r * cs - w0i * sn;
  wk[2 * k + 1] = w0r * sn + w0i * cs;
  wc[k] = (double)comp[k];
}

// Dense exponent GEMM on the matrix cores with the field epilogue fused.
// Waves: w = 2 wy + wx; wave tile 32 beams (wy) x 64 points (wx) = 2 x 4
// MFMA tiles of 16 x 16, for Re and for Im.  v_mfma_f64_16x16x4_f64 lane
// layout (checked on gfx950): A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k, D[i][j] in lane j + 16 (i % 4), element i / 4.  After each beam tile the epilogue
// values are summed over the tile's rows (in-lane, then across the four lane
// groups) and added to per-point accumulators in LDS.
__global__ void __launch_bounds__(RTHREADS)
rm_gemm_kernel(const double *__restrict__ wr, const double *__restrict__ wi, const double *__restrict__ wk,
               const double *__restrict__ wc, const double *__restrict__ phi, int64_t NB, int64_t QP, int64_t Q,
               int64_t tiles_per_chunk, double *__restrict__ partial) {
  __shared__ double Ws[2][2][RKS][RBK];   // [buffer][re/im][feature][beam]
  __shared__ double Ps[2][RKS][RBQ];      // [buffer][feature][point]
  __shared__ double Bw[RBK][3];           // beam weight re, im, component
  __shared__ double Acc[2][2 * SHGB_NCOMP][RBQ];  // [wave row][comp re/im][point]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wy = w >> 1, wx = w & 1;
  const int g = lane >> 4, li = lane & 15;
  const int64_t q0 = (int64_t)blockIdx.x * RBQ;
  const int64_t kt0 = (int64_t)blockIdx.y * tiles_per_chunk;
  for (int e = tid; e < 2 * 2 * SHGB_NCOMP * RBQ; e += RTHREADS) (&Acc[0][0][0])[e] = 0.0;
  // this thread's share of each slab: 4 W values and 4 Phi values
  int64_t woff[4], poff[4];
  const double *wsrc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + RTHREADS * u;  // 0..1023
    wsrc[u] = (e >> 9) ? wi : wr;
    woff[u] = (int64_t)((e >> 6) & 7) * NB + (e & 63);
    poff[u] = (int64_t)(e >> 7) * QP + q0 + (e & 127);
  }
  for (int64_t kt = kt0; kt < kt0 + tiles_per_chunk; ++kt) {
    const int64_t k0 = kt * RBK;
    if (k0 >= NB) break;  // uniform across the block
    dbl4 are[2][4], aim[2][4];
#pragma unroll
    for (int bt = 0; bt < 2; ++bt)
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) { are[bt][pt] = dbl4{0, 0, 0, 0}; aim[bt][pt] = dbl4{0, 0, 0, 0}; }
    double rw[4], rp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) { rw[u] = wsrc[u][woff[u] + k0]; rp[u] = phi[poff[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + RTHREADS * u;
      Ws[0][e >> 9][(e >> 6) & 7][e & 63] = rw[u];
      Ps[0][e >> 7][e & 127] = rp[u];
    }
    if (tid < RBK) {
      Bw[tid][0] = wk[2 * (k0 + tid)];
      Bw[tid][1] = wk[2 * (k0 + tid) + 1];
      Bw[tid][2] = wc[k0 + tid];
    }
    __syncthreads();
    for (int s = 0; s < RNSLAB; ++s) {
      const int buf = s & 1;
      const bool more = s + 1 < RNSLAB;
      if (more) {
        const int64_t fw = (int64_t)(s + 1) * RKS * NB + k0, fp = (int64_t)(s + 1) * RKS * QP;
#pragma unroll
        for (int u = 0; u < 4; ++u) { rw[u] = wsrc[u][woff[u] + fw]; rp[u] = phi[poff[u] + fp]; }
      }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const int f = 4 * ks + g;
        double bfr[4];
#pragma unroll
        for (int pt = 0; pt < 4; ++pt) bfr[pt] = Ps[buf][f][64 * wx + 16 * pt + li];
#pragma unroll
        for (int bt = 0; bt < 2; ++bt) {
          const double ar = Ws[buf][0][f][32 * wy + 16 * bt + li];
          const double ai = Ws[buf][1][f][32 * wy + 16 * bt + li];
#pragma unroll
          for (int pt = 0; pt < 4; ++pt) {
            are[bt][pt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bfr[pt], are[bt][pt], 0, 0, 0);
            aim[bt][pt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bfr[pt], aim[bt][pt], 0, 0, 0);
          }
        }
      }
      if (more) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = tid + RTHREADS * u;
          Ws[buf ^ 1][e >> 9][(e >> 6) & 7][e & 63] = rw[u];
          Ps[buf ^ 1][e >> 7][e & 127] = rp[u];
        }
      }
      __syncthreads();
    }
    // epilogue, one point tile at a time: w_k exp(E) per (beam, point), summed over the
    // lane's 8 beams per component, then over the four lane groups
#pragma unroll
    for (int pt = 0; pt < 4; ++pt) {
      double v[2 * SHGB_NCOMP];
#pragma unroll
      for (int c = 0; c < 2 * SHGB_NCOMP; ++c) v[c] = 0.0;
#pragma unroll
      for (int bt = 0; bt < 2; ++bt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int kb = 32 * wy + 16 * bt + g + 4 * r;
          const double e = exp(are[bt][pt][r]);
          double sn, cs;
          sincos(aim[bt][pt][r], &sn, &cs);
          const double gr = e * cs, gi = e * sn;
          const double bwr = Bw[kb][0], bwi = Bw[kb][1];
          const int cc = (int)Bw[kb][2];
          const double vr = bwr * gr - bwi * gi, vi = bwr * gi + bwi * gr;
#pragma unroll
          for (int c = 0; c < SHGB_NCOMP; ++c) {
            v[2 * c] += (cc == c) ? vr : 0.0;
            v[2 * c + 1] += (cc == c) ? vi : 0.0;
          }
        }
#pragma unroll
      for (int c = 0; c < 2 * SHGB_NCOMP; ++c) {
        double x = v[c];
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        if (g == 0) Acc[wy][c][64 * wx + 16 * pt + li] += x;
      }
    }
    __syncthreads();  // Bw and the slab buffers are rewritten by the next tile
  }
  // add the two wave rows and write this chunk's partial sums
  double *dst = partial + (int64_t)blockIdx.y * SHGB_NCOMP * Q * 2;
  for (int e = tid; e < 2 * SHGB_NCOMP * RBQ; e += RTHREADS) {
    const int c = e / RBQ, qq = e % RBQ;
    const int64_t q = q0 + qq;
    if (q < Q) dst[((c >> 1) * Q + q) * 2 + (c & 1)] = Acc[0][c][qq] + Acc[1][c][qq];
  }
}

__global__ void rm_reduce_kernel(const double *__restrict__ partial, int64_t n_chunks, int64_t len,
                                 double *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int64_t c = 0; c < n_chunks; ++c) s += partial[c * len + e];
  out[e] = s;
}

int64_t recon_mfma_workspace_bytes(int64_t n, int64_t Q) { return rm_layout(n, Q).total * (int64_t)sizeof(double); }

hipError_t launch_recon_mfma(const DevModel &md, const shgb_state &st, const double *pts, int64_t Q, double *out,
                             void *work, hipStream_t stream) {
  if (Q == 0) return hipSuccess;
  const int64_t len = SHGB_NCOMP * Q * 2;
  const RmLayout L = rm_layout(st.n_beams, Q);
  double *ws = (double *)work;
  if (st.n_beams == 0) {
    hipLaunchKernelGGL(rm_reduce_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream,
                       ws + L.off_partial, (int64_t)0, len, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(rm_center_kernel, dim3(1), dim3(RTHREADS), 0, stream, pts, Q, ws + L.off_c);
  hipLaunchKernelGGL(rm_points_kernel, dim3((unsigned)(L.QP / RTHREADS + 1)), dim3(RTHREADS), 0, stream, pts, Q,
                     L.QP, ws + L.off_c, ws + L.off_phi);
  const dim3 bgrid((unsigned)((L.NB + RTHREADS - 1) / RTHREADS));
  if (mixed(st))
    hipLaunchKernelGGL(rm_beams_kernel<float>, bgrid, dim3(RTHREADS), 0, stream, md, st.f32, scalar_block(st), st.comp,
                       st.n_beams, st.ld, L.NB, ws + L.off_c, ws + L.off_wr, ws + L.off_wi, ws + L.off_wk,
                       ws + L.off_cmp);
  else
    hipLaunchKernelGGL(rm_beams_kernel<double>, bgrid, dim3(RTHREADS), 0, stream, md, st.f64, scalar_block(st),
                       st.comp, st.n_beams, st.ld, L.NB, ws + L.off_c, ws + L.off_wr, ws + L.off_wi, ws + L.off_wk,
                       ws + L.off_cmp);
  hipLaunchKernelGGL(rm_gemm_kernel, dim3((unsigned)L.pt_tiles, (unsigned)L.n_chunks), dim3(RTHREADS), 0, stream,
                     ws + L.off_wr, ws + L.off_wi, ws + L.off_wk, ws + L.off_cmp, ws + L.off_phi, L.NB, L.QP, Q,
                     L.tiles_per_chunk, ws + L.off_partial);
  hipLaunchKernelGGL(rm_reduce_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream,
                     ws + L.off_partial, L.n_chunks, len, out);
  return hipGetLastError();
}

}  // namespace shgb
