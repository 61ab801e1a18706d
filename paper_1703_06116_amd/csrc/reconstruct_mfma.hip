// Superposition at evaluation points for phase space m = 24 on the FP64
// matrix cores (Sec. 2.3 eq:shgb, Sec. 2.4 step 6).
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
// 328).  It runs on v_mfma_f64_4x4x4f64 (four 4 x 4 blocks per instruction,
// which issues at the full FP64 matrix rate on gfx950, where the 16 x 16
// form reaches about half of it); the epilogue multiplies
// exp(Re) (cos Im + i sin Im) by the beam weight exp(omega) A exp(iS/eps)
// and sums per component and point.  Blocks own 64 points and a chunk of
// beams (64 per tile); partial sums per chunk are added in chunk order.
#include "device.h"

namespace shgb {

constexpr int RM = 24;
constexpr int RT = RM * (RM + 1) / 2;  // 300 quadratic features
constexpr int RF = RT + RM + 1;        // 325
#ifndef SHGB_RM_SLAB
#define SHGB_RM_SLAB 8
#endif
constexpr int RKS = SHGB_RM_SLAB;      // features per LDS slab (RKS / 4 MFMA k-steps)
constexpr int RFP = (RF + RKS - 1) / RKS * RKS;  // padded to a multiple of the slab
constexpr int RNSLAB = RFP / RKS;
constexpr int RBK = 64;                // beams per block tile (16 per wave)
constexpr int RBQ = 64;                // points per block tile
constexpr int RTHREADS = 256;
static_assert(RKS % 8 == 0 && RBK == 64 && RBQ == 64 && RTHREADS == 256,
              "the slab copy: four waves, rows of 64 doubles, two rows per instruction");
constexpr int64_t RBLOCKS = 2048;      // aim: 8 workgroups per CU over the launch
constexpr int64_t RMAXCHUNK = 512;
constexpr int kBufferFlags = 0x00020000;   // word 3 of a raw (untyped) buffer resource on gfx9

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
  // enough blocks to fill the chip several times when the work allows
  int64_t nc = (RBLOCKS + L.pt_tiles - 1) / L.pt_tiles;
  if (nc > RMAXCHUNK) nc = RMAXCHUNK;
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
// Wave w owns beams 16 w .. 16 w + 15 of the block tile and all 64 points,
// for Re and for Im.  v_mfma_f64_4x4x4f64 lane layout (checked on gfx950):
// block b, A_b[i][k] from lane 16k + 4b + i, B_b[k][j] from lane
// 16k + 4b + j, D_b[i][j] in lane 16i + 4b + j.  With A the same in all four
// blocks (four beams) and block b taking points 4b..4b+3 of a 16-point
// group, one instruction gives 4 beams x 16 points, lane l holding beam
// l / 16 and point l % 16; a wave tile is 4 beam quads x 4 point groups.
// Registers (at most 168 per lane) and LDS (two slab buffers, 42 KB in all)
// let three workgroups share a CU, so one's slab barriers and epilogue
// (exp, sincos) overlap the others' matrix work.  After each beam
// tile the epilogue values are summed over the lane's beams, then across
// the four lane groups, and added to per-point accumulators in LDS.
__global__ void __launch_bounds__(RTHREADS) __attribute__((amdgpu_waves_per_eu(3)))
rm_gemm_kernel(const double *__restrict__ wr, const double *__restrict__ wi, const double *__restrict__ wk,
               const double *__restrict__ wc, const double *__restrict__ phi, int64_t NB, int64_t QP, int64_t Q,
               int64_t tiles_per_chunk, double *__restrict__ partial) {
  // the two slab buffers as separate objects, so that reads of one are not
  // ordered behind the copies into the other
  __shared__ double Ws0[2][RKS][RBK], Ws1[2][RKS][RBK];   // [re/im][feature][beam]
  __shared__ double Ps0[RKS][RBQ], Ps1[RKS][RBQ];         // [feature][point]
  __shared__ double Bw[RBK][3];           // beam weight re, im, component
  __shared__ double Acc[4][2 * SHGB_NCOMP][RBQ];  // [wave][comp re/im][point]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, li = lane & 15, i4 = lane & 3;
  const int64_t q0 = (int64_t)blockIdx.x * RBQ;
  const int64_t kt0 = (int64_t)blockIdx.y * tiles_per_chunk;
  for (int e = tid; e < 4 * 2 * SHGB_NCOMP * RBQ; e += RTHREADS) (&Acc[0][0][0])[e] = 0.0;
  // Slabs are copied from global memory straight into LDS (two buffers) by
  // 16-byte buffer loads with an LDS destination: lane l of a wave writes
  // bytes [16 l, 16 l + 16) from the wave's LDS base (checked on gfx950), so
  // one instruction fills two 64-double rows of a slab.  The W slab has
  // 2 RKS rows (Re, Im), the Phi slab RKS; each wave copies RKS / 4 W row
  // pairs and RKS / 8 Phi row pairs.  The copy of slab s + 1 runs under the
  // matrix work of slab s.
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const uint32_t wvo = (uint32_t)(((int64_t)(lane >> 5) * NB + 2 * (lane & 31)) * 8);
  const uint32_t pvo = (uint32_t)(((int64_t)(lane >> 5) * QP + 2 * (lane & 31)) * 8);
  auto rsrc = [](const double *base, int64_t n_after) {
    const int64_t bytes = n_after * 8;
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff),
                                             kBufferFlags);
  };
  typedef __attribute__((address_space(3))) void *lds_ptr;
  auto copy_slab = [&](int64_t k0, int s, double (&Wd)[2][RKS][RBK], double (&Pd)[RKS][RBQ]) {
#pragma unroll
    for (int h = 0; h < RKS / 4; ++h) {
      const int j = wu * (RKS / 4) + h, part = j / (RKS / 2), f0 = 2 * (j % (RKS / 2));
      const int64_t fw = (int64_t)(s * RKS + f0) * NB + k0;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc((part ? wi : wr) + fw, (int64_t)RFP * NB - fw),
                                               (lds_ptr)&Wd[part][f0][0], 16, wvo, 0, 0, 0);
    }
#pragma unroll
    for (int h = 0; h < RKS / 8; ++h) {
      const int f0 = 2 * (wu * (RKS / 8) + h);
      const int64_t fp = (int64_t)(s * RKS + f0) * QP + q0;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc(phi + fp, (int64_t)RFP * QP - fp), (lds_ptr)&Pd[f0][0], 16,
                                               pvo, 0, 0, 0);
    }
  };
  for (int64_t kt = kt0; kt < kt0 + tiles_per_chunk; ++kt) {
    const int64_t k0 = kt * RBK;
    if (k0 >= NB) break;  // uniform across the block
    double are[4][4], aim[4][4];   // [beam quad][point group]
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) { are[u][v] = 0.0; aim[u][v] = 0.0; }
    copy_slab(k0, 0, Ws0, Ps0);
    if (tid < RBK) {
      Bw[tid][0] = wk[2 * (k0 + tid)];
      Bw[tid][1] = wk[2 * (k0 + tid) + 1];
      Bw[tid][2] = wc[k0 + tid];
    }
    __builtin_amdgcn_s_waitcnt(0);   // this wave's copies have landed
    __syncthreads();
    // slab s from (Wc, Pc) while slab s + 1 is copied into (Wn, Pn)
    auto slab = [&](int s, const double (&Wc)[2][RKS][RBK], const double (&Pc)[RKS][RBQ],
                    double (&Wn)[2][RKS][RBK], double (&Pn)[RKS][RBQ]) {
      if (s + 1 < RNSLAB) copy_slab(k0, s + 1, Wn, Pn);
      // every operand of the slab from LDS first, then the slab's MFMAs back to back
      double bq[RKS / 4][4], aqr[RKS / 4][4], aqi[RKS / 4][4];
#pragma unroll
      for (int ks = 0; ks < RKS / 4; ++ks) {
        const int f = 4 * ks + g;
#pragma unroll
        for (int v = 0; v < 4; ++v) bq[ks][v] = Pc[f][16 * v + li];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          aqr[ks][u] = Wc[0][f][16 * w + 4 * u + i4];
          aqi[ks][u] = Wc[1][f][16 * w + 4 * u + i4];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int ks = 0; ks < RKS / 4; ++ks)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            are[u][v] = __builtin_amdgcn_mfma_f64_4x4x4f64(aqr[ks][u], bq[ks][v], are[u][v], 0, 0, 0);
            aim[u][v] = __builtin_amdgcn_mfma_f64_4x4x4f64(aqi[ks][u], bq[ks][v], aim[u][v], 0, 0, 0);
          }
      // the next slab's copy must have landed (this wave's part) before the
      // barrier that publishes it; keep both behind the matrix work
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    };
    for (int s = 0; s < RNSLAB; s += 2) {
      slab(s, Ws0, Ps0, Ws1, Ps1);
      if (s + 1 < RNSLAB) slab(s + 1, Ws1, Ps1, Ws0, Ps0);
    }
    // epilogue, one point group at a time: w_k exp(E) per (beam, point), summed over the
    // lane's 4 beams per component, then over the four lane groups
#pragma unroll
    for (int pt = 0; pt < 4; ++pt) {
      double v[2 * SHGB_NCOMP];
#pragma unroll
      for (int c = 0; c < 2 * SHGB_NCOMP; ++c) v[c] = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kb = 16 * w + 4 * u + g;
        const double e = exp(are[u][pt]);
        double sn, cs;
        sincos(aim[u][pt], &sn, &cs);
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
        if (g == 0) Acc[w][c][16 * pt + li] += x;
      }
    }
    __syncthreads();  // Bw and the slab buffers are rewritten by the next tile
  }
  // add the four wave rows and write this chunk's partial sums
  double *dst = partial + (int64_t)blockIdx.y * SHGB_NCOMP * Q * 2;
  for (int e = tid; e < 2 * SHGB_NCOMP * RBQ; e += RTHREADS) {
    const int c = e / RBQ, qq = e % RBQ;
    const int64_t q = q0 + qq;
    if (q < Q) dst[((c >> 1) * Q + q) * 2 + (c & 1)] = (Acc[0][c][qq] + Acc[1][c][qq]) + (Acc[2][c][qq] + Acc[3][c][qq]);
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

// The slab copies address a feature row pair from a per-slab base with
// 32-bit byte offsets (two rows of NB or QP doubles): both counts below 2^26.
bool recon_mfma_supported(int64_t n, int64_t Q) {
  const RmLayout L = rm_layout(n, Q);
  return L.NB < ((int64_t)1 << 26) && L.QP < ((int64_t)1 << 26);
}

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
