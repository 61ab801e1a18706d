// Superposition at evaluation points for phase space m = 24 on the FP32
// matrix cores (Sec. 2.3 eq:shgb, Sec. 2.4 step 6): the mixed-precision
// form of reconstruct_mfma.hip.
//
// As there, the exponent of beam k at point x is the contraction of beam
// weights W[k][f] with point features Phi[f](x) (F = 325 features: the
// quadratic monomials, the coordinates and 1), here in FP32 on
// v_mfma_f32_16x16x4f32.  FP32 keeps about seven digits of each term, and the
// terms of the contraction grow with the distance of x and X from the centre
// they are taken about, so every tile of 64 beams has its own centre c (the
// mean of its beams' centres): W is formed in FP64 from X - c and rounded
// once; the point features are formed per tile from x - c (rounded to FP32
// from FP64) inside the kernel.  The beam weight exp(omega) A exp(iS/eps) is
// formed per beam in FP64, exp and sincos of the exponent in FP32, and every
// term is added to FP64 sums.  What remains is the cancellation inside the
// quadratic form of a strongly squeezed beam (Hessian eigenvalues from 1e-3
// to 1e3 on the 2000-interval ensemble), which FP32 cannot resolve: the field
// error is stated (about 1e-3 of sum |w G| at worst, 1e-4 relative L2) and
// the FP64 kernel stays the default.
//
// v_mfma_f32_16x16x4f32 lane layout (checked on gfx950): A[i][k] in lane
// i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane j + 16 (i / 4), register
// i % 4.  Wave w of a block owns beams 16w .. 16w + 15 of the tile (rows) and
// the block's 64 points as four groups of 16 (columns).
#include "device.h"

namespace shgb {

constexpr int R3M = 24;
constexpr int R3T = R3M * (R3M + 1) / 2;   // 300 quadratic features
constexpr int R3F = R3T + R3M + 1;         // 325
constexpr int R3FP = (R3F + 3) / 4 * 4;    // 328: whole k-steps of 4
constexpr int R3BK = 64;                   // beams per tile
constexpr int R3BQ = 64;                   // points per block
constexpr int R3THREADS = 256;
constexpr int64_t R3BLOCKS = 2048;
constexpr int64_t R3MAXCHUNK = 512;

struct Rm32Layout {
  int64_t NB, QP, n_chunks, tiles_per_chunk, pt_tiles;
  int64_t off_ct, off_wr, off_wi, off_wk, off_cmp, off_partial, total;   // bytes
};

Rm32Layout rm32_layout(int64_t n, int64_t Q) {
  Rm32Layout L;
  L.NB = (n + R3BK - 1) / R3BK * R3BK;
  if (L.NB == 0) L.NB = R3BK;
  L.QP = (Q + R3BQ - 1) / R3BQ * R3BQ;
  if (L.QP == 0) L.QP = R3BQ;
  L.pt_tiles = L.QP / R3BQ;
  const int64_t beam_tiles = L.NB / R3BK;
  int64_t nc = (R3BLOCKS + L.pt_tiles - 1) / L.pt_tiles;
  if (nc > R3MAXCHUNK) nc = R3MAXCHUNK;
  if (nc > beam_tiles) nc = beam_tiles;
  if (nc < 1) nc = 1;
  L.tiles_per_chunk = (beam_tiles + nc - 1) / nc;
  L.n_chunks = (beam_tiles + L.tiles_per_chunk - 1) / L.tiles_per_chunk;
  auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
  L.off_ct = 0;
  L.off_wr = al(L.off_ct + beam_tiles * R3M * 8);
  L.off_wi = al(L.off_wr + (int64_t)R3FP * L.NB * 4);
  L.off_wk = al(L.off_wi + (int64_t)R3FP * L.NB * 4);
  L.off_cmp = al(L.off_wk + 2 * L.NB * 8);
  L.off_partial = al(L.off_cmp + L.NB * 4);
  L.total = al(L.off_partial + L.n_chunks * SHGB_NCOMP * Q * 2 * 8);
  return L;
}

// One block of 64 threads per beam tile: the tile's centre (FP64, fixed
// order), then per beam the FP32 feature weights about it, the FP64 beam
// weight and the component.  Padded beams get zeros.
template <typename TS>
__global__ void __launch_bounds__(R3BK)
rm32_beams_kernel(DevModel md, const TS *__restrict__ fs, const double *__restrict__ sc,
                  const int32_t *__restrict__ comp, int64_t n, int64_t ld, int64_t NB, double *__restrict__ ct,
                  float *__restrict__ wr, float *__restrict__ wi, double *__restrict__ wk, int32_t *__restrict__ wc) {
  __shared__ double xs[R3BK][R3M + 1];
  __shared__ double cen[R3M];
  const int t = threadIdx.x;
  const int64_t k = (int64_t)blockIdx.x * R3BK + t;
  const bool live = k < n;
  const Layout L(R3M, ld);
  for (int i = 0; i < R3M; ++i) xs[t][i] = live ? (double)fs[L.X(i) * ld + k] : 0.0;
  __syncthreads();
  if (t < R3M) {
    const int64_t nl = n - (int64_t)blockIdx.x * R3BK;
    const int cnt = nl < R3BK ? (int)nl : R3BK;
    double s = 0.0;
    for (int b = 0; b < cnt; ++b) s += xs[b][t];
    cen[t] = s / (double)cnt;
    ct[blockIdx.x * R3M + t] = cen[t];
  }
  __syncthreads();
  if (!live) {
    for (int f = 0; f < R3FP; ++f) { wr[(int64_t)f * NB + k] = 0.0f; wi[(int64_t)f * NB + k] = 0.0f; }
    wk[2 * k] = wk[2 * k + 1] = 0.0;
    wc[k] = 0;
    return;
  }
  const double ie = 1.0 / md.eps, h2e = 0.5 / md.eps;
  double xt[R3M];
#pragma unroll
  for (int i = 0; i < R3M; ++i) xt[i] = xs[t][i] - cen[i];
  for (int f = 0, i = 0; i < R3M; ++i)
    for (int j = i; j < R3M; ++j, ++f) {
      const double s = (i == j) ? -h2e : -ie;
      wr[(int64_t)f * NB + k] = (float)(s * (double)fs[L.Zre(f) * ld + k]);
      wi[(int64_t)f * NB + k] = (float)(s * (double)fs[L.Zim(f) * ld + k]);
    }
  double cr = 0.0, ci = 0.0, px = 0.0;
  for (int i = 0; i < R3M; ++i) {
    double zr = 0.0, zi = 0.0;
    for (int j = 0; j < R3M; ++j) {
      const int tt = i <= j ? Layout::tri(R3M, i, j) : Layout::tri(R3M, j, i);
      zr += (double)fs[L.Zre(tt) * ld + k] * xt[j];
      zi += (double)fs[L.Zim(tt) * ld + k] * xt[j];
    }
    const double Pi = (double)fs[L.P(i) * ld + k];
    wr[(int64_t)(R3T + i) * NB + k] = (float)(zr * ie);
    wi[(int64_t)(R3T + i) * NB + k] = (float)((zi + Pi) * ie);
    cr += xt[i] * zr;
    ci += xt[i] * zi;
    px += Pi * xt[i];
  }
  wr[(int64_t)(R3F - 1) * NB + k] = (float)(-cr * h2e);
  wi[(int64_t)(R3F - 1) * NB + k] = (float)(-ci * h2e - px * ie);
  for (int f = R3F; f < R3FP; ++f) { wr[(int64_t)f * NB + k] = 0.0f; wi[(int64_t)f * NB + k] = 0.0f; }
  const double mag = exp(sc[kRowLogw * ld + k] + sc[kRowLam * ld + k]);
  const double pr = sc[kRowPhre * ld + k] * mag, pim = sc[kRowPhim * ld + k] * mag;
  const double ar = sc[kRowAre * ld + k], ai = sc[kRowAim * ld + k];
  double sn, cs;
  sincos(sc[kRowS * ld + k] * ie, &sn, &cs);
  const double w0r = pr * ar - pim * ai, w0i = pr * ai + pim * ar;
  wk[2 * k] = w0r * cs - w0i * sn;
  wk[2 * k + 1] = w0r * sn + w0i * cs;
  wc[k] = comp[k];
}

typedef float r3f4 __attribute__((ext_vector_type(4)));

// The exponents of one 64-beam tile at the block's 64 points on the FP32
// matrix cores, the field epilogue fused.  Point features are formed from
// x - c (c the tile's centre) in LDS: feature f is the product of columns
// fa[f] and fb[f] of the row [x - c, 1].
__global__ void __launch_bounds__(R3THREADS) __attribute__((amdgpu_waves_per_eu(2)))
rm32_gemm_kernel(const float *__restrict__ wr, const float *__restrict__ wi, const double *__restrict__ wk,
                 const int32_t *__restrict__ wc, const double *__restrict__ ct, const double *__restrict__ pts,
                 int64_t NB, int64_t Q, int64_t tiles_per_chunk, double *__restrict__ partial) {
  __shared__ float xt[R3BQ][R3M + 2];        // x - c of the block's points, column R3M = 1
  __shared__ unsigned char fa[R3FP], fb[R3FP];
  __shared__ double bw[R3BK][2];
  __shared__ int bc[R3BK];
  __shared__ double acc_s[4][2 * SHGB_NCOMP][R3BQ];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t q0 = (int64_t)blockIdx.x * R3BQ;
  const int64_t kt0 = (int64_t)blockIdx.y * tiles_per_chunk;
  // the feature table: (i, j) for the quadratic monomials, (i, 1) for the
  // coordinates, (1, 1) for the constant, (1, 1) times a zero weight for padding
  for (int f = tid; f < R3FP; f += R3THREADS) {
    int a = R3M, b = R3M;
    if (f < R3T) {
      int r = f, i = 0;
      while (r >= R3M - i) { r -= R3M - i; ++i; }
      a = i;
      b = i + r;
    } else if (f < R3T + R3M) {
      a = f - R3T;
    }
    fa[f] = (unsigned char)a;
    fb[f] = (unsigned char)b;
  }
  for (int e = tid; e < 4 * 2 * SHGB_NCOMP * R3BQ; e += R3THREADS) (&acc_s[0][0][0])[e] = 0.0;
  for (int64_t kt = kt0; kt < kt0 + tiles_per_chunk; ++kt) {
    const int64_t k0 = kt * R3BK;
    if (k0 >= NB) break;   // uniform across the block
    __syncthreads();       // the previous tile's LDS is no longer read
    for (int e = tid; e < R3BQ * R3M; e += R3THREADS) {
      const int p = e / R3M, c = e % R3M;
      const int64_t q = q0 + p;
      xt[p][c] = q < Q ? (float)(pts[q * R3M + c] - ct[kt * R3M + c]) : 0.0f;
    }
    if (tid < R3BQ) xt[tid][R3M] = 1.0f;
    if (tid < R3BK) {
      bw[tid][0] = wk[2 * (k0 + tid)];
      bw[tid][1] = wk[2 * (k0 + tid) + 1];
      bc[tid] = wc[k0 + tid];
    }
    __syncthreads();
    r3f4 er[4], ei[4];   // per point group: rows 4g + r (beams), column li (point)
#pragma unroll
    for (int v = 0; v < 4; ++v) er[v] = ei[v] = r3f4{0.f, 0.f, 0.f, 0.f};
    const int64_t beam = k0 + 16 * w + li;
#pragma unroll 2
    for (int f0 = 0; f0 < R3FP; f0 += 4) {
      const int f = f0 + g;
      const float a_r = wr[(int64_t)f * NB + beam], a_i = wi[(int64_t)f * NB + beam];
      const int ca = fa[f], cb = fb[f];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * v + li;
        const float b = xt[p][ca] * xt[p][cb];
        er[v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_r, b, er[v], 0, 0, 0);
        ei[v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_i, b, ei[v], 0, 0, 0);
      }
    }
    // epilogue: lane holds beams 16w + 4g + r (r = 0..3) at point 16v + li
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double s[2 * SHGB_NCOMP];
#pragma unroll
      for (int c = 0; c < 2 * SHGB_NCOMP; ++c) s[c] = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kb = 16 * w + 4 * g + r;
        const float e = expf(er[v][r]);
        float sn, cs;
        sincosf(ei[v][r], &sn, &cs);
        const double gr = (double)(e * cs), gi = (double)(e * sn);
        const double vr = bw[kb][0] * gr - bw[kb][1] * gi, vi = bw[kb][0] * gi + bw[kb][1] * gr;
        const int cc = bc[kb];
#pragma unroll
        for (int c = 0; c < SHGB_NCOMP; ++c) {
          s[2 * c] += (cc == c) ? vr : 0.0;
          s[2 * c + 1] += (cc == c) ? vi : 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < 2 * SHGB_NCOMP; ++c) {
        double x = s[c];
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        if (g == 0) acc_s[w][c][16 * v + li] += x;
      }
    }
  }
  __syncthreads();
  double *dst = partial + (int64_t)blockIdx.y * SHGB_NCOMP * Q * 2;
  for (int e = tid; e < 2 * SHGB_NCOMP * R3BQ; e += R3THREADS) {
    const int c = e / R3BQ, qq = e % R3BQ;
    const int64_t q = q0 + qq;
    if (q < Q)
      dst[((c >> 1) * Q + q) * 2 + (c & 1)] = (acc_s[0][c][qq] + acc_s[1][c][qq]) + (acc_s[2][c][qq] + acc_s[3][c][qq]);
  }
}

__global__ void rm32_reduce_kernel(const double *__restrict__ partial, int64_t n_chunks, int64_t len,
                                   double *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int64_t c = 0; c < n_chunks; ++c) s += partial[c * len + e];
  out[e] = s;
}

int64_t recon_mfma32_workspace_bytes(int64_t n, int64_t Q) { return rm32_layout(n, Q).total; }

bool recon_mfma32_supported(int64_t n, int64_t Q) {
  const Rm32Layout L = rm32_layout(n, Q);
  return L.NB < ((int64_t)1 << 31) / R3FP && L.QP < ((int64_t)1 << 31);
}

hipError_t launch_recon_mfma32(const DevModel &md, const shgb_state &st, const double *pts, int64_t Q, double *out,
                               void *work, hipStream_t stream) {
  if (Q == 0) return hipSuccess;
  const int64_t len = SHGB_NCOMP * Q * 2;
  const Rm32Layout L = rm32_layout(st.n_beams, Q);
  char *ws = (char *)work;
  double *partial = (double *)(ws + L.off_partial);
  if (st.n_beams == 0) {
    hipLaunchKernelGGL(rm32_reduce_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, partial,
                       (int64_t)0, len, out);
    return hipGetLastError();
  }
  double *ct = (double *)(ws + L.off_ct);
  float *wr = (float *)(ws + L.off_wr), *wi = (float *)(ws + L.off_wi);
  double *wk = (double *)(ws + L.off_wk);
  int32_t *wc = (int32_t *)(ws + L.off_cmp);
  const dim3 bgrid((unsigned)(L.NB / R3BK));
  if (mixed(st))
    hipLaunchKernelGGL(rm32_beams_kernel<float>, bgrid, dim3(R3BK), 0, stream, md, st.f32, scalar_block(st), st.comp,
                       st.n_beams, st.ld, L.NB, ct, wr, wi, wk, wc);
  else
    hipLaunchKernelGGL(rm32_beams_kernel<double>, bgrid, dim3(R3BK), 0, stream, md, st.f64, scalar_block(st),
                       st.comp, st.n_beams, st.ld, L.NB, ct, wr, wi, wk, wc);
  hipLaunchKernelGGL(rm32_gemm_kernel, dim3((unsigned)L.pt_tiles, (unsigned)L.n_chunks), dim3(R3THREADS), 0, stream,
                     wr, wi, wk, wc, ct, pts, L.NB, Q, L.tiles_per_chunk, partial);
  hipLaunchKernelGGL(rm32_reduce_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, stream, partial,
                     L.n_chunks, len, out);
  return hipGetLastError();
}

}  // namespace shgb
