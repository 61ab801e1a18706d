// Component populations (Sec. 2.3 eq:shgb integrated over x; Sec. 2.4
// steps 6-7).  For each beam
//   c = exp(logw + Lam) phase A exp(iS/eps) (2 pi eps)^(m/2) det(Z)^(-1/2)
//       exp(-P^T Z^-1 P / (2 eps)),
// the closed-form integral of exp(omega) G over R^m, with Z = L D L^T
// (complex symmetric, no pivoting: Re Z = M is positive definite, so every
// pivot has a positive real part) giving det(Z)^(1/2) = prod sqrt(d_j)
// (principal roots: the branch continuous from real Z) and
// P^T Z^-1 P = sum_j w_j^2 / d_j with L w = P.
// Per component the kernel sums c, (Re c)^2, (Im c)^2 and the count; each
// block writes its partial sums and one block adds the partials in a fixed
// order, so the result is bitwise reproducible.  The arithmetic is FP64 for
// either trajectory precision (TS: the element type of the stored X, P, Z).
#include <mutex>

#include "cplx.h"
#include "device.h"

namespace shgb {

constexpr int kPopVals = SHGB_NCOMP * 5;
constexpr int kPopThreads = 256;
constexpr int64_t kPopMaxBlocks = 2048;

int64_t pop_blocks(int64_t n) {
  int64_t b = (n + kPopThreads - 1) / kPopThreads;
  if (b < 1) b = 1;
  return b < kPopMaxBlocks ? b : kPopMaxBlocks;
}

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Block-sum kPopVals values per thread into out[0..kPopVals) (thread 0 writes).
__device__ inline void block_sum_store(const double (&acc)[kPopVals], double *out) {
  __shared__ double red[kPopThreads / 64][kPopVals];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kPopVals; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < kPopVals) {
    double s = 0.0;
    for (int w = 0; w < kPopThreads / 64; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

__device__ inline void tally(double (&acc)[kPopVals], int comp, cd c) {
#pragma unroll
  for (int i = 0; i < SHGB_NCOMP; ++i) {
    const bool on = (comp == i);
    acc[5 * i + 0] += on ? c.re : 0.0;
    acc[5 * i + 1] += on ? c.im : 0.0;
    acc[5 * i + 2] += on ? c.re * c.re : 0.0;
    acc[5 * i + 3] += on ? c.im * c.im : 0.0;
    acc[5 * i + 4] += on ? 1.0 : 0.0;
  }
}

// exp(omega) A exp(iS/eps) for beam b
__device__ inline cd beam_weight(const double *sc, int64_t ld, int64_t b, double inv_eps) {
  const cd ph = {sc[kRowPhre * ld + b], sc[kRowPhim * ld + b]};
  const cd A = {sc[kRowAre * ld + b], sc[kRowAim * ld + b]};
  const double mag = exp(sc[kRowLogw * ld + b] + sc[kRowLam * ld + b]);
  double s, c;
  sincos(sc[kRowS * ld + b] * inv_eps, &s, &c);
  return cmul(cmul(cscale(ph, mag), A), {c, s});
}

template <typename TS>
__global__ void __launch_bounds__(kPopThreads)
pop_m2_kernel(DevModel md, const TS *__restrict__ f, const double *__restrict__ sc, const int32_t *__restrict__ comp,
              int64_t n, int64_t ld, double norm, double *__restrict__ partial, uint64_t *diag) {
  const Layout L(2, ld);
  const double inv_eps = 1.0 / md.eps;
  double acc[kPopVals];
#pragma unroll
  for (int k = 0; k < kPopVals; ++k) acc[k] = 0.0;
  uint32_t nonspd = 0;
  for (int64_t b = (int64_t)blockIdx.x * kPopThreads + threadIdx.x; b < n;
       b += (int64_t)gridDim.x * kPopThreads) {
    const cd z11 = {(double)f[L.Zre(0) * ld + b], (double)f[L.Zim(0) * ld + b]};
    const cd z12 = {(double)f[L.Zre(1) * ld + b], (double)f[L.Zim(1) * ld + b]};
    const cd z22 = {(double)f[L.Zre(2) * ld + b], (double)f[L.Zim(2) * ld + b]};
    const double P1 = f[L.P(0) * ld + b], P2 = f[L.P(1) * ld + b];
    const cd d1 = z11;
    const cd l21 = cdiv(z12, z11);
    const cd d2 = csub(z22, cmul(l21, z12));
    if (!(d1.re > 0.0) || !(d2.re > 0.0)) ++nonspd;
    const cd w1 = {P1, 0.0};
    const cd w2 = {P2 - l21.re * P1, -l21.im * P1};
    const cd quad = cadd(cdiv(cmul(w1, w1), d1), cdiv(cmul(w2, w2), d2));
    const cd sq = cmul(csqrt_principal(d1), csqrt_principal(d2));
    const cd g = cdiv(cexp(cscale(quad, -0.5 * inv_eps)), sq);
    const cd c = cscale(cmul(beam_weight(sc, ld, b, inv_eps), g), norm);
    tally(acc, comp[b], c);
  }
  block_sum_store(acc, partial + (int64_t)blockIdx.x * kPopVals);
  if (diag) {
    uint32_t x = nonspd;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd((unsigned long long *)&diag[SHGB_DIAG_NONSPD], (unsigned long long)x);
  }
}

// One wave per beam for m > 2: Z in LDS, LDL^T with lanes over the trailing
// submatrix.  kWaves beams per block.
constexpr int kPopWaves = 4;

template <int M, typename TS>
__global__ void __launch_bounds__(64 * kPopWaves)
pop_wave_kernel(DevModel md, const TS *__restrict__ f, const double *__restrict__ sc,
                const int32_t *__restrict__ comp, int64_t n, int64_t ld, double norm, double *__restrict__ partial,
                uint64_t *diag) {
  __shared__ double zr[kPopWaves][M][M + 1];
  __shared__ double zi[kPopWaves][M][M + 1];
  __shared__ double pw_re[kPopWaves][M], pw_im[kPopWaves][M];
  const Layout L(M, ld);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double inv_eps = 1.0 / md.eps;
  double acc[kPopVals];
#pragma unroll
  for (int k = 0; k < kPopVals; ++k) acc[k] = 0.0;
  uint32_t nonspd = 0;
  for (int64_t b0 = (int64_t)blockIdx.x * kPopWaves; b0 < n; b0 += (int64_t)gridDim.x * kPopWaves) {
    const int64_t b = b0 + wid;
    const bool live = b < n;
    if (live) {
      for (int t = lane; t < M * M; t += 64) {
        const int i = t / M, j = t % M;
        const int k = i <= j ? Layout::tri(M, i, j) : Layout::tri(M, j, i);
        zr[wid][i][j] = f[L.Zre(k) * ld + b];
        zi[wid][i][j] = f[L.Zim(k) * ld + b];
      }
      if (lane < M) { pw_re[wid][lane] = f[L.P(lane) * ld + b]; pw_im[wid][lane] = 0.0; }
    }
    __syncthreads();
    cd sq = {1.0, 0.0}, quad = {0.0, 0.0};
    bool bad = false;
    if (live) {
      for (int k = 0; k < M; ++k) {
        const cd dk = {zr[wid][k][k], zi[wid][k][k]};
        if (!(dk.re > 0.0)) bad = true;
        sq = cmul(sq, csqrt_principal(dk));
        const cd wk = {pw_re[wid][k], pw_im[wid][k]};
        quad = cadd(quad, cdiv(cmul(wk, wk), dk));
        // trailing update: Z_ij -= Z_ik Z_kj / d_k, w_i -= (Z_ik / d_k) w_k  (i, j > k)
        const int r = M - 1 - k;
        for (int t = lane; t < r * r; t += 64) {
          const int i = k + 1 + t / r, j = k + 1 + t % r;
          const cd lik = cdiv({zr[wid][i][k], zi[wid][i][k]}, dk);
          const cd u = cmul(lik, {zr[wid][k][j], zi[wid][k][j]});
          zr[wid][i][j] -= u.re;
          zi[wid][i][j] -= u.im;
        }
        if (lane < r) {
          const int i = k + 1 + lane;
          const cd lik = cdiv({zr[wid][i][k], zi[wid][i][k]}, dk);
          const cd u = cmul(lik, wk);
          pw_re[wid][i] -= u.re;
          pw_im[wid][i] -= u.im;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    if (live && lane == 0) {
      if (bad) ++nonspd;
      const double pre = pow(2.0 * M_PI * md.eps, 0.5 * M);
      const cd g = cscale(cdiv(cexp(cscale(quad, -0.5 * inv_eps)), sq), pre);
      const cd c = cscale(cmul(beam_weight(sc, ld, b, inv_eps), g), norm);
      tally(acc, comp[b], c);
    }
  }
  block_sum_store(acc, partial + (int64_t)blockIdx.x * kPopVals);
  if (diag) {
    uint32_t x = nonspd;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd((unsigned long long *)&diag[SHGB_DIAG_NONSPD], (unsigned long long)x);
  }
}

__global__ void __launch_bounds__(kPopThreads)
pop_final_kernel(const double *__restrict__ partial, int64_t nblocks, double *__restrict__ out) {
  double acc[kPopVals];
#pragma unroll
  for (int k = 0; k < kPopVals; ++k) acc[k] = 0.0;
  for (int64_t p = threadIdx.x; p < nblocks; p += kPopThreads)
#pragma unroll
    for (int k = 0; k < kPopVals; ++k) acc[k] += partial[p * kPopVals + k];
  block_sum_store(acc, out);
}

// Sec. 2.4 step 7: the estimate of a component's population is its sum over
// trajectories divided by N_traj.  Per component i, from the raw sums
// {sum Re c, sum Im c, sum (Re c)^2, sum (Im c)^2, count}: the mean and its
// standard error sqrt((E[x^2] - E[x]^2) / (N_traj - 1)) for the real and
// imaginary parts (the variance clipped at zero against rounding).
__global__ void pop_stats_kernel(const double *__restrict__ sums, double n_traj, double *__restrict__ stats) {
  const int i = threadIdx.x;
  if (i >= SHGB_NCOMP) return;
  const double *s = sums + 5 * i;
  const double mr = s[0] / n_traj, mi = s[1] / n_traj;
  const double vr = fmax(s[2] / n_traj - mr * mr, 0.0), vi = fmax(s[3] / n_traj - mi * mi, 0.0);
  const double k = n_traj > 1.0 ? n_traj - 1.0 : 1.0;
  stats[4 * i + 0] = mr;
  stats[4 * i + 1] = mi;
  stats[4 * i + 2] = sqrt(vr / k);
  stats[4 * i + 3] = sqrt(vi / k);
}

hipError_t launch_population_stats(const double *sums, int64_t n_traj, double *stats, hipStream_t stream) {
  hipLaunchKernelGGL(pop_stats_kernel, dim3(1), dim3(64), 0, stream, sums, (double)n_traj, stats);
  return hipGetLastError();
}

int64_t pop_workspace_bytes(int64_t n, int m) {
  const int64_t blocks = (m == 2) ? pop_blocks(n) : pop_blocks((n + kPopWaves - 1) / kPopWaves * kPopThreads);
  return blocks * kPopVals * (int64_t)sizeof(double);
}

// Partial sums of the allocation-free entry point: one array per GPU for the
// life of the process.  pop_blocks() never exceeds kPopMaxBlocks, so these
// 320 KiB hold the partials of any ensemble size.  Every block writes its
// own partial before the final kernel reads it: nothing must start at zero.
static __device__ __align__(256) double scratch[kPopMaxBlocks * kPopVals];

constexpr int kMaxDevices = 64;
int64_t pop_scratch_bytes() { return (int64_t)sizeof(scratch); }

// Device address of `scratch` on the current device (the host symbol is only a
// stand-in), looked up once per device with that device current.
hipError_t pop_scratch_ptr(void **ptr) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_populations(const DevModel &md, const shgb_state &st, double *out, void *work,
                              uint64_t *diag, hipStream_t stream) {
  double *partial = (double *)work;
  const double *sc = scalar_block(st);
  if (st.m == 2) {
    const int64_t blocks = pop_blocks(st.n_beams);
    const double norm = 2.0 * M_PI * md.eps;  // (2 pi eps)^(m/2)
    if (mixed(st))
      hipLaunchKernelGGL(pop_m2_kernel<float>, dim3((unsigned)blocks), dim3(kPopThreads), 0, stream, md, st.f32, sc,
                         st.comp, st.n_beams, st.ld, norm, partial, diag);
    else
      hipLaunchKernelGGL(pop_m2_kernel<double>, dim3((unsigned)blocks), dim3(kPopThreads), 0, stream, md, st.f64,
                         sc, st.comp, st.n_beams, st.ld, norm, partial, diag);
    hipLaunchKernelGGL(pop_final_kernel, dim3(1), dim3(kPopThreads), 0, stream, partial, blocks, out);
    return hipGetLastError();
  }
  const int64_t blocks = pop_blocks((st.n_beams + kPopWaves - 1) / kPopWaves * kPopThreads);
#define SHGB_POP_CASE(MM)                                                                             \
  case MM:                                                                                            \
    if (mixed(st))                                                                                    \
      hipLaunchKernelGGL((pop_wave_kernel<MM, float>), dim3((unsigned)blocks), dim3(64 * kPopWaves), 0, \
                         stream, md, st.f32, sc, st.comp, st.n_beams, st.ld, 1.0, partial, diag);     \
    else                                                                                              \
      hipLaunchKernelGGL((pop_wave_kernel<MM, double>), dim3((unsigned)blocks), dim3(64 * kPopWaves), 0, \
                         stream, md, st.f64, sc, st.comp, st.n_beams, st.ld, 1.0, partial, diag);     \
    break;
  switch (st.m) {
    SHGB_POP_CASE(4)
    SHGB_POP_CASE(6)
    SHGB_POP_CASE(8)
    SHGB_POP_CASE(24)
    default:
      return hipErrorInvalidValue;
  }
#undef SHGB_POP_CASE
  hipLaunchKernelGGL(pop_final_kernel, dim3(1), dim3(kPopThreads), 0, stream, partial, blocks, out);
  return hipGetLastError();
}

}  // namespace shgb
