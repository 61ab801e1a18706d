// Initial beam sampling (Sec. 2.5, Sec. 2.4 step 2) and the stand-alone hop
// event (Sec. 2.4 step 5) for listed beams; one thread per beam.
#include "device.h"

namespace shgb {

// Standard normal for phase-space coordinate c of beam gid: Box-Muller
// (Box & Muller 1958) on the words of Philox block (gid, c/4, NORMAL).
__device__ inline double normal_coord(uint64_t seed, uint64_t gid, int c) {
  const U64x4 w = draw(seed, gid, (uint64_t)(c / 4), kTagNormal);
  const int pair = (c % 4) / 2;
  const double u1 = u01(w.v[2 * pair]);
  const double u2 = u01(w.v[2 * pair + 1]);
  const double r = sqrt(-2.0 * log(u1));
  const double ang = (2.0 * M_PI) * u2;
  return (c % 2 == 0) ? r * cos(ang) : r * sin(ang);
}

__global__ void __launch_bounds__(256)
init_kernel(DevModel md, shgb_init_spec spec, double *__restrict__ f, int32_t *__restrict__ comp,
            uint32_t *__restrict__ nhop, int64_t n, int64_t ld, int m, uint64_t gid0, uint64_t seed,
            double A0) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const Layout L(m, ld);
  const int d = md.d;
  const uint64_t gid = gid0 + (uint64_t)b;
  f[L.X(0) * ld + b] = spec.q_mean + spec.q_std * normal_coord(seed, gid, 0);
  double p1;
  if (spec.p_dist == SHGB_DIST_NORMAL) {
    p1 = spec.p_a + spec.p_b * normal_coord(seed, gid, d);
  } else {
    const U64x4 w = draw(seed, gid, (uint64_t)d, kTagUnif);
    p1 = spec.p_a + (spec.p_b - spec.p_a) * u01(w.v[0]);
  }
  f[L.X(d) * ld + b] = p1;
  for (int k = 1; k < d; ++k) {
    const double wk = md.bath_w[k];
    f[L.X(k) * ld + b] = sqrt(md.eps / (2.0 * md.mass * wk)) * normal_coord(seed, gid, k);
    f[L.X(d + k) * ld + b] = sqrt(md.eps * md.mass * wk / 2.0) * normal_coord(seed, gid, d + k);
  }
  for (int i = 0; i < m; ++i) f[L.P(i) * ld + b] = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j) {
      const int t = Layout::tri(m, i, j);
      f[L.Zre(t) * ld + b] = (i == j) ? 1.0 : 0.0;
      f[L.Zim(t) * ld + b] = 0.0;
    }
  f[L.S() * ld + b] = 0.0;
  f[L.Are() * ld + b] = A0;
  f[L.Aim() * ld + b] = 0.0;
  f[L.logw() * ld + b] = 0.0;
  f[L.phre() * ld + b] = 1.0;
  f[L.phim() * ld + b] = 0.0;
  f[L.Lam() * ld + b] = 0.0;
  const U64x4 w = draw(seed, gid, 0, kTagHop);
  f[L.E() * ld + b] = -log(1.0 - u01(w.v[1]));
  comp[b] = spec.comp0;
  nhop[b] = 0u;
}

hipError_t launch_init(const DevModel &md, const shgb_init_spec &spec, const shgb_state &st,
                       uint64_t seed, hipStream_t stream) {
  if (st.n_beams == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (st.n_beams + threads - 1) / threads;
  const double A0 = pow(2.0 * M_PI * md.eps, -0.5 * st.m);
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, md, spec, st.f64,
                     st.comp, st.nhop, st.n_beams, st.ld, st.m, st.beam_id_offset, seed, A0);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
hop_kernel(DevModel md, double *__restrict__ f, int32_t *__restrict__ comp,
           uint32_t *__restrict__ nhop, int64_t n, int64_t ld, int m, uint64_t gid0,
           const int32_t *__restrict__ idx, int64_t n_idx, uint64_t seed, uint64_t *diag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Counters cnt;
  uint32_t bad = 0;
  if (t < n_idx) {
    const int64_t b = idx[t];
    if (b < 0 || b >= n) {
      bad = 1;
    } else {
      const Layout L(m, ld);
      const int d = m / 2;
      HopScalars h;
      h.logw = f[L.logw() * ld + b];
      h.phre = f[L.phre() * ld + b];
      h.phim = f[L.phim() * ld + b];
      h.Lam = f[L.Lam() * ld + b];
      h.E = f[L.E() * ld + b];
      h.comp = comp[b];
      h.nhop = nhop[b];
      hop_event(md, f[L.X(0) * ld + b], f[L.X(d) * ld + b], h, gid0 + (uint64_t)b, seed, cnt);
      f[L.logw() * ld + b] = h.logw;
      f[L.phre() * ld + b] = h.phre;
      f[L.phim() * ld + b] = h.phim;
      f[L.Lam() * ld + b] = h.Lam;
      f[L.E() * ld + b] = h.E;
      comp[b] = h.comp;
      nhop[b] = h.nhop;
    }
  }
  flush_counters(cnt, diag);
  if (diag) {
    uint32_t x = bad;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd((unsigned long long *)&diag[SHGB_DIAG_BAD_INDEX], (unsigned long long)x);
  }
}

hipError_t launch_hop(const DevModel &md, const shgb_state &st, const int32_t *idx, int64_t n_idx,
                      uint64_t seed, uint64_t *diag, hipStream_t stream) {
  if (n_idx == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (n_idx + threads - 1) / threads;
  hipLaunchKernelGGL(hop_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, md, st.f64, st.comp,
                     st.nhop, st.n_beams, st.ld, st.m, st.beam_id_offset, idx, n_idx, seed, diag);
  return hipGetLastError();
}

__global__ void philox_kernel(uint64_t seed, const uint64_t *__restrict__ ctr, uint64_t *__restrict__ out,
                              int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const U64x4 r = philox4x64_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], seed, 0);
  for (int k = 0; k < 4; ++k) out[4 * i + k] = r.v[k];
}

hipError_t launch_philox(uint64_t seed, const uint64_t *ctr, uint64_t *out, int64_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const int threads = 256;
  hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, stream,
                     seed, ctr, out, n);
  return hipGetLastError();
}

}  // namespace shgb
