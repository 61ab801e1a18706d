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

// TS: element type of the trajectory rows (double, or float for a mixed
// state; coordinates are drawn in FP64 and rounded once when stored).
template <typename TS>
__global__ void __launch_bounds__(256)
init_kernel(DevModel md, shgb_init_spec spec, TS *__restrict__ tr, double *__restrict__ sc,
            int32_t *__restrict__ comp, uint32_t *__restrict__ nhop, int64_t n, int64_t ld, int m, uint64_t gid0,
            uint64_t seed, double A0) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const Layout L(m, ld);
  const int d = md.d;
  const uint64_t gid = gid0 + (uint64_t)b;
  tr[L.X(0) * ld + b] = (TS)(spec.q_mean + spec.q_std * normal_coord(seed, gid, 0));
  double p1;
  if (spec.p_dist == SHGB_DIST_NORMAL) {
    p1 = spec.p_a + spec.p_b * normal_coord(seed, gid, d);
  } else {
    const U64x4 w = draw(seed, gid, (uint64_t)d, kTagUnif);
    p1 = spec.p_a + (spec.p_b - spec.p_a) * u01(w.v[0]);
  }
  tr[L.X(d) * ld + b] = (TS)p1;
  for (int k = 1; k < d; ++k) {
    const double wk = md.bath_w[k];
    tr[L.X(k) * ld + b] = (TS)(sqrt(md.eps / (2.0 * md.mass * wk)) * normal_coord(seed, gid, k));
    tr[L.X(d + k) * ld + b] = (TS)(sqrt(md.eps * md.mass * wk / 2.0) * normal_coord(seed, gid, d + k));
  }
  for (int i = 0; i < m; ++i) tr[L.P(i) * ld + b] = (TS)0;
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j) {
      const int t = Layout::tri(m, i, j);
      tr[L.Zre(t) * ld + b] = (TS)((i == j) ? 1 : 0);
      tr[L.Zim(t) * ld + b] = (TS)0;
    }
  sc[kRowS * ld + b] = 0.0;
  sc[kRowAre * ld + b] = A0;
  sc[kRowAim * ld + b] = 0.0;
  sc[kRowLogw * ld + b] = 0.0;
  sc[kRowPhre * ld + b] = 1.0;
  sc[kRowPhim * ld + b] = 0.0;
  sc[kRowLam * ld + b] = 0.0;
  const U64x4 w = draw(seed, gid, 0, kTagHop);
  sc[kRowE * ld + b] = -log(1.0 - u01(w.v[1]));
  comp[b] = spec.comp0;
  nhop[b] = 0u;
}

hipError_t launch_init(const DevModel &md, const shgb_init_spec &spec, const shgb_state &st,
                       uint64_t seed, double A0, hipStream_t stream) {
  if (st.n_beams == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (st.n_beams + threads - 1) / threads;
  double *sc = scalar_block(st);
  if (mixed(st))
    hipLaunchKernelGGL(init_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, stream, md, spec, st.f32, sc,
                       st.comp, st.nhop, st.n_beams, st.ld, st.m, st.beam_id_offset, seed, A0);
  else
    hipLaunchKernelGGL(init_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, stream, md, spec, st.f64, sc,
                       st.comp, st.nhop, st.n_beams, st.ld, st.m, st.beam_id_offset, seed, A0);
  return hipGetLastError();
}

// The hop of a listed beam at its stored state; the coupling is evaluated in
// FP64 from the stored (q1, p1).
template <typename TS>
__global__ void __launch_bounds__(256)
hop_kernel(DevModel md, const TS *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
           uint32_t *__restrict__ nhop, int64_t n, int64_t ld, int m, uint64_t gid0,
           const int32_t *__restrict__ idx, int64_t n_idx, uint64_t seed, double tie_rel, uint64_t *diag) {
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
      h.logw = sc[kRowLogw * ld + b];
      h.phre = sc[kRowPhre * ld + b];
      h.phim = sc[kRowPhim * ld + b];
      h.Lam = sc[kRowLam * ld + b];
      h.E = sc[kRowE * ld + b];
      h.comp = comp[b];
      h.nhop = nhop[b];
      hop_event(md, (double)tr[L.X(0) * ld + b], (double)tr[L.X(d) * ld + b], h, gid0 + (uint64_t)b, seed, cnt,
                tie_rel);
      sc[kRowLogw * ld + b] = h.logw;
      sc[kRowPhre * ld + b] = h.phre;
      sc[kRowPhim * ld + b] = h.phim;
      sc[kRowLam * ld + b] = h.Lam;
      sc[kRowE * ld + b] = h.E;
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
  double *sc = scalar_block(st);
  if (mixed(st))
    hipLaunchKernelGGL(hop_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, stream, md, st.f32, sc, st.comp,
                       st.nhop, st.n_beams, st.ld, st.m, st.beam_id_offset, idx, n_idx, seed, kTieRelMixed, diag);
  else
    hipLaunchKernelGGL(hop_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, stream, md, st.f64, sc, st.comp,
                       st.nhop, st.n_beams, st.ld, st.m, st.beam_id_offset, idx, n_idx, seed, kTieRel, diag);
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
