// Reverse-mode derivative of the populations for the one-dimensional QCLE
// (m = 2): one thread per beam.
//
// Objective: L = sum_i (w_re[i] Re U_i + w_im[i] Im U_i), U_i = (1/N_traj)
// sum_{l_k = i} c_k the populations (Sec. 2.3 eq:shgb integrated over x,
// Sec. 2.4 step 7), w a cotangent given by the caller.  Per beam the sweep
// starts from the adjoint of its final contribution (a2_seed), then for each
// segment of `every` intervals, last to first: the segment is run forward
// from its checkpoint, every interval's start state going to a per-thread
// slot store in the workspace, and the intervals are swept in reverse
// (a2_interval_rev), accumulating the derivative with respect to
// (A, B, C, D); the adjoint of the initial p1 is that of p_mean (the mean
// initial momentum shifts every beam's p1).  Block partials are summed in a
// fixed order.
#include "adjoint_m2.h"

namespace shgb {

constexpr int kAdjThreads = 256;
constexpr int64_t kAdjM2MaxBlocks = 512;
constexpr int kSlotF = 15;   // 12 integrated values, E, comp, nhop
constexpr int kTraj2 = 10;   // trajectory rows of an m = 2 state: X, P, Re Z, Im Z

int64_t adj_m2_blocks(int64_t n) {
  int64_t b = (n + kAdjThreads - 1) / kAdjThreads;
  if (b < 1) b = 1;
  return b < kAdjM2MaxBlocks ? b : kAdjM2MaxBlocks;
}

int64_t adj_m2_workspace_bytes(int64_t n, int every) {
  const int64_t threads = adj_m2_blocks(n) * kAdjThreads;
  return threads * (int64_t)every * kSlotF * 8 + adj_m2_blocks(n) * kAdjVals * 8;
}

__device__ inline void a2_load(const double *f, int64_t ld, int64_t b, A2 &y) {
  const Layout L(2, ld);
  y.q = f[L.X(0) * ld + b];
  y.p = f[L.X(1) * ld + b];
  y.Pq = f[L.P(0) * ld + b];
  y.Pp = f[L.P(1) * ld + b];
  y.zr11 = f[L.Zre(0) * ld + b];
  y.zr12 = f[L.Zre(1) * ld + b];
  y.zr22 = f[L.Zre(2) * ld + b];
  y.zi11 = f[L.Zim(0) * ld + b];
  y.zi12 = f[L.Zim(1) * ld + b];
  y.zi22 = f[L.Zim(2) * ld + b];
  const double *sc = f + (int64_t)kTraj2 * ld;
  y.S = sc[kRowS * ld + b];
  y.Lam = sc[kRowLam * ld + b];
}

__global__ void __launch_bounds__(kAdjThreads)
adjoint_m2_kernel(DevModel md, const double *__restrict__ fin, const int32_t *__restrict__ fcomp, int64_t n,
                  int64_t ld, uint64_t gid0, const char *__restrict__ ckpt, CkptLayout cl, int nsteps, double dt,
                  uint64_t seed, int every, const double *__restrict__ cot, double inv_ntraj, double *__restrict__ slots,
                  double *__restrict__ partial) {
  const int64_t nthr = (int64_t)gridDim.x * kAdjThreads;
  const int64_t t = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
  const double norm = 2.0 * M_PI * md.eps;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t b = t; b < n; b += nthr) {
    // adjoint of the final contribution
    A2 y;
    a2_load(fin, ld, b, y);
    const double *fs = fin + (int64_t)kTraj2 * ld;
    const int l = fcomp[b];
    const cd w = {cot[2 * l] * inv_ntraj, -cot[2 * l + 1] * inv_ntraj};
    A2 yb;
    double logwb;
    acc[5] += a2_seed(md.eps, norm, y, fs[kRowLogw * ld + b], {fs[kRowPhre * ld + b], fs[kRowPhim * ld + b]},
                      {fs[kRowAre * ld + b], fs[kRowAim * ld + b]}, w, yb, logwb);
    double th[4] = {0.0, 0.0, 0.0, 0.0};
    const uint64_t gid = gid0 + (uint64_t)b;
    Counters cnt;
    for (int c = cl.n_ckpt - 1; c >= 0; --c) {
      const int start = c * every, len = nsteps - start < every ? nsteps - start : every;
      const char *base = ckpt + (int64_t)c * cl.stride_bytes;
      A2 ys;
      a2_load((const double *)base, n, b, ys);
      const double *cs = (const double *)base + (int64_t)kTraj2 * n;
      const int32_t *ci = (const int32_t *)(base + cl.rows * n * 8);
      HopScalars hs;
      hs.logw = 0.0;
      hs.phre = 1.0;
      hs.phim = 0.0;
      hs.Lam = 0.0;
      hs.E = cs[kRowE * n + b];
      hs.comp = ci[b];
      hs.nhop = (uint32_t)ci[n + b];
      // forward over the segment, keeping every interval's start
      for (int i = 0; i < len; ++i) {
        double *sl = slots + (int64_t)i * kSlotF * nthr + t;
        int f = 0;
#define F(x) sl[(f++) * nthr] = ys.x;
        SHGB_A2_FIELDS(F)
#undef F
        sl[12 * nthr] = hs.E;
        sl[13 * nthr] = (double)hs.comp;
        sl[14 * nthr] = (double)hs.nhop;
        double rem;
        a2_legs(md, ys, hs, gid, seed, dt, -1, rem, cnt);
      }
      // reverse over the segment
      for (int i = len - 1; i >= 0; --i) {
        const double *sl = slots + (int64_t)i * kSlotF * nthr + t;
        int f = 0;
#define F(x) ys.x = sl[(f++) * nthr];
        SHGB_A2_FIELDS(F)
#undef F
        hs.E = sl[12 * nthr];
        hs.comp = (int)sl[13 * nthr];
        hs.nhop = (uint32_t)sl[14 * nthr];
        a2_interval_rev(md, ys, hs, gid, seed, dt, yb, logwb, th);
      }
    }
    acc[0] += th[0];
    acc[1] += th[1];
    acc[2] += th[2];
    acc[3] += th[3];
    acc[4] += yb.p;
  }
  // block sum in a fixed order
  __shared__ double red[kAdjThreads / 64][6];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double s = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < kAdjVals) {
    double s = 0.0;
    if (threadIdx.x < 6)
      for (int w = 0; w < kAdjThreads / 64; ++w) s += red[w][threadIdx.x];
    partial[(int64_t)blockIdx.x * kAdjVals + threadIdx.x] = s;
  }
}

hipError_t launch_adj_final(const double *, int64_t, double *, hipStream_t);

hipError_t launch_adjoint_m2(const DevModel &md, const shgb_state &fin, const void *ckpt, int nsteps, double dt,
                             uint64_t seed, int every, const double *cot, int64_t n_traj, double *out, void *work,
                             hipStream_t stream) {
  const int64_t n = fin.n_beams;
  const int64_t blocks = adj_m2_blocks(n);
  const int64_t threads = blocks * kAdjThreads;
  double *slots = (double *)work;
  double *partial = slots + threads * (int64_t)every * kSlotF;
  const CkptLayout cl = ckpt_layout(n, 2, nsteps, every);
  hipLaunchKernelGGL(adjoint_m2_kernel, dim3((unsigned)blocks), dim3(kAdjThreads), 0, stream, md, fin.f64, fin.comp,
                     n, fin.ld, fin.beam_id_offset, (const char *)ckpt, cl, nsteps, dt, seed, every, cot,
                     1.0 / (double)n_traj, slots, partial);
  return launch_adj_final(partial, blocks, out, stream);
}

}  // namespace shgb
