// Checkpointed forward run for the reverse-mode derivative, and the final
// sum of the reverse kernels' block partials.
//
// The forward run is the ordinary stepping (shgb_step_ensemble's kernels,
// called once per segment of `every` intervals); before each segment the
// whole state is copied into its checkpoint.  Splitting the run into calls
// leaves an FP64 state bitwise as one call would.  With a record buffer
// (d > 1) each segment is run by the recording stepping kernel instead,
// which keeps every interval's stage records and the start states of the
// intervals with a hop, so that the reverse sweep need not run the segments
// again: segment c's records are at recs + c n every adj_interval_rec(d),
// in the layout of one replay, and after the n_seg segments' records come
// the segments' slots, segment c's at
// recs + n_seg n every adj_interval_rec(d) + c n kAdjSlots adj_slot_doubles(d).
#include "adjoint.h"

namespace shgb {

hipError_t launch_step_m2(const DevModel &, const shgb_state &, int, double, uint64_t, uint64_t *, hipStream_t);
hipError_t launch_step_wave(const DevModel &, const shgb_state &, int, double, uint64_t, uint64_t *, hipStream_t);
hipError_t launch_step_wave_record(const DevModel &, const shgb_state &, int, double, uint64_t, double *, int,
                                   double *, uint64_t *, hipStream_t);

// Copy the FP64 state (rows of ld) into a checkpoint (rows of n).
__global__ void __launch_bounds__(256) ckpt_save_kernel(const double *__restrict__ f64, const int32_t *__restrict__ comp,
                                                        const uint32_t *__restrict__ nhop, int64_t n, int64_t ld,
                                                        int64_t rows, char *__restrict__ dst) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double *d = (double *)dst;
  for (int64_t f = 0; f < rows; ++f) d[f * n + b] = f64[f * ld + b];
  int32_t *di = (int32_t *)(dst + rows * n * 8);
  di[b] = comp[b];
  di[n + b] = (int32_t)nhop[b];
}

hipError_t launch_step_checkpointed(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                                    int every, void *ckpt, double *recs, uint64_t *diag, hipStream_t stream) {
  const CkptLayout cl = ckpt_layout(st.n_beams, st.m, nsteps, every);
  if (st.n_beams == 0) return hipSuccess;
  if (recs && st.m == 2) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((st.n_beams + 255) / 256);
  const int64_t seg = st.n_beams * (int64_t)every * adj_interval_rec(st.m / 2);
  const int64_t sseg = st.n_beams * (int64_t)kAdjSlots * adj_slot_doubles(st.m / 2);
  double *slots = recs ? recs + cl.n_ckpt * seg : nullptr;
  for (int c = 0; c < cl.n_ckpt; ++c) {
    hipLaunchKernelGGL(ckpt_save_kernel, dim3(blocks), dim3(256), 0, stream, st.f64, st.comp, st.nhop, st.n_beams,
                       st.ld, cl.rows, (char *)ckpt + (int64_t)c * cl.stride_bytes);
    const int len = nsteps - c * every < every ? nsteps - c * every : every;
    const hipError_t e =
        recs        ? launch_step_wave_record(md, st, len, dt, seed, recs + c * seg, every, slots + c * sseg, diag,
                                              stream)
        : st.m == 2 ? launch_step_m2(md, st, len, dt, seed, diag, stream)
                    : launch_step_wave(md, st, len, dt, seed, diag, stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Sum the partial rows (kAdjVals doubles each: per block or per beam) into
// the six outputs: 256 lanes take rows k, k + 256, ... in order, then a
// fixed tree over the lanes (the same order on every call).
__global__ void __launch_bounds__(256) adj_final_kernel(const double *__restrict__ partial, int64_t nrows,
                                                        double *__restrict__ out) {
  __shared__ double red[6][256];
  const int t = threadIdx.x;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t r = t; r < nrows; r += 256)
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] += partial[r * kAdjVals + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) red[k][t] = s[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int k = 0; k < 6; ++k) red[k][t] += red[k][t + h];
    __syncthreads();
  }
  if (t < 6) out[t] = red[t][0];
}

hipError_t launch_adj_final(const double *partial, int64_t nblocks, double *out, hipStream_t stream) {
  hipLaunchKernelGGL(adj_final_kernel, dim3(1), dim3(256), 0, stream, partial, nblocks, out);
  return hipGetLastError();
}

}  // namespace shgb
