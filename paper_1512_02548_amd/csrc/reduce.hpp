// Deterministic reductions shared by the Krylov kernels and the stiffness
// kernel's fused inner products: wavefront butterflies, the last-workgroup
// detection of single-launch reductions, and the final sum of per-workgroup
// partials in a fixed order.
#pragma once
#include <hip/hip_runtime.h>

#include "mfma.hpp"
#include "sem_internal.hpp"

namespace sem {

// butterfly sum over a 64-lane wavefront (every lane gets the total)
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Whether this workgroup is the last of nblk to finish its partials.  The
// barrier orders every wave's partial stores before thread 0's count, whose
// device-scope release makes them visible and whose acquire (in the last
// workgroup) makes the others' visible; the second barrier passes that on to
// the workgroup.  (One release-acquire operation per workgroup: a device-scope
// fence in every thread cost about 1.3 us more per launch.)
__device__ inline bool last_block(int32_t* counter, int nblk) {
  __shared__ int is_last;
  __syncthreads();
  if (threadIdx.x == 0)
    is_last = (__hip_atomic_fetch_add(counter, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == nblk - 1);
  __syncthreads();
  return is_last != 0;
}

// final sums of nblk partials: wave w takes vectors w, w+4, ...; lanes stride
// over the workgroup partials in a fixed order, then a butterfly
// (a lane's partials are requested four at a time from clamped addresses and
// added in order, so that one round trip serves four of them)
__device__ __forceinline__ double lane_partials(const double* __restrict__ part, int ldp, int k, int nblk, int lane) {
  double t = 0;
  for (int b0 = lane; b0 < nblk; b0 += 4 * 64) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[(size_t)min(b0 + 64 * u, nblk - 1) * ldp + k];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (b0 + 64 * u < nblk) t += v[u];
  }
  return t;
}

__device__ __forceinline__ void dots_reduce(int nvec, const double* __restrict__ part, int ldp,
                                            double* __restrict__ out, int nblk) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = wv; k < nvec; k += kBlockThreads / 64) {
    double t = lane_partials(part, ldp, k, nblk, lane);
    t = wave_sum(t);
    if (lane == 0) out[k] = t;
  }
}

// Block b's part of <y, V_i>, i < nvec, from its own contributions to an
// element-kernel output (blocks of cb columns of a tank of nx columns, nc
// nodes per column, nl per line): the nodes of its columns (in y) and its
// right line (in the side buffer), so that the sum over the blocks is the
// product with the fixed-up output without a fix-up before it; into
// part[b][i].  Thread-strided sums over the block's nodes, wave butterflies,
// the four wave totals in order.  The block's values must be visible to the
// workgroup.  Used by the single-tank stiffness launch (fused) and by the
// batched products, so that the two give the same sums.
template <typename T>
__device__ inline void block_dots_part(int cb, int nx, int nc, int nl, int periodic, const T* __restrict__ y,
                                       const T* __restrict__ side, const T* __restrict__ V, int64_t n, int nvec,
                                       double* __restrict__ part, int ldp, int b) {
  static_assert(kBlockThreads == 256, "four wave totals");
  __shared__ double red[kBlockThreads / 64][kMaxVec];
  const int c0 = b * cb, cbb = min(cb, nx - c0);
  const int nown = cbb * nc, nq = nown + nl;
  const int64_t obase = (int64_t)c0 * nc;
  const int64_t rbase = (c0 + cbb < nx) ? (int64_t)(c0 + cbb) * nc : (periodic ? 0 : (int64_t)nx * nc);
  const int lane = threadIdx.x & 63, wv = wave_id();
  const SEM_GLOBAL T* yg = gview(y);
  const SEM_GLOBAL T* sg = gview(side);
  const SEM_GLOBAL T* vg = gview(V);
  // eight vectors per pass, a thread's nodes two at a time (their loads
  // requested together, from clamped addresses; the sums run over its nodes
  // in order)
  constexpr int U = 2;
  for (int k0 = 0; k0 < nvec; k0 += 8) {
    double sacc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sacc[u] = 0;
    for (int q0 = threadIdx.x; q0 < nq; q0 += U * kBlockThreads) {
      T yv[U], xv[U][8];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int q = min(q0 + e * kBlockThreads, nq - 1);
        const bool own = q < nown;
        const T yo = yg[obase + min(q, nown - 1)];
        const T ys = sg[(size_t)b * nl + max(q - nown, 0)];
        const int64_t gi = own ? obase + q : rbase + (q - nown);
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[e][u] = vg[(int64_t)min(k0 + u, nvec - 1) * n + gi];
        yv[e] = own ? yo : ys;
      }
#pragma unroll
      for (int e = 0; e < U; ++e) {
        if (q0 + e * kBlockThreads < nq) {
#pragma unroll
          for (int u = 0; u < 8; ++u) sacc[u] += (double)xv[e][u] * (double)yv[e];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double t = wave_sum(sacc[u]);
      if (lane == 0 && k0 + u < nvec) red[wv][k0 + u] = t;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nvec; k += kBlockThreads)
    part[(size_t)b * ldp + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  __syncthreads();   // (red is reused by the next block)
}

}  // namespace sem
