// Matrix-core (MFMA) version of the quadrature-free stiffness apply.
//
// Per element the operator is y = sum_a (M D_a)^T (sum_b G_ab (D_b u)), i.e.
// two dense contractions around a pointwise 2x2 mixing (paper Secs. 3.1.2,
// 3.2).  A wave handles a tile of 16 elements:
//   stage 1:  T (2NpP x 16) = [Dr; Ds] (2NpP x NpP) . U (NpP x 16)
//   mixing:   F_r = G_rr T_r + G_rs T_s,  F_s = G_rs T_r + G_ss T_s (registers)
//   stage 2:  Y (NpP x 16)  = [(M Dr)^T | (M Ds)^T] (NpP x 2NpP) . [F_r; F_s]
// with 16x16x4 MFMA tiles.  The accumulator layout of stage 1 (lane l holds
// column l%16, rows 4v+l/16 for FP64 and 4(l/16)+v for FP32, v = 0..3) is
// read directly as the B operand of stage 2 by ordering stage 2's K index as
// (block, M-tile, v, l/16): no data movement between the two contractions.
// U is gathered from the LDS-staged input region, G streams from HBM in the
// matching tile order, Y goes to LDS for the deterministic per-node sums
// shared with the reference kernel.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "mfma.hpp"

namespace sem {

template <typename T, typename GS>
__device__ inline T load_g(const TankDev& d, int64_t i);
template <>
__device__ inline double load_g<double, double>(const TankDev& d, int64_t i) { return d.G[i]; }
template <>
__device__ inline float load_g<float, float>(const TankDev& d, int64_t i) { return d.G32[i]; }
struct BF16m {};
template <>
__device__ inline float load_g<float, BF16m>(const TankDev& d, int64_t i) {
  return __uint_as_float(((uint32_t)d.G16[i]) << 16);
}

template <typename T>
__device__ inline const T* opmat(const TankDev& d, int which);
template <>
__device__ inline const double* opmat<double>(const TankDev& d, int w) {
  return w == 0 ? d.Dr : w == 1 ? d.Ds : w == 2 ? d.MDr : d.MDs;
}
template <>
__device__ inline const float* opmat<float>(const TankDev& d, int w) {
  return w == 0 ? d.Dr32 : w == 1 ? d.Ds32 : w == 2 ? d.MDr32 : d.MDs32;
}

template <int P, typename T, typename GS>
__global__ void __launch_bounds__(kBlockThreads)
k_stiff_mfma(const TankDev* __restrict__ td, const T* __restrict__ u, T* __restrict__ y, T* __restrict__ side,
             int flags) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const TankDev& d = *td;
  if ((flags & F_GATE) && d.ks->done) return;
  constexpr int Np = (P + 1) * (P + 2) / 2;
  constexpr int NpP = (Np + 15) / 16 * 16;
  constexpr int MT = NpP / 16;      // M-tiles per operator block
  constexpr int KS = NpP / 4;       // K-steps of stage 1
  extern __shared__ unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int b = blockIdx.x;
  const int c0 = b * d.cb;
  const int cbb = min(d.cb, d.nx - c0);
  const int nc = d.nc, nl = d.nl, nz2 = 2 * d.nz;
  const int nreg = cbb * nc + nl;
  const int EBb = cbb * nz2;
  T* ureg = lds;                          // [cb*nc + nl]
  T* st3 = ureg + (d.cb * nc + nl);       // [T*16][NpP]
#pragma unroll 4
  for (int q = threadIdx.x; q < nreg; q += blockDim.x) {
    int lc = q / nc, ql = q - lc * nc;
    int64_t gi;
    if (lc < cbb) gi = (int64_t)(c0 + lc) * nc + ql;
    else gi = (ql < nl) ? ((c0 + cbb < d.nx) ? (int64_t)(c0 + cbb) * nc : (d.periodic ? 0 : (int64_t)d.nx * nc)) + ql : -1;
    ureg[q] = gi >= 0 ? u[gi] : T(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int ntile = (EBb + 15) >> 4;
  const T* Dr = opmat<T>(d, 0);
  const T* Ds = opmat<T>(d, 1);
  const T* MDr = opmat<T>(d, 2);
  const T* MDs = opmat<T>(d, 3);
  for (int t = wave; t < ntile; t += kBlockThreads / 64) {
    const int eb = t * 16 + col;
    const bool valid = eb < EBb;
    const int lc = valid ? eb / nz2 : 0;
    const int jt = valid ? eb - lc * nz2 : 0;
    const int32_t* loc = d.elem_loc + jt * NpP;
    // stage 1
    V4 acc[2 * MT];
#pragma unroll
    for (int i = 0; i < 2 * MT; ++i) acc[i] = V4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 4 * s + grp;
      T bval = (valid && k < Np) ? ureg[lc * nc + loc[k]] : T(0);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int row = 16 * mt + col;
        acc[mt] = MF::op(Dr[row * NpP + k], bval, acc[mt]);
        acc[MT + mt] = MF::op(Ds[row * NpP + k], bval, acc[MT + mt]);
      }
    }
    // pointwise mixing with the geometric factors (tile layout: contiguous per (comp, mt, v))
    const int64_t gbase = (((int64_t)b * d.T + t) * 3) * (int64_t)NpP * 16;
    T fr[MT][4], fs[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // FP64 copy: natural rows, node 16mt+4v+g at row 16mt+4v+g -> contiguous in lane
        // FP32 copies: perm rows, node 16mt+4g+v at row 16mt+4v+g -> contiguous in lane
        const int64_t o = (int64_t)(mt * 16 + v * 4) * 16 + lane;
        T grr = load_g<T, GS>(d, gbase + o);
        T grs = load_g<T, GS>(d, gbase + (int64_t)NpP * 16 + o);
        T gss = load_g<T, GS>(d, gbase + 2 * (int64_t)NpP * 16 + o);
        T tr = acc[mt][v], ts = acc[MT + mt][v];
        fr[mt][v] = grr * tr + grs * ts;
        fs[mt][v] = grs * tr + gss * ts;
      }
    // stage 2: K index (blk, mt, v, grp) -> operator row 16 mt + row(v, grp)
    V4 out[MT];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) out[mo] = V4{0, 0, 0, 0};
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int krow = 16 * mt + MF::row(v, grp);
#pragma unroll
        for (int mo = 0; mo < MT; ++mo) {
          const int icol = 16 * mo + col;
          out[mo] = MF::op(MDr[krow * NpP + icol], fr[mt][v], out[mo]);
          out[mo] = MF::op(MDs[krow * NpP + icol], fs[mt][v], out[mo]);
        }
      }
    if (valid) {
#pragma unroll
      for (int mo = 0; mo < MT; ++mo)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * mo + MF::row(v, grp);
          st3[eb * NpP + i] = out[mo][v];
        }
    }
  }
  __syncthreads();
  // node sums in a fixed order (same table as the reference kernel)
  const T sgn = (flags & F_NEG) ? T(-1) : T(1);
  const int nown = cbb * nc;
  for (int q = threadIdx.x; q < nown + nl; q += blockDim.x) {
    int lc = q / nc, ql = q - lc * nc;
    T a = 0;
    if (lc < cbb) {
      // the node's contributions: count and up to kMaxContrib table entries,
      // loaded together (two 16-byte loads)
      const int cnt = d.acc_cnt[ql];
      const int4* e4 = reinterpret_cast<const int4*>(d.acc_ent + (size_t)ql * kMaxContrib);
      const int4 ea = e4[0], eb = e4[1];
      const int ent[kMaxContrib] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
#pragma unroll
      for (int k = 0; k < kMaxContrib; ++k) {
        if (k >= cnt) break;
        const int e = ent[k];
        const int prev = (e >> 30) & 1;
        const int off = e & 0x3fffffff;
        if (prev) {
          if (lc == 0) continue;  // previous column belongs to the left block
          a += st3[(lc - 1) * nz2 * NpP + off];
        } else {
          a += st3[lc * nz2 * NpP + off];
        }
      }
      a *= sgn;
      if ((flags & F_MASK_SURF) && d.is_surf_loc[ql]) a = T(0);
      y[(int64_t)(c0 + lc) * nc + ql] = a;
    } else {
      if (ql >= nl) continue;
      const int cnt = d.acc_cnt[ql];
      const int4* e4 = reinterpret_cast<const int4*>(d.acc_ent + (size_t)ql * kMaxContrib);
      const int4 ea = e4[0], eb = e4[1];
      const int ent[kMaxContrib] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
#pragma unroll
      for (int k = 0; k < kMaxContrib; ++k) {
        if (k >= cnt) break;
        const int e = ent[k];
        if (((e >> 30) & 1) == 0) continue;
        a += st3[(cbb - 1) * nz2 * NpP + (e & 0x3fffffff)];
      }
      a *= sgn;
      if ((flags & F_MASK_SURF) && d.is_surf_loc[ql]) a = T(0);
      side[(size_t)b * nl + ql] = a;
    }
  }
}

// Lane-layout self-test of the two MFMA builtins: D = A B with known A, B;
// each lane writes its four accumulator values to out[lane*4 + v].
__global__ void k_mfma_probe(double* out64, float* out32) {
  const int lane = threadIdx.x;
  const int i = lane & 15, k = lane >> 4;
  // A[i][k] = 1 + i + 16 k ; B[k][j] = 1 + 2 k + 3 j  (j = lane & 15 for B)
  double a = 1.0 + i + 16.0 * k;
  double bb = 1.0 + 2.0 * k + 3.0 * (lane & 15);
  d4 c = {0, 0, 0, 0};
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, c, 0, 0, 0);
  f4 cf = {0, 0, 0, 0};
  cf = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)bb, cf, 0, 0, 0);
  for (int v = 0; v < 4; ++v) {
    out64[lane * 4 + v] = c[v];
    out32[lane * 4 + v] = cf[v];
  }
}

size_t stiff_mfma_lds_bytes(const TankDev& h, size_t word) {
  return word * ((size_t)h.cb * h.nc + h.nl + (size_t)h.T * 16 * h.NpP);
}

#define SEM_MP_CASE(V, ...) \
  case V: {                 \
    constexpr int PP = V;   \
    __VA_ARGS__;            \
  } break;
#define SEM_MP_SWITCH(P, ...)                                                                              \
  switch (P) {                                                                                             \
    SEM_MP_CASE(1, __VA_ARGS__) SEM_MP_CASE(2, __VA_ARGS__) SEM_MP_CASE(3, __VA_ARGS__)                    \
    SEM_MP_CASE(4, __VA_ARGS__) SEM_MP_CASE(5, __VA_ARGS__) SEM_MP_CASE(6, __VA_ARGS__)                    \
    SEM_MP_CASE(7, __VA_ARGS__) SEM_MP_CASE(8, __VA_ARGS__) default : break;                               \
  }

void launch_stiff_mfma(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, int flags,
                       hipStream_t st) {
  size_t lds = stiff_mfma_lds_bytes(h, sizeof(double));
  SEM_MP_SWITCH(h.P, hipLaunchKernelGGL((k_stiff_mfma<PP, double, double>), dim3(h.nb), dim3(kBlockThreads), lds, st,
                                        d, u, y, side, flags));
}
void launch_stiff_mfma(const TankDev& h, const TankDev* d, const float* u, float* y, float* side, int flags,
                       int gstore, hipStream_t st) {
  size_t lds = stiff_mfma_lds_bytes(h, sizeof(float));
  if (gstore == 2) {
    SEM_MP_SWITCH(h.P, hipLaunchKernelGGL((k_stiff_mfma<PP, float, BF16m>), dim3(h.nb), dim3(kBlockThreads), lds, st,
                                          d, u, y, side, flags));
  } else {
    SEM_MP_SWITCH(h.P, hipLaunchKernelGGL((k_stiff_mfma<PP, float, float>), dim3(h.nb), dim3(kBlockThreads), lds, st,
                                          d, u, y, side, flags));
  }
}

// Same launches with start/stop events taken from the dispatch itself (no
// marker packets around the kernel): used to time the kernel inside solves.
void launch_stiff_mfma_timed(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, int flags,
                             hipEvent_t e0, hipEvent_t e1, hipStream_t st) {
  size_t lds = stiff_mfma_lds_bytes(h, sizeof(double));
  SEM_MP_SWITCH(h.P, hipExtLaunchKernelGGL((k_stiff_mfma<PP, double, double>), dim3(h.nb), dim3(kBlockThreads), lds,
                                           st, e0, e1, 0, d, u, y, side, flags));
}
void launch_stiff_mfma_timed(const TankDev& h, const TankDev* d, const float* u, float* y, float* side, int flags,
                             int gstore, hipEvent_t e0, hipEvent_t e1, hipStream_t st) {
  size_t lds = stiff_mfma_lds_bytes(h, sizeof(float));
  if (gstore == 2) {
    SEM_MP_SWITCH(h.P, hipExtLaunchKernelGGL((k_stiff_mfma<PP, float, BF16m>), dim3(h.nb), dim3(kBlockThreads), lds,
                                             st, e0, e1, 0, d, u, y, side, flags));
  } else {
    SEM_MP_SWITCH(h.P, hipExtLaunchKernelGGL((k_stiff_mfma<PP, float, float>), dim3(h.nb), dim3(kBlockThreads), lds,
                                             st, e0, e1, 0, d, u, y, side, flags));
  }
}

void launch_mfma_probe(double* out64, float* out32, hipStream_t st) {
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, st, out64, out32);
}

}  // namespace sem
