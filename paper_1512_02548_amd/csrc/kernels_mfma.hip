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

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <set>
#include <utility>
#include <type_traits>

#include "launch.hpp"
#include "mfma.hpp"
#include "reduce.hpp"

namespace sem {

template <typename T, typename GS>
struct GLoad;
template <>
struct GLoad<double, double> {
  __device__ static double at(const void* G, int64_t i) { return gview((const double*)G)[i]; }
};
template <>
struct GLoad<float, float> {
  __device__ static float at(const void* G, int64_t i) { return gview((const float*)G)[i]; }
};
struct BF16m {};
template <>
struct GLoad<float, BF16m> {
  __device__ static float at(const void* G, int64_t i) {
    return __uint_as_float(((uint32_t)gview((const uint16_t*)G)[i]) << 16);
  }
};

// Everything the stiffness kernel reads, passed by value (the kernel-argument
// segment) so that no argument costs a dependent load.
template <typename T>
struct StiffArgs {
  const void* G;                  // factor copy in tile layout (T, or bfloat16 bits)
  const T* opf;                   // operators in MFMA fragment order: stage 1 then stage 2
  const int32_t* elem_loc;        // [2nz][NpP]
  const uint16_t* acc_pk;         // [nc][kMaxContrib] packed node-sum entries
  const uint16_t* acc_cm;         // [nc] count | surface << 4
  const KrylovState* ks;          // cycle state (launches gated on done)
  const double* lay;              // [2nz][8] element constants (S_z: sigma derivatives and J)
  const double* invd;             // 1/d at the element nodes, tile layout (S_z)
  int32_t nx, nz, nc, nl, cb, tiles, periodic, pad;
  int32_t kb, pad2;               // blocks per workgroup (single-tank launches)
};

template <typename T>
__host__ __device__ inline StiffArgs<T> stiff_args(const TankDev& h, const void* G, const T* opf, int ops_in_lds) {
  StiffArgs<T> a;
  a.G = G;
  a.opf = opf;
  a.elem_loc = h.elem_loc;
  a.acc_pk = h.acc_pk;
  a.acc_cm = h.acc_cm;
  a.ks = h.ks;
  a.lay = h.lay;
  a.invd = h.invd;
  a.nx = h.nx;
  a.nz = h.nz;
  a.nc = h.nc;
  a.nl = h.nl;
  a.cb = h.cb;
  a.tiles = h.T;
  a.periodic = h.periodic;
  a.pad = ops_in_lds;
  a.kb = 1;
  a.pad2 = 0;
  return a;
}

// LDS: [operators 4 NpP^2 (if they fit)] [elem_loc 2nz NpP ints] [u region cb nc + nl]
// [element outputs T 16 (NpP + 1): rows padded against bank conflicts]
// [packed node-sum table: nc x kMaxContrib 16-bit entries, nc 16-bit counts]
template <typename T>
__host__ __device__ inline size_t stiff_lds_layout(const TankDev& h, int ops_in_lds, size_t* o_loc, size_t* o_u,
                                                   size_t* o_st, size_t* o_tab) {
  size_t off = ops_in_lds ? 4 * (size_t)h.NpP * h.NpP * sizeof(T) : 0;
  *o_loc = off;
  off += (size_t)2 * h.nz * h.NpP * sizeof(int32_t);
  off = (off + 15) / 16 * 16;
  *o_u = off;
  off += ((size_t)h.cb * h.nc + h.nl) * sizeof(T);
  off = (off + 15) / 16 * 16;
  *o_st = off;
  off += (size_t)h.T * 16 * (h.NpP + 1) * sizeof(T);
  off = (off + 15) / 16 * 16;
  *o_tab = off;
  off += (size_t)h.nc * (kMaxContrib + 1) * sizeof(uint16_t);
  return off;
}

// Registers per thread holding the next block's input region in the
// several-blocks-per-workgroup kernel: cover cb nc + nl <= 32 P (P + 1) + 64
// values (blocks of at most four 16-element tiles, a layer or more).
__host__ __device__ constexpr int stiff_u_regs(int P) { return (32 * P * (P + 1) + 64 + kBlockThreads - 1) / kBlockThreads; }

// Whether a tank's blocks fit that kernel: at most one tile per wavefront
// and its input region in stiff_u_regs registers per thread.
__host__ __device__ inline bool stiff_mb_fits(const TankDev& h) {
  return h.T <= kBlockThreads / 64 && (int64_t)h.cb * h.nc + h.nl <= (int64_t)stiff_u_regs(h.P) * kBlockThreads;
}

// Node sums of block b (columns c0 .. c0 + cbb - 1) in a fixed order, the
// same contributions in the same order as the reference kernel's table; the
// right line's sum over the block's last column goes to the side buffer.
// tab(ql, e, cm) yields column-local node ql's packed entries (eight 16-bit
// offsets into the element outputs, in four words) and its count word; each
// thread walks its nodes q = tid, tid + kBlockThreads, ... with the column
// and column-local index advanced incrementally (no division per node).
static_assert(kMaxContrib == 8, "a node's packed entries are one 16-byte word");
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int NpP, typename T, typename Tab>
__device__ __forceinline__ void node_sums_packed(const T* st3, T* __restrict__ y, T* __restrict__ side, int flags,
                                                 int nc, int nl, int nz2, int b, int c0, int cbb, Tab tab) {
  constexpr int NS = NpP + 1;
  const int colstride = nz2 * NS;
  const int nq = cbb * nc + nl;
  const T sgn = (flags & F_NEG) ? T(-1) : T(1);
  const bool mask_surf = flags & F_MASK_SURF;
  const int dq = kBlockThreads / nc, dr = kBlockThreads - dq * nc;
  int lq = threadIdx.x / nc, ql = threadIdx.x - lq * nc;
  for (int q = threadIdx.x; q < nq; q += kBlockThreads) {
    uint32_t e[kMaxContrib / 2];
    int cm;
    tab(ql, e, cm);
    const int cnt = cm & 15;
    const bool masked = mask_surf && ((cm >> 4) & 1);
    T acc = 0;
    if (lq < cbb) {
      const T* own = st3 + lq * colstride;
#pragma unroll
      for (int k = 0; k < kMaxContrib; ++k) {
        if (k >= cnt) break;
        const int en = (e[k >> 1] >> (16 * (k & 1))) & 0xffff;
        if (en >> 15) {
          if (lq == 0) continue;  // previous column belongs to the left block
          acc += own[(en & 0x7fff) - colstride];
        } else {
          acc += own[en];
        }
      }
      y[(int64_t)(c0 + lq) * nc + ql] = masked ? T(0) : acc * sgn;
    } else {
      // right line: contributions of the block's last column
      const T* last = st3 + (cbb - 1) * colstride;
#pragma unroll
      for (int k = 0; k < kMaxContrib; ++k) {
        if (k >= cnt) break;
        const int en = (e[k >> 1] >> (16 * (k & 1))) & 0xffff;
        if ((en >> 15) == 0) continue;
        acc += last[en & 0x7fff];
      }
      side[(size_t)b * nl + ql] = masked ? T(0) : acc * sgn;
    }
    ql += dr;
    lq += dq;
    if (ql >= nc) {
      ql -= nc;
      ++lq;
    }
  }
}

// A workgroup's staging into LDS, every global load requested before any
// store (one round trip, not one per table): the four operators (OPS_LDS),
// the element table, the packed node-sum table and, KU > 0, the input
// region of columns c0 .. c0 + cbb - 1 (their own nodes and the first line
// of the next column: the wall line at a wall, line 0 of a periodic tank)
// from clamped addresses; the first
// kStageRegs entries per thread of each table and KU of the region come
// through registers, any rest (deeper tanks) in a loop after them.
constexpr int kStageRegs = 2;
template <int NpP, int KU, bool OPS_LDS, typename T>
__device__ __forceinline__ void stage_block(const StiffArgs<T>& a, const T* __restrict__ u, T* lop, int32_t* lloc,
                                            u32x4* tent4, uint16_t* tcm, T* ureg, int c0, int cbb) {
  const int tid = threadIdx.x;
  constexpr int kVec = 16 / sizeof(T);
  typedef double dv2 __attribute__((ext_vector_type(2)));
  using V = typename std::conditional<sizeof(T) == 8, dv2, f4>::type;
  static_assert((4 * NpP * NpP / kVec) % kBlockThreads == 0, "whole operator fragments per thread");
  constexpr int KO = OPS_LDS ? 4 * NpP * NpP / kVec / kBlockThreads : 0;
  V ov[KO > 0 ? KO : 1];
  if constexpr (OPS_LDS) {
    const SEM_GLOBAL V* src = (const SEM_GLOBAL V*)gview(a.opf);
#pragma unroll
    for (int k = 0; k < KO; ++k) ov[k] = src[tid + k * kBlockThreads];
  }
  const int nloc = 2 * a.nz * NpP, nc = a.nc;
  int32_t lv[kStageRegs];
  u32x4 tv[kStageRegs];
  uint16_t cv[kStageRegs];
#pragma unroll
  for (int k = 0; k < kStageRegs; ++k) {
    lv[k] = gview(a.elem_loc)[min(tid + k * kBlockThreads, nloc - 1)];
    const int q = min(tid + k * kBlockThreads, nc - 1);
    tv[k] = ((const SEM_GLOBAL u32x4*)gview(a.acc_pk))[q];
    cv[k] = gview(a.acc_cm)[q];
  }
  const int nreg = KU > 0 ? cbb * nc + a.nl : 0;
  const int64_t rbase = (c0 + cbb < a.nx) ? (int64_t)(c0 + cbb) * nc : (a.periodic ? 0 : (int64_t)a.nx * nc);
  auto region_at = [&](int q) -> int64_t {
    const int lc = q / nc, ql = q - lc * nc;
    return (lc < cbb) ? (int64_t)(c0 + lc) * nc + ql : rbase + ql;
  };
  T rv[KU > 0 ? KU : 1];
  if constexpr (KU > 0) {
#pragma unroll
    for (int k = 0; k < KU; ++k) rv[k] = gview(u)[region_at(min(tid + k * kBlockThreads, nreg - 1))];
  }
  // the stores
  if constexpr (OPS_LDS) {
    V* dst = reinterpret_cast<V*>(lop);
#pragma unroll
    for (int k = 0; k < KO; ++k) dst[tid + k * kBlockThreads] = ov[k];
  }
#pragma unroll
  for (int k = 0; k < kStageRegs; ++k) {
    const int i = tid + k * kBlockThreads;
    if (i < nloc) lloc[i] = lv[k];
    if (i < nc) {
      tent4[i] = tv[k];
      tcm[i] = cv[k];
    }
  }
  if constexpr (KU > 0) {
#pragma unroll
    for (int k = 0; k < KU; ++k)
      if (tid + k * kBlockThreads < nreg) ureg[tid + k * kBlockThreads] = rv[k];
  }
  // the rest
  for (int i = tid + kStageRegs * kBlockThreads; i < nloc; i += kBlockThreads) lloc[i] = gview(a.elem_loc)[i];
  for (int q = tid + kStageRegs * kBlockThreads; q < nc; q += kBlockThreads) {
    tent4[q] = ((const SEM_GLOBAL u32x4*)gview(a.acc_pk))[q];
    tcm[q] = gview(a.acc_cm)[q];
  }
  if constexpr (KU > 0)
    for (int q = tid + KU * kBlockThreads; q < nreg; q += kBlockThreads) ureg[q] = gview(u)[region_at(q)];
}

// a node's packed entries from the LDS copy of the table
struct LdsTab {
  const u32x4* tent4;
  const uint16_t* tcm;
  __device__ void operator()(int ql, uint32_t (&e)[kMaxContrib / 2], int& cm) const {
    const u32x4 v = tent4[ql];
    e[0] = v.x;
    e[1] = v.y;
    e[2] = v.z;
    e[3] = v.w;
    cm = tcm[ql];
  }
};

// Workgroup b of the tank's grid (columns b cb .. b cb + cb - 1).
// SZ: the operator of the w~ recovery instead (paper Sec. 3.1.3),
// y = J M diag(1/d) (r_sigma Dr + s_sigma Ds) u per element: the same stage 1,
// the mixing F = (r_sigma T_r + s_sigma T_s) / d at the nodes, stage 2 with M
// alone, and J per element (FP64 only).
template <int P, typename T, typename GS, bool OPS_LDS, bool SZ = false>
__device__ __forceinline__ void stiff_body(const StiffArgs<T>& a, const T* __restrict__ u, T* __restrict__ y,
                                           T* __restrict__ side, int flags, uint32_t o_loc, uint32_t o_u,
                                           uint32_t o_st, uint32_t o_tab, int b) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  constexpr int Np = (P + 1) * (P + 2) / 2;
  constexpr int NpP = (Np + 15) / 16 * 16;
  constexpr int MT = NpP / 16;      // M-tiles per operator block
  constexpr int KS = NpP / 4;       // K-steps of stage 1
  extern __shared__ unsigned char lds_raw[];
  T* lop = reinterpret_cast<T*>(lds_raw);                        // [4][NpP][NpP]
  int32_t* lloc = reinterpret_cast<int32_t*>(lds_raw + o_loc);   // [2nz][NpP]
  T* ureg = reinterpret_cast<T*>(lds_raw + o_u);                 // [cb nc + nl]
  T* st3 = reinterpret_cast<T*>(lds_raw + o_st);                 // [T 16][NpP]
  u32x4* tent4 = reinterpret_cast<u32x4*>(lds_raw + o_tab);      // [nc]: kMaxContrib packed entries
  uint16_t* tcm = reinterpret_cast<uint16_t*>(tent4 + a.nc);      // [nc]: count | surface << 4
  const int c0 = b * a.cb;
  const int cbb = min(a.cb, a.nx - c0);
  const int nc = a.nc, nl = a.nl, nz2 = 2 * a.nz;
  const int EBb = cbb * nz2;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int col = lane & 15, grp = lane >> 4;
  const int ntile = (EBb + 15) >> 4;
  // geometric factors of this wave's first tile, requested before anything
  // else (tile layout: one (component, M-tile, v) group is 64 consecutive values)
  T g[SZ ? 1 : 3][MT][4];
  auto load_g = [&](int t) {
    if constexpr (SZ) {
      // 1/d of node 16 mt + 4 v + grp of element col (its tile-layout row is permuted)
      const int64_t ibase = ((int64_t)b * a.tiles + t) * (int64_t)NpP * 16;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          g[0][mt][v] = gview(a.invd)[ibase + (16 * mt + 4 * grp + v) * 16 + col];
    } else {
      const int64_t gbase = (((int64_t)b * a.tiles + t) * 3) * (int64_t)NpP * 16;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            // (a group whose four rows are all past the element's nodes is
            // padding and not read: FP64 groups hold rows 16 mt + 4 v + 0..3,
            // FP32 groups rows 16 mt + v + 0, 4, 8, 12)
            g[c][mt][v] = mt * 16 + (sizeof(T) == sizeof(double) ? 4 * v : v) < Np
                              ? GLoad<T, GS>::at(a.G, gbase + (int64_t)c * NpP * 16 + (mt * 16 + v * 4) * 16 + lane)
                              : T(0);
    }
  };
  // prefetching holds the factors live across stage 1; FP64 with three
  // M-tiles (P = 8) would run out of registers, it loads them after stage 1
  constexpr bool kPrefetch = MT <= 2 || sizeof(T) == sizeof(float);
  if (kPrefetch && wave < ntile) load_g(wave);
  // stage operators, element tables and the input region in LDS
  stage_block<NpP, stiff_u_regs(P), OPS_LDS>(a, u, lop, lloc, tent4, tcm, ureg, c0, cbb);
  __syncthreads();
  // operator fragments: LDS copies, or global memory when they do not fit
  auto opv = [&](int i) -> T {
    if constexpr (OPS_LDS) return lop[i];
    else return gview(a.opf)[i];
  };
  constexpr int kS2 = 2 * NpP * NpP;   // start of the stage-2 fragments
  constexpr int NS = NpP + 1;          // padded row stride of the element outputs
  for (int t = wave; t < ntile; t += kBlockThreads / 64) {
    const int eb = t * 16 + col;
    const bool valid = eb < EBb;
    const int lc = valid ? eb / nz2 : 0;
    const int jt = valid ? eb - lc * nz2 : 0;
    const int32_t* loc = lloc + jt * NpP;
    // stage 1: [Dr; Ds] U
    V4 acc[2 * MT];
#pragma unroll
    for (int i = 0; i < 2 * MT; ++i) acc[i] = V4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 4 * s + grp;
      // (read from a clamped index, then selected: no branch around the read)
      const T bv = ureg[lc * nc + loc[min(k, Np - 1)]];
      const T bval = (valid && k < Np) ? bv : T(0);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int f = ((mt * KS + s) * 2) * 64 + lane;
        acc[mt] = MF::op(opv(f), bval, acc[mt]);
        acc[MT + mt] = MF::op(opv(f + 64), bval, acc[MT + mt]);
      }
    }
    if (!kPrefetch) load_g(t);
    // pointwise mixing with the geometric factors
    T fr[MT][4], fs[MT][4];
    T jel = T(1);
    if constexpr (SZ) {
      const SEM_GLOBAL double* lay = gview(a.lay) + jt * 8;
      const T rsig = T(lay[1]), ssig = T(lay[3]);
      jel = T(lay[4]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T dsig = rsig * acc[mt][v] + ssig * acc[MT + mt][v];
          fr[mt][v] = dsig * g[0][mt][v];
          fs[mt][v] = T(0);
        }
    } else {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T tr = acc[mt][v], ts = acc[MT + mt][v];
          fr[mt][v] = g[0][mt][v] * tr + g[1][mt][v] * ts;
          fs[mt][v] = g[1][mt][v] * tr + g[2][mt][v] * ts;
        }
    }
    // the next tile's factors stream in during stage 2
    if (kPrefetch && t + kBlockThreads / 64 < ntile) load_g(t + kBlockThreads / 64);
    // stage 2: K index (blk, mt, v, grp) -> operator row 16 mt + row(v, grp)
    V4 out[MT];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) out[mo] = V4{0, 0, 0, 0};
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int mo = 0; mo < MT; ++mo) {
          const int f = kS2 + (((mt * 4 + v) * MT + mo) * 2) * 64 + lane;
          out[mo] = MF::op(opv(f), fr[mt][v], out[mo]);
          if constexpr (!SZ) out[mo] = MF::op(opv(f + 64), fs[mt][v], out[mo]);
        }
      }
    if (valid) {
#pragma unroll
      for (int mo = 0; mo < MT; ++mo)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          st3[eb * NS + 16 * mo + MF::row(v, grp)] = SZ ? T(out[mo][v] * jel) : out[mo][v];
    }
  }
  __syncthreads();
  node_sums_packed<NpP, T>(st3, y, side, flags, nc, nl, nz2, b, c0, cbb, LdsTab{tent4, tcm});
}

// Workgroup blocks b0 .. b0 + nblk - 1 of the tank's grid, one after the
// other, for blocks of at most one tile per wavefront (the stiffness grids
// never exceed four tiles per block).  The operators, the element table and
// the packed node-sum table go to LDS once; each block
// then runs its tiles and sums its nodes exactly as stiff_body's workgroup of
// its own would (the same values, bit for bit).  Every global load of a block
// is issued one block ahead, unconditionally, from clamped addresses: its
// input region (into registers, stored to LDS at the block's start) before
// the first contraction, a wavefront's geometric factors after it; the node
// sums read LDS only.
template <int P, typename T, typename GS, bool OPS_LDS, bool SZ = false>
__device__ __forceinline__ void stiff_body_mb(const StiffArgs<T>& a, const T* __restrict__ u, T* __restrict__ y,
                                              T* __restrict__ side, int flags, uint32_t o_loc, uint32_t o_u,
                                              uint32_t o_st, uint32_t o_tab, int b0, int nblk) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  constexpr int Np = (P + 1) * (P + 2) / 2;
  constexpr int NpP = (Np + 15) / 16 * 16;
  constexpr int MT = NpP / 16;      // M-tiles per operator block
  constexpr int KS = NpP / 4;       // K-steps of stage 1
  constexpr int NS = NpP + 1;       // padded row stride of the element outputs
  constexpr int kU = stiff_u_regs(P);
  extern __shared__ unsigned char lds_raw[];
  T* lop = reinterpret_cast<T*>(lds_raw);                        // [4][NpP][NpP]
  int32_t* lloc = reinterpret_cast<int32_t*>(lds_raw + o_loc);   // [2nz][NpP]
  T* ureg = reinterpret_cast<T*>(lds_raw + o_u);                 // [cb nc + nl]
  T* st3 = reinterpret_cast<T*>(lds_raw + o_st);                 // [T 16][NpP + 1]
  u32x4* tent4 = reinterpret_cast<u32x4*>(lds_raw + o_tab);      // [nc]: kMaxContrib packed entries
  uint16_t* tcm = reinterpret_cast<uint16_t*>(tent4 + a.nc);      // [nc]: count | surface << 4
  const int nc = a.nc, nl = a.nl, nz2 = 2 * a.nz;
  const int nbt = (a.nx + a.cb - 1) / a.cb;
  const int b1 = min(b0 + nblk, nbt);
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int col = lane & 15, grp = lane >> 4;
  auto cols_of = [&](int b) { return min(a.cb, a.nx - b * a.cb); };
  auto tiles_of = [&](int b) { return (cols_of(b) * nz2 + 15) >> 4; };
  // operators, element table and node-sum table: requested first, stored once
  stage_block<NpP, 0, OPS_LDS>(a, u, lop, lloc, tent4, tcm, static_cast<T*>(nullptr), 0, 0);
  // input region of block b into registers (kU per thread cover any block;
  // the host checks cb nc + nl <= kU * kBlockThreads)
  T ur[kU];
  auto fetch_u = [&](int b) {
    const int c0 = b * a.cb, cbb = cols_of(b);
    const int nreg = cbb * nc + nl;
    const int64_t rbase = (c0 + cbb < a.nx) ? (int64_t)(c0 + cbb) * nc : (a.periodic ? 0 : (int64_t)a.nx * nc);
#pragma unroll
    for (int j = 0; j < kU; ++j) {
      const int q = min((int)threadIdx.x + j * kBlockThreads, nreg - 1);
      const int lc = q / nc, ql = q - lc * nc;
      ur[j] = gview(u)[(lc < cbb) ? (int64_t)(c0 + lc) * nc + ql : rbase + ql];
    }
  };
  // geometric factors of tile t of block b (tile layout: one (component,
  // M-tile, v) group is 64 consecutive values)
  T g[SZ ? 1 : 3][MT][4];
  auto load_g = [&](int b, int t) {
    if constexpr (SZ) {
      // 1/d of node 16 mt + 4 v + grp of element col (its tile-layout row is permuted)
      const int64_t ibase = ((int64_t)b * a.tiles + t) * (int64_t)NpP * 16;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          g[0][mt][v] = gview(a.invd)[ibase + (16 * mt + 4 * grp + v) * 16 + col];
    } else {
      const int64_t gbase = (((int64_t)b * a.tiles + t) * 3) * (int64_t)NpP * 16;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            // (a group whose four rows are all past the element's nodes is
            // padding and not read: FP64 groups hold rows 16 mt + 4 v + 0..3,
            // FP32 groups rows 16 mt + v + 0, 4, 8, 12)
            g[c][mt][v] = mt * 16 + (sizeof(T) == sizeof(double) ? 4 * v : v) < Np
                              ? GLoad<T, GS>::at(a.G, gbase + (int64_t)c * NpP * 16 + (mt * 16 + v * 4) * 16 + lane)
                              : T(0);
    }
  };
  // a wavefront's tile of block b, clamped to the block's last one (the
  // factors of a wavefront without a tile there are loaded but never used)
  auto tile_of = [&](int b) { return min(wave, tiles_of(b) - 1); };
  // prefetching holds the factors live across the first contraction; FP64
  // with three M-tiles (P = 8) would run out of registers, it loads them
  // after that contraction
  constexpr bool kPrefetch = MT <= 2 || sizeof(T) == sizeof(float);
  fetch_u(b0);
  if constexpr (kPrefetch) load_g(b0, tile_of(b0));
  auto opv = [&](int i) -> T {
    if constexpr (OPS_LDS) return lop[i];
    else return gview(a.opf)[i];
  };
  constexpr int kS2 = 2 * NpP * NpP;   // start of the stage-2 fragments
  for (int b = b0; b < b1; ++b) {
    const int c0 = b * a.cb;
    const int cbb = cols_of(b);
    const int EBb = cbb * nz2;
    const int ntile = (EBb + 15) >> 4;
    const int nreg = cbb * nc + nl;
    const int bn = min(b + 1, b1 - 1);
    // the block's input region into LDS (every wavefront is past the previous
    // block's node sums, which read only the tables and the element outputs)
#pragma unroll
    for (int j = 0; j < kU; ++j)
      if ((int)threadIdx.x + j * kBlockThreads < nreg) ureg[threadIdx.x + j * kBlockThreads] = ur[j];
    lds_barrier();
    if (b + 1 < b1) fetch_u(bn);   // in flight during this block's contractions and sums (uniform)
    const int eb = wave * 16 + col;
    const bool valid = eb < EBb;
    const int lc = valid ? eb / nz2 : 0;
    const int jt = valid ? eb - lc * nz2 : 0;
    T fr[MT][4], fs[MT][4];
    T jel = T(1);
    if (wave < ntile) {
      const int32_t* loc = lloc + jt * NpP;
      // stage 1: [Dr; Ds] U
      V4 acc[2 * MT];
#pragma unroll
      for (int i = 0; i < 2 * MT; ++i) acc[i] = V4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = 4 * s + grp;
        // (read from a clamped index, then selected: no branch around the read)
        const T bv = ureg[lc * nc + loc[min(k, Np - 1)]];
        const T bval = (valid && k < Np) ? bv : T(0);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int f = ((mt * KS + s) * 2) * 64 + lane;
          acc[mt] = MF::op(opv(f), bval, acc[mt]);
          acc[MT + mt] = MF::op(opv(f + 64), bval, acc[MT + mt]);
        }
      }
      if constexpr (!kPrefetch) load_g(b, wave);
      // pointwise mixing with the geometric factors
      if constexpr (SZ) {
        const SEM_GLOBAL double* lay = gview(a.lay) + jt * 8;
        const T rsig = T(lay[1]), ssig = T(lay[3]);
        jel = T(lay[4]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T dsig = rsig * acc[mt][v] + ssig * acc[MT + mt][v];
            fr[mt][v] = dsig * g[0][mt][v];
            fs[mt][v] = T(0);
          }
      } else {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T tr = acc[mt][v], ts = acc[MT + mt][v];
            fr[mt][v] = g[0][mt][v] * tr + g[1][mt][v] * ts;
            fs[mt][v] = g[1][mt][v] * tr + g[2][mt][v] * ts;
          }
      }
    }
    // this wavefront's factors of the next block stream in during the second
    // contraction and the node sums
    if constexpr (kPrefetch)
      if (b + 1 < b1) load_g(bn, tile_of(bn));   // (uniform)
    if (wave < ntile) {
      // stage 2: K index (blk, mt, v, grp) -> operator row 16 mt + row(v, grp)
      V4 out[MT];
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) out[mo] = V4{0, 0, 0, 0};
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
          for (int mo = 0; mo < MT; ++mo) {
            const int f = kS2 + (((mt * 4 + v) * MT + mo) * 2) * 64 + lane;
            out[mo] = MF::op(opv(f), fr[mt][v], out[mo]);
            if constexpr (!SZ) out[mo] = MF::op(opv(f + 64), fs[mt][v], out[mo]);
          }
        }
      if (valid) {
#pragma unroll
        for (int mo = 0; mo < MT; ++mo)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            st3[eb * NS + 16 * mo + MF::row(v, grp)] = SZ ? T(out[mo][v] * jel) : out[mo][v];
      }
    }
    lds_barrier();
    // node sums in a fixed order (the reference kernel's table), from LDS
    node_sums_packed<NpP, T>(st3, y, side, flags, nc, nl, nz2, b, c0, cbb, LdsTab{tent4, tcm});
    // (the next block's input may be stored while these sums run: they read
    // only the tables and the element outputs, which the next tiles overwrite
    // after the barrier that follows that store)
  }
}

// Block b's part of the products of its output with the Krylov vectors
template <typename T>
__device__ inline void stiff_block_dots(const StiffArgs<T>& a, const T* __restrict__ y, const T* __restrict__ side,
                                        const T* __restrict__ V, int64_t n, int nvec, double* __restrict__ part,
                                        int ldp, int b) {
  block_dots_part<T>(a.cb, a.nx, a.nc, a.nl, a.periodic, y, side, V, n, nvec, part, ldp, b);
}

// DOTS: the variant with the fused inner products (dt), a kernel of its own
// (the plain apply keeps its registers, and a profile tells the two apart)
template <int P, typename T, typename GS, bool OPS_LDS, bool MB, bool DOTS>
__global__ void __launch_bounds__(kBlockThreads)
k_stiff_mfma(const StiffArgs<T> a, const T* __restrict__ u, T* __restrict__ y, T* __restrict__ side, int flags,
             uint32_t o_loc, uint32_t o_u, uint32_t o_st, uint32_t o_tab, StiffDots dt) {
  if ((flags & F_GATE) && gview(a.ks)->done) return;
  const int b0 = MB ? (int)blockIdx.x * a.kb : (int)blockIdx.x;
  if constexpr (MB) stiff_body_mb<P, T, GS, OPS_LDS>(a, u, y, side, flags, o_loc, o_u, o_st, o_tab, b0, a.kb);
  else stiff_body<P, T, GS, OPS_LDS>(a, u, y, side, flags, o_loc, o_u, o_st, o_tab, b0);
  if constexpr (!DOTS) return;
  // the inner products with the Krylov vectors: the blocks' parts, then their
  // sum in the last workgroup
  const int nbt = (a.nx + a.cb - 1) / a.cb;
  __syncthreads();
  for (int b = b0; b < min(b0 + (MB ? a.kb : 1), nbt); ++b)
    stiff_block_dots<T>(a, y, side, reinterpret_cast<const T*>(dt.V), dt.n, dt.nvec, dt.part, dt.ldp, b);
  if (!last_block(dt.counter, gridDim.x)) return;
  dots_reduce(dt.nvec, dt.part, dt.ldp, dt.out, nbt);
  if (threadIdx.x == 0) *dt.counter = 0;
}

template <typename T, typename GS>
__device__ inline const void* stiff_factors(const TankDev& d) {
  if constexpr (sizeof(T) == sizeof(double)) return d.G;
  else if constexpr (sizeof(GS) == sizeof(float)) return d.G32;
  else return d.G16;
}
template <typename T>
__device__ inline const T* stiff_ops(const TankDev& d) {
  if constexpr (sizeof(T) == sizeof(double)) return d.opf;
  else return d.opf32;
}

// batched: the tank's arguments and LDS offsets come from its descriptor;
// MB: each work item runs `by` consecutive blocks of its tank
template <int P, typename T, typename GS, bool OPS_LDS, bool MB>
__global__ void __launch_bounds__(kBlockThreads) k_stiff_mfma_b(BatchArgs ba, VSel u, VSel y, int flags) {
  SEM_BATCH_TANK(ba)
  if ((flags & F_GATE) && d.ks->done) return;
  const StiffArgs<T> a = stiff_args<T>(d, stiff_factors<T, GS>(d), stiff_ops<T>(d), OPS_LDS ? 1 : 0);
  size_t ol, ou, os, ot;
  stiff_lds_layout<T>(d, OPS_LDS ? 1 : 0, &ol, &ou, &os, &ot);
  if constexpr (MB)
    stiff_body_mb<P, T, GS, OPS_LDS>(a, bvec<T>(d, u), bvec<T>(d, y), reinterpret_cast<T*>(d.side), flags,
                                     (uint32_t)ol, (uint32_t)ou, (uint32_t)os, (uint32_t)ot, it_.bx, it_.by);
  else
    stiff_body<P, T, GS, OPS_LDS>(a, bvec<T>(d, u), bvec<T>(d, y), reinterpret_cast<T*>(d.side), flags, (uint32_t)ol,
                                  (uint32_t)ou, (uint32_t)os, (uint32_t)ot, it_.bx);
}

// S_z of the w~ recovery on the matrix cores (FP64), single tank and batched
template <int P, bool OPS_LDS>
__global__ void __launch_bounds__(kBlockThreads)
k_sz_mfma(const StiffArgs<double> a, const double* __restrict__ u, double* __restrict__ y,
          double* __restrict__ side, uint32_t o_loc, uint32_t o_u, uint32_t o_st, uint32_t o_tab) {
  stiff_body<P, double, double, OPS_LDS, true>(a, u, y, side, 0, o_loc, o_u, o_st, o_tab, blockIdx.x);
}
template <int P, bool OPS_LDS>
__global__ void __launch_bounds__(kBlockThreads) k_sz_mfma_b(BatchArgs ba, SSel u) {
  SEM_BATCH_TANK(ba)
  const StiffArgs<double> a = stiff_args<double>(d, d.G, d.opf_sz, OPS_LDS ? 1 : 0);
  size_t ol, ou, os, ot;
  stiff_lds_layout<double>(d, OPS_LDS ? 1 : 0, &ol, &ou, &os, &ot);
  // the stiffness plan's items, which may span several blocks
  const int nbt = (d.nx + d.cb - 1) / d.cb;
  const int b1 = min(it_.bx + (it_.by > 1 ? it_.by : 1), nbt);
  for (int b = it_.bx; b < b1; ++b) {
    if (b > it_.bx) __syncthreads();
    stiff_body<P, double, double, OPS_LDS, true>(a, svec(ba, d, it_.tank, u), d.b, d.side, 0, (uint32_t)ol,
                                                 (uint32_t)ou, (uint32_t)os, (uint32_t)ot, b);
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

// operators go to LDS unless they would take more than 80 KiB (a workgroup
// may hold up to 160 KiB).  The 72 KiB seventh- and eighth-order FP64
// operators leave room for one workgroup per CU, which is also all their
// registers allow (one wavefront per SIMD); reading the fragments from LDS
// instead of through the caches measured 1.7x faster on the 256-tank batch.
template <typename T>
__host__ __device__ inline int stiff_ops_in_lds(const TankDev& h) {
  return 4 * (size_t)h.NpP * h.NpP * sizeof(T) <= 80 * 1024 ? 1 : 0;
}

// Kernels whose dynamic LDS exceeds the default 64 KiB get the chip's full
// 160 KiB cap.  The cap is runtime state shared by every thread that launches
// the kernel, so it is raised once per (kernel, device), under a lock, before
// that device's first such launch; concurrent workers (batch mode with several
// streams) never set it while another thread launches the same kernel.
static std::mutex g_lds_mu;
static std::set<std::pair<const void*, int>> g_lds_done;

// The limit on a kernel's dynamic LDS is raised once per kernel and device
// to what its static LDS leaves of the 160 KiB (the fused inner products give
// the stiffness kernels some), for every kernel that takes dynamic LDS.
template <typename K>
static void allow_lds(K kern, size_t bytes) {
  if (bytes == 0) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(g_lds_mu);
  if (g_lds_done.insert({(const void*)kern, dev}).second) {
    hipFuncAttributes fa{};
    size_t stat = 0;
    if (hipFuncGetAttributes(&fa, (const void*)kern) == hipSuccess) stat = fa.sharedSizeBytes;
    const int lim = (int)(160 * 1024 - std::min<size_t>(stat, 160 * 1024));
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
      (void)hipGetLastError();   // (the launch itself reports a size beyond the limit)
  }
}

// Blocks per workgroup of a stiffness launch over `blocks` blocks: enough to
// keep about 3 072 workgroups (twelve per CU), or 1 024 when a workgroup's
// LDS (`lds` bytes) leaves room for one per CU, so that the operators' copy
// into LDS is shared and each block's loads are issued during the previous
// block.  (Measured on the 256-tank batch against 2 048 workgroups: fourth
// and sixth order 5% faster, eighth-order FP64 3% faster.)  The results do
// not depend on it; SEM_STIFF_BLOCKS (environment) sets it explicitly.  The
// FP64 variant that reads its operators from global memory has no registers
// to spare for it and keeps one block per workgroup, and so do tanks whose
// blocks do not fit that kernel (stiff_mb_fits).
int stiff_blocks_per_workgroup(int64_t blocks, bool register_bound, bool fits, size_t lds) {
  if (register_bound || !fits) return 1;
  if (const char* e = std::getenv("SEM_STIFF_BLOCKS")) {
    const int k = std::atoi(e);
    if (k >= 1) return (int)std::min<int64_t>(k, std::max<int64_t>(1, blocks));
  }
  const int64_t target = lds > 80 * 1024 ? 1024 : 3072;
  return (int)std::max<int64_t>(1, blocks / target);
}

size_t stiff_mfma_lds_bytes(const TankDev& h, size_t word) {
  size_t a, b, c, e;
  return word == sizeof(double) ? stiff_lds_layout<double>(h, stiff_ops_in_lds<double>(h), &a, &b, &c, &e)
                                : stiff_lds_layout<float>(h, stiff_ops_in_lds<float>(h), &a, &b, &c, &e);
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

// gstore: 0 = FP64 factors (T = double), 1 = FP32, 2 = bfloat16
template <typename T, typename GS>
static void stiff_launch(const TankDev& h, const TankDev* d, const T* u, T* y, T* side, int flags, hipEvent_t e0,
                         hipEvent_t e1, hipStream_t st, const StiffDots& dots = StiffDots{}) {
  const int inl = stiff_ops_in_lds<T>(h);
  size_t ol, ou, os, ot;
  const int kb = stiff_blocks_per_workgroup(h.nb, sizeof(T) == sizeof(double) && !inl, stiff_mb_fits(h),
                                            stiff_lds_layout<T>(h, inl, &ol, &ou, &os, &ot));
  const size_t lds = stiff_lds_layout<T>(h, inl, &ol, &ou, &os, &ot);
  const void* G;
  const T* opf;
  if constexpr (sizeof(T) == sizeof(double)) {
    G = h.G;
    opf = h.opf;
  } else {
    G = sizeof(GS) == sizeof(float) ? (const void*)h.G32 : (const void*)h.G16;
    opf = h.opf32;
  }
  StiffArgs<T> a = stiff_args<T>(h, G, opf, inl);
  a.kb = kb;
  const int nwg = (h.nb + a.kb - 1) / a.kb;
#define SEM_SL3(INL, MB, DT)                                                                                     \
  SEM_MP_SWITCH(h.P, allow_lds(k_stiff_mfma<PP, T, GS, INL, MB, DT>, lds));                                     \
  if (e0) {                                                                                                     \
    SEM_MP_SWITCH(h.P, hipExtLaunchKernelGGL((k_stiff_mfma<PP, T, GS, INL, MB, DT>), dim3(nwg),                   \
                                             dim3(kBlockThreads), (uint32_t)lds, st, e0, e1, 0, a, u, y, side,    \
                                             flags, (uint32_t)ol, (uint32_t)ou, (uint32_t)os, (uint32_t)ot,       \
                                             dots));                                                              \
  } else {                                                                                                      \
    SEM_MP_SWITCH(h.P, hipLaunchKernelGGL((k_stiff_mfma<PP, T, GS, INL, MB, DT>), dim3(nwg), dim3(kBlockThreads), \
                                          lds, st, a, u, y, side, flags, (uint32_t)ol, (uint32_t)ou, (uint32_t)os, \
                                          (uint32_t)ot, dots));                                                   \
  }
#define SEM_SL(INL, MB)      \
  if (dots.nvec > 0) {       \
    SEM_SL3(INL, MB, true)   \
  } else {                   \
    SEM_SL3(INL, MB, false)  \
  }
  if (inl) {
    if (a.kb > 1) {
      SEM_SL(true, true)
    } else {
      SEM_SL(true, false)
    }
  } else {
    if (a.kb > 1) {
      SEM_SL(false, true)
    } else {
      SEM_SL(false, false)
    }
  }
#undef SEM_SL
#undef SEM_SL3
}

void launch_stiff_mfma(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, int flags,
                       hipStream_t st) {
  stiff_launch<double, double>(h, d, u, y, side, flags, nullptr, nullptr, st);
}
void launch_stiff_mfma(const TankDev& h, const TankDev* d, const float* u, float* y, float* side, int flags,
                       int gstore, hipStream_t st) {
  if (gstore == 2) stiff_launch<float, BF16m>(h, d, u, y, side, flags, nullptr, nullptr, st);
  else stiff_launch<float, float>(h, d, u, y, side, flags, nullptr, nullptr, st);
}

// Same launches with start/stop events taken from the dispatch itself (no
// marker packets around the kernel): used to time the kernel inside solves.
void launch_stiff_mfma_timed(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, int flags,
                             hipEvent_t e0, hipEvent_t e1, hipStream_t st, const StiffDots& dots) {
  stiff_launch<double, double>(h, d, u, y, side, flags, e0, e1, st, dots);
}
void launch_stiff_mfma_timed(const TankDev& h, const TankDev* d, const float* u, float* y, float* side, int flags,
                             int gstore, hipEvent_t e0, hipEvent_t e1, hipStream_t st, const StiffDots& dots) {
  if (gstore == 2) stiff_launch<float, BF16m>(h, d, u, y, side, flags, e0, e1, st, dots);
  else stiff_launch<float, float>(h, d, u, y, side, flags, e0, e1, st, dots);
}

void launch_sz_mfma(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, hipStream_t st) {
  const int inl = stiff_ops_in_lds<double>(h);
  size_t ol, ou, os, ot;
  const size_t lds = stiff_lds_layout<double>(h, inl, &ol, &ou, &os, &ot);
  const StiffArgs<double> a = stiff_args<double>(h, h.G, h.opf_sz, inl);
  if (inl) {
    SEM_MP_SWITCH(h.P, allow_lds(k_sz_mfma<PP, true>, lds));
    SEM_MP_SWITCH(h.P, hipLaunchKernelGGL((k_sz_mfma<PP, true>), dim3(h.nb), dim3(kBlockThreads), lds, st, a, u, y,
                                          side, (uint32_t)ol, (uint32_t)ou, (uint32_t)os, (uint32_t)ot));
  } else {
    SEM_MP_SWITCH(h.P, allow_lds(k_sz_mfma<PP, false>, lds));
    SEM_MP_SWITCH(h.P, hipLaunchKernelGGL((k_sz_mfma<PP, false>), dim3(h.nb), dim3(kBlockThreads), lds, st, a, u, y,
                                          side, (uint32_t)ol, (uint32_t)ou, (uint32_t)os, (uint32_t)ot));
  }
}

void launch_sz_mfma_b(const BatchArgs& a0, const BatchStage& p, int P, SSel u, hipStream_t st) {
  if (p.items.empty()) return;
  BatchArgs a = a0;
  a.items = p.dev;
  TankDev probe{};
  probe.NpP = ((P + 1) * (P + 2) / 2 + 15) / 16 * 16;
  const dim3 grid((unsigned)p.items.size());
  if (stiff_ops_in_lds<double>(probe)) {
    SEM_MP_SWITCH(P, allow_lds(k_sz_mfma_b<PP, true>, p.lds));
    SEM_MP_SWITCH(P, hipLaunchKernelGGL((k_sz_mfma_b<PP, true>), grid, dim3(kBlockThreads), p.lds, st, a, u));
  } else {
    SEM_MP_SWITCH(P, allow_lds(k_sz_mfma_b<PP, false>, p.lds));
    SEM_MP_SWITCH(P, hipLaunchKernelGGL((k_sz_mfma_b<PP, false>), grid, dim3(kBlockThreads), p.lds, st, a, u));
  }
}

void plan_stiff(const std::vector<TankDev>& tanks, const std::vector<int>& ids, int P, int f32, BatchStage* out) {
  *out = BatchStage{};
  int64_t blocks = 0;
  for (int t : ids)
    if (tanks[t].P == P) blocks += tanks[t].nb;
  TankDev probe{};
  probe.NpP = ((P + 1) * (P + 2) / 2 + 15) / 16 * 16;
  bool fits = true;
  size_t lds_mb = 0;
  for (int t : ids) {
    const TankDev& h = tanks[t];
    if (h.P != P) continue;
    fits = fits && stiff_mb_fits(h);
    size_t a, b, c, e;
    lds_mb = std::max(lds_mb, f32 ? stiff_lds_layout<float>(h, stiff_ops_in_lds<float>(h), &a, &b, &c, &e)
                                  : stiff_lds_layout<double>(h, stiff_ops_in_lds<double>(h), &a, &b, &c, &e));
  }
  const int kb = stiff_blocks_per_workgroup(blocks, !f32 && !stiff_ops_in_lds<double>(probe), fits, lds_mb);
  for (int t : ids) {
    const TankDev& h = tanks[t];
    if (h.P != P) continue;
    size_t a, b, c, e;
    const size_t lds = f32 ? stiff_lds_layout<float>(h, stiff_ops_in_lds<float>(h), &a, &b, &c, &e)
                           : stiff_lds_layout<double>(h, stiff_ops_in_lds<double>(h), &a, &b, &c, &e);
    // item {tank, first block, blocks, tank's block count}
    for (int x = 0; x < h.nb; x += kb) out->items.push_back(BatchItem{t, x, kb, h.nb});
    out->lds = std::max(out->lds, lds);
  }
}

template <typename T, typename GS>
static void stiff_b_t(const BatchArgs& a0, const BatchStage& p, int P, VSel u, VSel y, int flags, hipStream_t st) {
  if (p.items.empty()) return;
  BatchArgs a = a0;
  a.items = p.dev;
  // whether the operators fit in LDS depends on P and the word size only
  TankDev probe{};
  probe.NpP = ((P + 1) * (P + 2) / 2 + 15) / 16 * 16;
  const int inl = stiff_ops_in_lds<T>(probe);
  const bool mb = p.items[0].by > 1;     // every item of a plan spans the same block count
  const dim3 grid((unsigned)p.items.size());
#define SEM_SB(INL, MB)                                                                                      \
  SEM_MP_SWITCH(P, allow_lds(k_stiff_mfma_b<PP, T, GS, INL, MB>, p.lds));                                   \
  SEM_MP_SWITCH(P, hipLaunchKernelGGL((k_stiff_mfma_b<PP, T, GS, INL, MB>), grid, dim3(kBlockThreads), p.lds, st, \
                                      a, u, y, flags));
  if (inl) {
    if (mb) {
      SEM_SB(true, true)
    } else {
      SEM_SB(true, false)
    }
  } else {
    if (mb) {
      SEM_SB(false, true)
    } else {
      SEM_SB(false, false)
    }
  }
#undef SEM_SB
}

void launch_stiff_b(const BatchArgs& a, const BatchStage& p, int P, VSel u, VSel y, int flags, int gstore,
                    hipStream_t st) {
  if (gstore == 0) stiff_b_t<double, double>(a, p, P, u, y, flags, st);
  else if (gstore == 1) stiff_b_t<float, float>(a, p, P, u, y, flags, st);
  else stiff_b_t<float, BF16m>(a, p, P, u, y, flags, st);
}

void launch_mfma_probe(double* out64, float* out32, hipStream_t st) {
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, st, out64, out32);
}

}  // namespace sem
