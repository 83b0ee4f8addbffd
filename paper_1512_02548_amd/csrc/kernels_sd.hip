// Exact inverse of a column-coupled operator on a periodic tank, on matrix
// cores.
//
// The operator A (the still-water flat-bed Laplace operator on the free
// nodes, used as the preconditioner, or the 2D mass matrix) couples the
// nodes of one element column to its two vertical lines only.  Condensing
// each column's interior unknowns onto the lines leaves a block-circulant
// system in x, which a DFT along x splits into one q x q complex system per
// Fourier mode.  With R_c the interior right side of column c:
//
//   condense   [Y; T_L; T_R](:, c) = [A_II^-1; A_LI A_II^-1; A_RI A_II^-1] R_c
//   modes      g_c = r_L,c - T_L,c - T_R,c-1,   g^_k = sum_c e^{-2 pi i k c/nx} g_c,
//              x^_k = S^_k^{-1} g^_k
//   back       x_L,c = Re sum_k e^{+2 pi i k c/nx} x^_k / nx,
//              z_I,c = Y_c - A_II^-1 [A_IL | A_IR] [x_L,c; x_L,c+1]
//
// Every step over many columns (or modes) is a dense product, run as 16x16x4
// MFMA tiles with 16 columns (or modes) per N (or M) tile; the per-mode
// solves are small complex matrix-vector products.  Matrices are uploaded in
// MFMA fragment order ([M-tile][K-step][lane]) so each operand load is 64
// consecutive words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <type_traits>
#include <utility>
#include <vector>

#include "launch.hpp"
#include "mfma.hpp"

namespace sem {

namespace {
constexpr int kWaves = kBlockThreads / 64;

__host__ __device__ inline int sd_part_words(int q) { return max(kWaves * 16 * 16 * 2, 32 * q); }

// Reading the input r / hn (the unnormalised next Krylov vector and its norm)
// instead of r: 1/hn, 0 when hn is not positive, 1 without a scale.
__device__ inline double sd_in_scale(const double* nscale) {
  if (!nscale) return 1.0;
  const double hn = *nscale;
  return hn > 0.0 ? 1.0 / hn : 0.0;
}

// (a + b) mod n for a, b in [0, n), as a select rather than a branch
__device__ inline int wrap_add(int a, int b, int n) {
  const int s = a + b;
  return s >= n ? s - n : s;
}

__device__ inline double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
struct SdMat;
template <>
struct SdMat<double> {
  __device__ static const double* A1(const SDData& s) { return s.A1; }
  __device__ static const double* C3(const SDData& s) { return s.C3; }
  __device__ static const double* Shat(const SDData& s) { return s.Shat; }
};
template <>
struct SdMat<float> {
  __device__ static const float* A1(const SDData& s) { return s.A1_32; }
  __device__ static const float* C3(const SDData& s) { return s.C3_32; }
  __device__ static const float* Shat(const SDData& s) { return s.Shat32; }
};
}  // namespace

// Launch shape of the condensation and back-substitution products of a
// tank (nMT M-tiles): ntw N-tiles of 16 columns per workgroup (wider groups
// reuse each factor fragment over more columns) and four M-tiles, one per
// wave; or, for small tanks (split = 1), one M-tile per workgroup with its K
// range split over the four waves (more workgroups, shorter chains).  A
// function of the tank alone.  ch: accumulator chains per tile (below).
struct SdShape {
  int ntw, split, ch;
};
__host__ __device__ inline SdShape sd_shape(int nx, int nMT) {
  const int ct = (nx + 15) / 16, mg = (nMT + 3) / 4;
  if (((ct + 3) / 4) * mg >= 256) return SdShape{4, 0, 1};
  if (((ct + 1) / 2) * mg >= 256) return SdShape{2, 0, 1};
  if (ct * mg >= 256) return SdShape{1, 0, 1};
  return SdShape{1, 1, 1};
}
constexpr int kNTMax = 4;    // N-tiles per wave at most
// In a batched launch workgroups never run short, so every tank's products
// run as wide tiles: four M-tiles (one per wave) and kNTB N-tiles per
// workgroup, which reuse each factor fragment and each staged column over
// more of the product than the split shape does.  An output must not depend
// on the launch, so a tank whose own launch splits K keeps that summation
// order: its wide tiles carry four accumulator chains (chain r takes the
// K-steps = r mod 4, as wave r does in the split shape, and the chains are
// added in order at the end).  narrow: one N-tile (the back-substitution of
// tanks that form their line values by the inverse transform in the
// workgroup, whose layout covers 16 columns).
constexpr int kNTB = 4;      // N-tiles of a wide tile, one chain
// N-tiles of a wide tile with four chains: two in FP32, one in FP64 (two
// would halve the FP64 kernels' occupancy)
__host__ __device__ constexpr int ntb4(size_t word) { return word == 4 ? 2 : 1; }
__host__ __device__ inline SdShape sd_shape_b(int nx, int nMT, bool narrow, size_t word) {
  const SdShape s = sd_shape(nx, nMT);
  return SdShape{narrow ? 1 : (s.split ? ntb4(word) : kNTB), 0, s.split ? 4 : 1};
}
// Small direct-transform tanks (nx <= 64, lines of at most 32 unknowns): the
// back-substitution workgroups form the line values they need by the inverse
// transform themselves (17 lines x 32 unknowns, one 16 x 16 tile per wave),
// instead of a separate inverse-transform launch.
__host__ __device__ inline bool sd_back_dft(int nx, int q, int fft_n1, int nMT3) {
  return fft_n1 == 0 && nx <= 64 && q <= 32 && sd_shape(nx, nMT3).ntw == 1;
}
constexpr int kKC = 16;      // K-steps of the right-hand factor staged in LDS at a time (64 rows)
// LDS of the condensation's staging area (and, split, of its wave partials),
// before the interior index table
__host__ __device__ inline size_t sd_cond_stage_bytes(int ntw, size_t word, int split) {
  const size_t st = word * 4 * kKC * (16 * (size_t)ntw + 1);
  const size_t red = split ? sizeof(double) * kWaves * ntw * 256 : 0;
  return ((st > red ? st : red) + 15) / 16 * 16;
}

// condense, as the product [Y; T_L; T_R] = A1 R over the tank's columns:
// workgroup (column group bx, M-tiles 4 by .. 4 by + 3), one M-tile per wave
// and NTW N-tiles of 16 columns, the full K range in order (so an output does
// not depend on the grouping); R is staged in LDS in chunks of kKC K-steps.
// SPLIT (small tanks, NTW = 1): one M-tile per workgroup, wave w takes the
// K-steps w, w + 4, ... and the four partial tiles are added in wave order.
// CH = 4 (batched wide tiles of such tanks): the same sums, chain r of a
// tile taking the K-steps = r mod 4.
template <typename T, int NTW, bool SPLIT, int CH>
__device__ __forceinline__ void sd_cond_impl(const TankDev& d, const SDData& sd, const T* __restrict__ r,
                                             const double* __restrict__ nscale, T* __restrict__ vout, int bx,
                                             int by) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  extern __shared__ unsigned char lds_raw[];
  const int nI = sd.nI, q = sd.q, nx = d.nx, KS = sd.KS1, nMT = sd.nMT1;
  constexpr int ldr = 16 * NTW + 1;                      // odd stride: conflict-free staging
  T* Rs = reinterpret_cast<T*>(lds_raw);                 // [4 kKC][ldr]
  int32_t* lidx = reinterpret_cast<int32_t*>(lds_raw + sd_cond_stage_bytes(NTW, sizeof(T), SPLIT));   // [nI]
  const int c0 = bx * 16 * NTW;
  for (int k = threadIdx.x; k < nI; k += blockDim.x) lidx[k] = sd.I_idx[k];
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const int mt = SPLIT ? by : 4 * by + wv;
  const int s_first = SPLIT ? wv : 0;
  constexpr int s_step = SPLIT ? kWaves : 1;
  constexpr int kSteps = kKC / s_step;                   // K-steps of one wave per chunk
  const double rs = sd_in_scale(nscale);
  const SEM_GLOBAL T* A = gview(SdMat<T>::A1(sd)) + (size_t)min(mt, nMT - 1) * KS * 64;
  const SEM_GLOBAL T* rg = gview(r);
  static_assert(CH == 1 || (CH == 4 && !SPLIT && kKC % 4 == 0), "chains: wide tiles, whole chunks of 4 K-steps");
  V4 acc[CH][NTW];
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int u = 0; u < NTW; ++u) acc[c][u] = V4{0, 0, 0, 0};
  // R chunk s0 (4 kKC = 64 interior rows x 16 NTW columns): lane l of wave w
  // reads row l of columns w, w + 4, ... (consecutive lanes, consecutive
  // interior unknowns of a column).  Fetched into registers one chunk ahead,
  // so that its loads are in flight during the previous chunk's products,
  // and staged into LDS after them.  Every load is issued unconditionally
  // from a clamped address (no branch around it, so that all of them are in
  // flight together); rows and columns outside the tank are staged as zeros,
  // and the scale is applied, when the chunk is staged.
  static_assert(4 * kKC == 64, "one chunk row per lane");
  constexpr int kR = 4 * NTW;
  const int64_t ncl = d.nc;
  T pre[kR];
  auto fetch = [&](int s0) {
    const int64_t li = lidx[min(4 * s0 + lane, nI - 1)];
#pragma unroll
    for (int i = 0; i < kR; ++i) pre[i] = rg[min(c0 + wv + 4 * i, nx - 1) * ncl + li];
  };
  auto stage = [&](int s0) {
    const int k = 4 * s0 + lane;
    const bool kv = k < nI;
    const int64_t li = lidx[min(k, nI - 1)];
#pragma unroll
    for (int i = 0; i < kR; ++i) {
      const int cc = wv + 4 * i;
      const bool ok = kv && c0 + cc < nx;
      const T v = ok ? (nscale ? T((double)pre[i] * rs) : pre[i]) : T(0);
      Rs[lane * ldr + cc] = v;
      if (vout && by == 0 && ok) vout[(c0 + cc) * ncl + li] = v;
    }
  };
  // This wave's factor fragments, requested one chunk ahead: a fragment of
  // chunk s0 + kKC is requested as soon as the products of the same slot of
  // chunk s0 have been issued.  K-steps past the tank's last (kc < kKC) take
  // the chunk's last fragment and multiply staged zero rows: they add exact
  // zeros.  The barriers order LDS only, so that these requests stay in
  // flight across them.
  T ab[kSteps];
  auto load_ab = [&](int p2, int s0) {
    const int kc = min(kKC, KS - s0);
    ab[p2] = A[(size_t)(s0 + min(s_first + p2 * s_step, kc - 1)) * 64 + lane];
  };
  lds_barrier();   // interior index table
  if (KS > 0) {
    fetch(0);
#pragma unroll
    for (int p2 = 0; p2 < kSteps; ++p2) load_ab(p2, 0);
  }
  for (int s0 = 0; s0 < KS; s0 += kKC) {
    const bool more = s0 + kKC < KS;
    lds_barrier();   // every wave is past the previous chunk's products
    stage(s0);
    lds_barrier();
    if (more) fetch(s0 + kKC);   // the next chunk's input, in flight during the products
    if (mt < nMT) {
#pragma unroll
      for (int p2 = 0; p2 < kSteps; ++p2) {
        const T* brow = Rs + (4 * (s_first + p2 * s_step) + grp) * ldr + col;
#pragma unroll
        for (int u = 0; u < NTW; ++u) acc[p2 % CH][u] = MF::op(ab[p2], brow[16 * u], acc[p2 % CH][u]);
        if (more) load_ab(p2, s0 + kKC);
      }
    }
  }
  if constexpr (SPLIT) {
    // partial tiles added in wave order (the staging area is free again)
    double* red = reinterpret_cast<double*>(lds_raw);   // [kWaves][NTW][256]
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(wv * NTW + u) * 256 + MF::row(v, grp) * 16 + col] = (double)acc[0][u][v];
    __syncthreads();
    const int rr = threadIdx.x >> 4, cc = threadIdx.x & 15;
    const int row = 16 * mt + rr;
    for (int u = 0; u < NTW; ++u) {
      const int c = c0 + 16 * u + cc;
      if (c >= nx) continue;
      double val = 0;
      for (int w = 0; w < kWaves; ++w) val += red[(w * NTW + u) * 256 + threadIdx.x];
      if (row < nI) sd.yI[(size_t)c * nI + row] = val;
      else if (row < nI + q) sd.TL[(size_t)c * q + row - nI] = val;
      else if (row < nI + 2 * q) sd.TR[(size_t)c * q + row - nI - q] = val;
    }
    return;
  }
  if (mt >= nMT) return;
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int c = c0 + 16 * u + col;
    if (c >= nx) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * mt + MF::row(v, grp);
      double val = 0;
      if constexpr (CH == 1) {
        val = (double)acc[0][u][v];
      } else {
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) val += (double)acc[ch][u][v];
      }
      if (row < nI) sd.yI[(size_t)c * nI + row] = val;
      else if (row < nI + q) sd.TL[(size_t)c * q + row - nI] = val;
      else if (row < nI + 2 * q) sd.TR[(size_t)c * q + row - nI - q] = val;
    }
  }
}

// B: a batched launch (wide tiles, sd_shape_b)
template <typename T, bool B>
__device__ __forceinline__ void sd_cond_body(const TankDev& d, int which, const T* __restrict__ r,
                                             const double* __restrict__ nscale, T* __restrict__ vout, int bx,
                                             int by) {
  const SDData& sd = d.sd[which];
  if constexpr (B) {
    if (sd_shape_b(d.nx, sd.nMT1, false, sizeof(T)).ch == 4)
      sd_cond_impl<T, ntb4(sizeof(T)), false, 4>(d, sd, r, nscale, vout, bx, by);
    else sd_cond_impl<T, kNTB, false, 1>(d, sd, r, nscale, vout, bx, by);
    return;
  }
  const SdShape sh = sd_shape(d.nx, sd.nMT1);
  if (sh.split) sd_cond_impl<T, 1, true, 1>(d, sd, r, nscale, vout, bx, by);
  else if (sh.ntw == 4) sd_cond_impl<T, 4, false, 1>(d, sd, r, nscale, vout, bx, by);
  else if (sh.ntw == 2) sd_cond_impl<T, 2, false, 1>(d, sd, r, nscale, vout, bx, by);
  else sd_cond_impl<T, 1, false, 1>(d, sd, r, nscale, vout, bx, by);
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sd_cond(const TankDev* __restrict__ td, int which, const T* __restrict__ r, int gate,
          const double* __restrict__ nscale, T* __restrict__ vout) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sd_cond_body<T, false>(d, which, r, nscale, vout, (int)blockIdx.x, (int)blockIdx.y);
}

// modes: one block per 8 or 16 Fourier modes; waves split the sum over
// columns.  U: K-steps of a wave whose loads are requested together.  SQ:
// the mode solves of tanks with at most kSolveQ line unknowns and one (mode,
// row) item per thread, whose row of the inverse symbol is requested at once
// (the other tanks walk it kSolveUnroll entries at a time).
constexpr int kSolveQ = 32;
constexpr int kSolveChunk = 16;
constexpr int kSolveUnroll = 8;
__host__ __device__ inline bool sd_modes_small(int nx, int q) {
  return q <= kSolveQ && modes_per_block(nx) * q <= kBlockThreads;
}
template <typename T, int U, bool SQ>
__device__ __forceinline__ void sd_modes_body(const TankDev& d, int which, const T* __restrict__ r, const double* __restrict__ nscale, T* __restrict__ vout, int bx, int by) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const SDData& sd = d.sd[which];
  extern __shared__ double sh[];
  const int q = sd.q, nx = d.nx, nc = d.nc;
  double* part = sh;                      // [kWaves][16][16][2], later x^ of the block's modes [16][q][2]
  double* gh = sh + sd_part_words(q);     // [16][q][2]
  const int nNT = (q + 15) / 16, KS = (nx + 3) / 4;
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const int kModesPB = modes_per_block(nx), kPairs = kModesPB / 2;
  const double rs = sd_in_scale(nscale);
  // A row of this lane: the mode of slot `col` (rows past the block's slots are discarded)
  const int kmode = col < kModesPB ? paired_mode(bx, col, kPairs, nx) : -1;
  const bool kval = kmode >= 0;
  const int kr = kval ? kmode : 0;
  // twiddle index (kmode * c) mod nx for c = 4 s + grp, s = wv, wv + 4, ...
  const int step = (int)(((int64_t)16 * kr) % nx);
  // small tanks (SQ: one (mode, row) of the solve per thread): the first
  // kSolveChunk entries of the thread's row of the inverse symbol, requested
  // before the transform (they do not depend on it)
  const int tk = (int)threadIdx.x / max(q, 1), ti = (int)threadIdx.x - tk * q;
  const int tmode = SQ && tk < kModesPB ? paired_mode(bx, tk, kPairs, nx) : -1;
  const int tkm = tmode >= 0 ? tmode : 0;
  const SEM_GLOBAL T* tS = gview(SdMat<T>::Shat(sd)) + (size_t)(2 * tkm > nx ? nx - tkm : tkm) * q * q * 2;
  double sv0[SQ ? 2 * kSolveChunk : 1];
  if constexpr (SQ) {
#pragma unroll
    for (int e = 0; e < kSolveChunk; ++e) {
      const int jj = min(e, q - 1);
      sv0[2 * e] = (double)tS[((size_t)jj * q + min(ti, q - 1)) * 2];
      sv0[2 * e + 1] = (double)tS[((size_t)jj * q + min(ti, q - 1)) * 2 + 1];
    }
  }
  for (int nt0 = 0; nt0 < nNT; nt0 += 4) {
    const int ntn = min(4, nNT - nt0);
    V4 are[4], aim[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) are[u] = aim[u] = V4{0, 0, 0, 0};
    int mm = (int)(((int64_t)kr * (4 * wv + grp)) % nx);
    // the loads of U K-steps are issued before their products, from clamped
    // addresses (no branch around a load); entries outside the tank are
    // zeroed afterwards, and K-steps past the last multiply zeros
    const SEM_GLOBAL T* rg = gview(r);
    const SEM_GLOBAL double* tlg = gview(sd.TL);
    const SEM_GLOBAL double* trg = gview(sd.TR);
    const SEM_GLOBAL double* twg = gview(d.twid);
    const int jb = 16 * nt0 + col;
#pragma unroll 1
    for (int s0 = wv; s0 < KS; s0 += U * kWaves) {
      double twr[U], twi[U], rv[U][4], tl[U][4], tr[U][4], rw[U][4];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int cc = min(4 * (s0 + e * kWaves) + grp, nx - 1);
        const int cm = cc == 0 ? nx - 1 : cc - 1;
        twr[e] = twg[2 * mm];
        twi[e] = twg[2 * mm + 1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (u >= ntn) break;   // (uniform)
          const int jj = min(jb + 16 * u, q - 1);
          rv[e][u] = (double)rg[(int64_t)cc * nc + jj];
          tl[e][u] = tlg[(size_t)cc * q + jj];
          tr[e][u] = trg[(size_t)cm * q + jj];
          if (sd.wall) rw[e][u] = (double)rg[(int64_t)nx * nc + jj];   // (uniform: walled tanks fold their wall line onto line 0)
        }
        mm = wrap_add(mm, step, nx);
      }
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int c = 4 * (s0 + e * kWaves) + grp;
        const bool cv = c < nx;
        const T fre = (cv && kval) ? T(twr[e]) : T(0);
        const T fim = (cv && kval) ? T(twi[e]) : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (u >= ntn) break;
          const int j = jb + 16 * u;
          const bool ok = cv && j < q;
          double v = rv[e][u] * rs;
          if (vout && bx == 0 && ok) vout[(int64_t)c * nc + j] = T(v);
          if (sd.wall && c == 0 && ok) {   // wall line folded onto line 0
            const double w = rw[e][u] * rs;
            if (vout && bx == 0) vout[(int64_t)nx * nc + j] = T(w);
            v += w;
          }
          const T gv = ok ? T(v - tl[e][u] - tr[e][u]) : T(0);
          are[u] = MF::op(fre, gv, are[u]);
          aim[u] = MF::op(fim, gv, aim[u]);
        }
      }
    }
    for (int u = 0; u < ntn; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = MF::row(v, grp);
        part[((wv * 16 + row) * 16 + col) * 2] = (double)are[u][v];
        part[((wv * 16 + row) * 16 + col) * 2 + 1] = (double)aim[u][v];
      }
      __syncthreads();
      {
        const int row = threadIdx.x >> 4, jc = threadIdx.x & 15;
        const int j = 16 * (nt0 + u) + jc;
        double sr = 0, si = 0;
        for (int w = 0; w < kWaves; ++w) {
          sr += part[((w * 16 + row) * 16 + jc) * 2];
          si += part[((w * 16 + row) * 16 + jc) * 2 + 1];
        }
        if (j < q) {
          gh[(row * q + j) * 2] = sr;
          gh[(row * q + j) * 2 + 1] = si;
        }
      }
      __syncthreads();
    }
  }
  // x^_k = S^_k^{-1} g^_k (column-major: thread per (mode, row)), the sum
  // over j in order
  auto solve = [&](int kk, int i, int k, auto load_all) {
    const bool cj = 2 * k > nx;   // stored as the conjugate of mode nx - k
    const SEM_GLOBAL T* S = gview(SdMat<T>::Shat(sd)) + (size_t)(cj ? nx - k : k) * q * q * 2;
    const double sgn = cj ? -1.0 : 1.0;
    double xr = 0, xi = 0;
    if constexpr (decltype(load_all)::value) {
      // kSolveChunk entries requested together (clamped addresses; the first
      // chunk's came before the transform)
      for (int j0 = 0; j0 < q; j0 += kSolveChunk) {
        double sv[2 * kSolveChunk];
#pragma unroll
        for (int e = 0; e < kSolveChunk; ++e) {
          const int jj = min(j0 + e, q - 1);
          sv[2 * e] = j0 == 0 ? sv0[2 * e] : (double)S[((size_t)jj * q + i) * 2];
          sv[2 * e + 1] = j0 == 0 ? sv0[2 * e + 1] : (double)S[((size_t)jj * q + i) * 2 + 1];
        }
#pragma unroll
        for (int e = 0; e < kSolveChunk; ++e) {
          const int j = j0 + e;
          if (j < q) {   // (uniform)
            const double sr = sv[2 * e], si = sgn * sv[2 * e + 1];
            const double gr = gh[(kk * q + j) * 2], gi = gh[(kk * q + j) * 2 + 1];
            xr += sr * gr - si * gi;
            xi += sr * gi + si * gr;
          }
        }
      }
    } else {
#pragma unroll kSolveUnroll
      for (int j = 0; j < q; ++j) {
        const double sr = (double)S[((size_t)j * q + i) * 2], si = sgn * (double)S[((size_t)j * q + i) * 2 + 1];
        const double gr = gh[(kk * q + j) * 2], gi = gh[(kk * q + j) * 2 + 1];
        xr += sr * gr - si * gi;
        xi += sr * gi + si * gr;
      }
    }
    sd.XH[((size_t)k * q + i) * 2] = xr;
    sd.XH[((size_t)k * q + i) * 2 + 1] = xi;
  };
  if constexpr (SQ) {
    // (kModesPB q <= kBlockThreads: thread (tk, ti) alone)
    if (tmode >= 0) solve(tk, ti, tmode, std::integral_constant<bool, SQ>{});
  } else {
    for (int t = threadIdx.x; t < kModesPB * q; t += blockDim.x) {
      const int kk = t / q, i = t - kk * q, k = paired_mode(bx, kk, kPairs, nx);
      if (k < 0) continue;
      solve(kk, i, k, std::integral_constant<bool, SQ>{});
    }
  }
}

// K-steps per wave requested together by the direct transform: two, or all
// four of a tank of at most 64 columns launched alone (B: a batched launch,
// whose registers also serve its long tanks).  Only K-steps past the last
// depend on it, and they add zeros.
template <typename T, bool B>
__device__ __forceinline__ void sd_modes_any(const TankDev& d, int which, const T* __restrict__ r,
                                             const double* __restrict__ nscale, T* __restrict__ vout, int bx,
                                             int by) {
  const int q = d.sd[which].q;
  if (sd_modes_small(d.nx, q)) {
    if (!B && d.nx <= 64) sd_modes_body<T, B ? 2 : 4, true>(d, which, r, nscale, vout, bx, by);
    else sd_modes_body<T, 2, true>(d, which, r, nscale, vout, bx, by);
  } else {
    sd_modes_body<T, 2, false>(d, which, r, nscale, vout, bx, by);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sd_modes(const TankDev* __restrict__ td, int which, const T* __restrict__ r, int gate,
           const double* __restrict__ nscale, T* __restrict__ vout) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sd_modes_any<T, false>(d, which, r, nscale, vout, (int)blockIdx.x, (int)blockIdx.y);
}

// inverse transform of the line solution (direct products, small nx): grid
// (16-line tiles, 16-wide tiles of line unknowns); the K range (modes x
// re/im) is split over the wavefronts and the partial tiles added in LDS
template <typename T>
__device__ __forceinline__ void sd_idft_body(const TankDev& d, int which, int bx, int by) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const SDData& sd = d.sd[which];
  __shared__ double red[kWaves][256];
  const int q = sd.q, nx = d.nx;
  const int KS = (2 * nx + 3) / 4;
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const int c0 = bx * 16, nt = by;
  // A[c][kk] = twiddle part (kk & 1) of mode kk / 2 at line c; B[kk][j] = that part of x^_{kk/2}[j]
  const int cr = (c0 + col) % nx;
  const int pr = grp & 1;
  const int j = 16 * nt + col;
  const int step = (int)(((int64_t)2 * kWaves * cr) % nx);   // the mode advances by 8 per pass
  int mm = (int)(((int64_t)cr * (2 * wv + (grp >> 1))) % nx);
  V4 acc = V4{0, 0, 0, 0};
  // operands loaded from clamped addresses and zeroed outside the range (no
  // branch around a load, so that the loads of several K-steps are in flight)
  const SEM_GLOBAL double* twg = gview(d.twid);
  const SEM_GLOBAL double* xhg = gview(sd.XH);
  const int jc = min(j, q - 1);
  // kIU K-steps of a wave per request (the kernel's registers leave room:
  // fewer round trips over the long tanks' modes)
  constexpr int kIU = 8;
  for (int s0 = wv; s0 < KS; s0 += kIU * kWaves) {
    double ta[kIU], tb[kIU];
    bool kv[kIU];
#pragma unroll
    for (int u = 0; u < kIU; ++u) {
      const int s = s0 + u * kWaves;
      const int k = 2 * s + (grp >> 1);
      kv[u] = s < KS && k < nx;
      ta[u] = twg[2 * mm + pr];
      tb[u] = xhg[((size_t)min(k, nx - 1) * q + jc) * 2 + pr];
      mm = wrap_add(mm, step, nx);
    }
#pragma unroll
    for (int u = 0; u < kIU; ++u) acc = MF::op(kv[u] ? T(ta[u]) : T(0), (kv[u] && j < q) ? T(tb[u]) : T(0), acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv][MF::row(v, grp) * 16 + col] = (double)acc[v];
  __syncthreads();
  const int row = threadIdx.x >> 4, jl = threadIdx.x & 15;
  const int c = c0 + row, jj = 16 * nt + jl;
  if (c >= nx || jj >= q) return;
  double v = 0;
  for (int w = 0; w < kWaves; ++w) v += red[w][threadIdx.x];
  sd.XL[(size_t)c * q + jj] = v / nx;
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sd_idft(const TankDev* __restrict__ td, int which, int gate) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sd_idft_body<T>(d, which, (int)blockIdx.x, (int)blockIdx.y);
}

// The product of the back-substitution for M-tile mt and NTW N-tiles of 16
// columns from c0, the line values of the columns in LDS (xl, row stride
// q + 1): z_I = Y - C [x_L,c; x_L,c+1].  SPLIT: wave w takes the K-steps
// w, w + 4, ... and the partial tiles are added in wave order; CH = 4: the
// same sums, chain r of the tile taking the K-steps = r mod 4.
// PRE (split): the first group of factor fragments (pre), and Y and the
// interior index of the thread's output (ypre, ipre) were requested by the
// caller, before the line solutions were formed.
template <typename T, int NTW, bool SPLIT, int CH, bool PRE = false>
__device__ __forceinline__ void sd_back_product(const TankDev& d, const SDData& sd, T* __restrict__ z,
                                                double* xl, int c0, int mt, const T* pre = nullptr,
                                                double ypre = 0, int ipre = 0) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const int nI = sd.nI, q = sd.q, nx = d.nx, nc = d.nc, KS3 = sd.KS3;
  const int qp = q + 1;
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const int s_first = SPLIT ? wv : 0;
  constexpr int s_step = SPLIT ? kWaves : 1;
  const SEM_GLOBAL T* C = gview(SdMat<T>::C3(sd)) + (size_t)mt * KS3 * 64;
  // factor fragments loaded kPre K-steps at a time, one group ahead of their
  // MFMAs; rows k >= 2q of the last K-step multiply zeros (exact zeros added)
  constexpr int kPre = 8;
  static_assert(CH == 1 || (CH == 4 && !SPLIT && kPre % 4 == 0), "chains: wide tiles, groups of 4 K-steps");
  V4 acc[CH][NTW];
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int u = 0; u < NTW; ++u) acc[c][u] = V4{0, 0, 0, 0};
  T ab[kPre], an[kPre];
  auto load = [&](int s, T (&dst)[kPre]) {
#pragma unroll
    for (int p2 = 0; p2 < kPre; ++p2) dst[p2] = C[(size_t)min(s + p2 * s_step, KS3 - 1) * 64 + lane];
  };
  if constexpr (PRE) {
#pragma unroll
    for (int p2 = 0; p2 < kPre; ++p2) ab[p2] = pre[p2];
  } else {
    load(s_first, ab);
  }
  for (int s = s_first; s < KS3; s += kPre * s_step) {
    if (s + kPre * s_step < KS3) load(s + kPre * s_step, an);
#pragma unroll
    for (int p2 = 0; p2 < kPre; ++p2) {
      if (s + p2 * s_step >= KS3) break;   // (wave-uniform)
      const int kk = 4 * (s + p2 * s_step) + grp;
      // B[kk][col] = x_L of column col (kk < q) or of the next column
      const bool kv = kk < 2 * q;
      const int off = kk < q ? kk : qp + kk - q;
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        const double bx = xl[(16 * u + col) * qp + (kv ? off : 0)];
        acc[p2 % CH][u] = MF::op(ab[p2], kv ? T(bx) : T(0), acc[p2 % CH][u]);
      }
    }
#pragma unroll
    for (int p2 = 0; p2 < kPre; ++p2) ab[p2] = an[p2];
  }
  if constexpr (SPLIT) {
    // partial tiles added in wave order
    const int ncol = 16 * NTW;
    double* red = xl + (ncol + 1) * qp;   // [kWaves][NTW][256]
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(wv * NTW + u) * 256 + MF::row(v, grp) * 16 + col] = (double)acc[0][u][v];
    __syncthreads();
    const int rr = threadIdx.x >> 4, cc = threadIdx.x & 15;
    const int row = 16 * mt + rr;
    for (int u = 0; u < NTW; ++u) {
      const int c = c0 + 16 * u + cc;
      if (c >= nx || row >= nI) continue;
      double sacc = 0;
      for (int w = 0; w < kWaves; ++w) sacc += red[(w * NTW + u) * 256 + threadIdx.x];
      if constexpr (PRE && NTW == 1) z[(int64_t)c * nc + ipre] = T(ypre - sacc);
      else z[(int64_t)c * nc + sd.I_idx[row]] = T(sd.yI[(size_t)c * nI + row] - sacc);
    }
    return;
  }
  // the interior indices and Y of the tile's outputs requested together
  // (clamped addresses), then the stores
  int idx[4];
  double yv[NTW][4];
#pragma unroll
  for (int v = 0; v < 4; ++v) idx[v] = gview(sd.I_idx)[min(16 * mt + MF::row(v, grp), nI - 1)];
#pragma unroll
  for (int u = 0; u < NTW; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      yv[u][v] = gview(sd.yI)[(size_t)min(c0 + 16 * u + col, nx - 1) * nI + min(16 * mt + MF::row(v, grp), nI - 1)];
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int c = c0 + 16 * u + col;
    if (c >= nx) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * mt + MF::row(v, grp);
      double sacc = 0;
      if constexpr (CH == 1) {
        sacc = (double)acc[0][u][v];
      } else {
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) sacc += (double)acc[ch][u][v];
      }
      if (row < nI) z[(int64_t)c * nc + idx[v]] = T(yv[u][v] - sacc);
    }
  }
}

// back-substitution z_I = Y - A_II^-1 [A_IL | A_IR] [x_L,c; x_L,c+1] as a
// tiled product: workgroup (column group bx, M-tiles 4 by .. 4 by + 3), one
// M-tile per wave, the full K range (2q) in order; the lines of the group's
// columns and the next one come from XL through LDS.  Workgroups of row 0
// also write the line values (and the wall line).  B: a batched launch
// (wide tiles, sd_shape_b).
template <typename T, bool B>
__device__ __forceinline__ void sd_back_body(const TankDev& d, int which, T* __restrict__ z, T* __restrict__ vout,
                                             int bx, int by) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const SDData& sd = d.sd[which];
  extern __shared__ double sh[];
  const int nI = sd.nI, q = sd.q, nx = d.nx, nc = d.nc, nMT = sd.nMT3, KS3 = sd.KS3;
  const bool dft = sd_back_dft(nx, q, sd.fft_n1, nMT);
  const SdShape shp = B ? sd_shape_b(nx, nMT, dft, sizeof(T)) : sd_shape(nx, nMT);
  const int ntw = shp.ntw;
  const int ncol = 16 * ntw;
  const int qp = q + 1;                      // odd stride: conflict-free reads across columns
  double* xl = sh;                           // [ncol + 1][qp] line solutions of columns c0 .. c0 + ncol
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const int c0 = bx * ncol;
  const int mt = shp.split ? by : 4 * by + wv;
  // a single tank's split product: its first factor fragments, and Y and the
  // interior index of the thread's output, requested before the line
  // solutions are formed (they do not depend on them)
  constexpr int kPreB = 8;
  T abp[kPreB];
  double ysp = 0;
  int isp = 0;
  if (!B && shp.split && mt < nMT) {
    const SEM_GLOBAL T* C = gview(SdMat<T>::C3(sd)) + (size_t)mt * KS3 * 64;
#pragma unroll
    for (int p2 = 0; p2 < kPreB; ++p2) abp[p2] = C[(size_t)min(wv + p2 * kWaves, KS3 - 1) * 64 + lane];
    const int row = min(16 * mt + (int)(threadIdx.x >> 4), nI - 1);
    const int c = min(c0 + (int)(threadIdx.x & 15), nx - 1);
    ysp = gview(sd.yI)[(size_t)c * nI + row];
    isp = gview(sd.I_idx)[row];
  }
  if (dft) {
    // x_L,c = Re sum_k e^{2 pi i k c / nx} x^_k / nx for lines c0 .. c0 + 16:
    // wave (line tile lt, unknown tile jt), the whole K range (modes x re/im)
    // in order, operands loaded kD K-steps at a time
    const int lt = wv >> 1, jt = wv & 1;
    const int cr = (c0 + 16 * lt + col) % nx, pr = grp & 1, jb = 16 * jt + col;
    const int KSd = (2 * nx + 3) / 4;
    V4 acc = V4{0, 0, 0, 0};
    constexpr int kD = 8;
    // twiddle index (cr k) mod nx, k = 2 s + grp / 2: advances by 2 cr per K-step
    const int step = (2 * cr) % nx;
    int mm = (cr * (grp >> 1)) % nx;
    for (int s0 = 0; s0 < KSd; s0 += kD) {
      T av[kD], bv[kD];
#pragma unroll
      for (int u = 0; u < kD; ++u) {
        // (loaded from clamped addresses, zeroed outside the range)
        const int k = 2 * (s0 + u) + (grp >> 1);
        const bool kv = s0 + u < KSd && k < nx;
        const double ta = gview(d.twid)[2 * mm + pr];
        const double tb = gview(sd.XH)[((size_t)min(k, nx - 1) * q + min(jb, q - 1)) * 2 + pr];
        av[u] = kv ? T(ta) : T(0);
        bv[u] = (kv && jb < q) ? T(tb) : T(0);
        mm = wrap_add(mm, step, nx);
      }
      // (the scheduler would otherwise interleave the loads with the
      // products and wait for each: all kD K-steps' loads go first; batched
      // launches, where few tanks take this path, keep their registers)
      if constexpr (!B) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kD; ++u) acc = MF::op(av[u], bv[u], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int cc = 16 * lt + MF::row(v, grp);
      if (cc <= ncol && jb < q) xl[cc * qp + jb] = (double)acc[v] / nx;
    }
  } else {
#pragma unroll 4
    for (int t = threadIdx.x; t < (ncol + 1) * q; t += blockDim.x) {
      const int cc = t / q, j = t - cc * q;
      xl[cc * qp + j] = sd.XL[(size_t)((c0 + cc) % nx) * q + j];
    }
  }
  __syncthreads();
  if (by == 0) {
    for (int t = threadIdx.x; t < ncol * q; t += blockDim.x) {
      const int cc = t / q, j = t - cc * q, c = c0 + cc;
      if (c < nx) z[(int64_t)c * nc + j] = T(xl[cc * qp + j]);
    }
    if (sd.zero_surface) {
      for (int t = threadIdx.x; t < ncol * d.P; t += blockDim.x) {
        const int cc = t / d.P, k = t - cc * d.P, c = c0 + cc;
        if (c < nx) {
          const int64_t gi = (int64_t)c * nc + (k == 0 ? d.nl - 1 : d.surf_loc[k]);
          z[gi] = T(0);
          if (vout) vout[gi] = T(0);   // the normalised Krylov vector vanishes at the surface
        }
      }
    }
    if (sd.wall && bx == 0) {
      // wall line = line 0 + v
      for (int j = threadIdx.x; j < q; j += blockDim.x) z[(int64_t)nx * nc + j] = T(xl[j] + sd.vbuf[j]);
      if (sd.zero_surface && threadIdx.x == 0) {
        z[(int64_t)nx * nc + d.nl - 1] = T(0);
        if (vout) vout[(int64_t)nx * nc + d.nl - 1] = T(0);
      }
    }
  }
  if (mt >= nMT) return;   // (uniform over the workgroup in split mode)
  if constexpr (B) {
    if (shp.ch == 4) {
      if (ntw == 1) sd_back_product<T, 1, false, 4>(d, sd, z, xl, c0, mt);
      else sd_back_product<T, ntb4(sizeof(T)), false, 4>(d, sd, z, xl, c0, mt);
    } else {
      if (ntw == 1) sd_back_product<T, 1, false, 1>(d, sd, z, xl, c0, mt);
      else sd_back_product<T, kNTB, false, 1>(d, sd, z, xl, c0, mt);
    }
    return;
  }
  if (shp.split) sd_back_product<T, 1, true, 1, true>(d, sd, z, xl, c0, mt, abp, ysp, isp);
  else if (ntw == 4) sd_back_product<T, 4, false, 1>(d, sd, z, xl, c0, mt);
  else if (ntw == 2) sd_back_product<T, 2, false, 1>(d, sd, z, xl, c0, mt);
  else sd_back_product<T, 1, false, 1>(d, sd, z, xl, c0, mt);
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sd_back(const TankDev* __restrict__ td, int which, T* __restrict__ z, int gate, T* __restrict__ vout) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sd_back_body<T, false>(d, which, z, vout, (int)blockIdx.x, (int)blockIdx.y);
}

// Sum of a workgroup's values in a fixed order (wave butterflies, then the
// four wave totals in order); the result is valid in every thread.
__device__ inline double block_total(double v) {
  __shared__ double wt[kWaves];
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) wt[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((wt[0] + wt[1]) + wt[2]) + wt[3];
}

// Wall correction, first part (a workgroup per value): lines nx-1 and 0 of
// the periodic solve straight from the modal solution,
// x_c = Re sum_k e^{2 pi i k c / nx} x^_k / nx, into WP = [x_{nx-1}; x_0].
__device__ __forceinline__ void sd_wall_lines_body(const TankDev& d, int which, int bx, int by) {
  const SDData& sd = d.sd[which];
  const int q = sd.q, nx = d.nx;
  const int ln = bx / q, j = bx - ln * q;
  const int c = ln == 0 ? nx - 1 : 0;
  const SEM_GLOBAL double* xh = gview(sd.XH);
  const SEM_GLOBAL double* tw = gview(d.twid);
  // a thread's modes k = tid, tid + 256, ... four at a time: their loads
  // requested together (clamped indices), the sum in order
  constexpr int kU = 4;
  double acc = 0;
  for (int k0 = threadIdx.x; k0 < nx; k0 += kU * kBlockThreads) {
    double hr[kU], hi[kU], tr[kU], ti[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = min(k0 + u * kBlockThreads, nx - 1);
      const int mm = (int)(((int64_t)k * c) % nx);
      hr[u] = xh[((size_t)k * q + j) * 2];
      hi[u] = xh[((size_t)k * q + j) * 2 + 1];
      tr[u] = tw[2 * mm];
      ti[u] = tw[2 * mm + 1];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (k0 + u * kBlockThreads < nx) acc += hr[u] * tr[u] + hi[u] * ti[u];
  }
  acc = block_total(acc);
  if (threadIdx.x == 0) sd.WP[bx] = acc / nx;
}

// Wall correction, second part (a workgroup per component a of v):
// v_a = W_a . [r_wall; x_{nx-1}; x_0; y_I(nx-1)]  (the three sources loaded
// from clamped indices and selected: no branch around a load)
template <typename T>
__device__ __forceinline__ void sd_wall_body(const TankDev& d, const SDData& sd, const T* __restrict__ r,
                                             const double* __restrict__ nscale, int bx, int by) {
  const int nI = sd.nI, q = sd.q, nx = d.nx, nc = d.nc;
  const int np = 3 * q + nI;
  const double rs = sd_in_scale(nscale);
  const SEM_GLOBAL double* row = gview(sd.Wv) + (size_t)bx * np;
  const SEM_GLOBAL T* rg = gview(r);
  const SEM_GLOBAL double* wp = gview(sd.WP);
  const SEM_GLOBAL double* yi = gview(sd.yI);
  double acc = 0;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const double w = row[p];
    const double a = (double)rg[(int64_t)nx * nc + min(p, q - 1)] * rs;
    const double b = wp[min(max(p - q, 0), 2 * q - 1)];
    const double c = yi[(size_t)(nx - 1) * nI + max(p - 3 * q, 0)];
    const double in = p < q ? a : (p < 3 * q ? b : c);
    acc += w * in;
  }
  acc = block_total(acc);
  if (threadIdx.x == 0) sd.vbuf[bx] = acc;
}
template <typename T>
__device__ __forceinline__ void sd_wall_body(const TankDev& d, int which, const T* __restrict__ r,
                                             const double* __restrict__ nscale, int bx, int by) {
  sd_wall_body<T>(d, d.sd[which], r, nscale, bx, by);
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sd_wall(const TankDev* __restrict__ td, int which, const T* __restrict__ r, int gate,
          const double* __restrict__ nscale) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sd_wall_body<T>(d, which, r, nscale, (int)blockIdx.x, (int)blockIdx.y);
}

__global__ void __launch_bounds__(kBlockThreads) k_sd_wall_lines(const TankDev* __restrict__ td, int which, int gate) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sd_wall_lines_body(d, which, (int)blockIdx.x, (int)blockIdx.y);
}

// x^_k -= H_k v for every mode (thread per mode and line unknown); the
// last column's interior solve y_I -= Q v (threads past nx q)
__device__ __forceinline__ void sd_wall_modes_body(const TankDev& d, int which, int bx, int by) {
  const SDData& sd = d.sd[which];
  const int q = sd.q, nI = sd.nI;
  const int64_t nm = (int64_t)d.nx * q;
  const int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  if (t < nm) {
    const int64_t k = t / q;
    const int i = (int)(t - k * q);
    const bool cj = 2 * k > d.nx;   // stored as the conjugate of mode nx - k
    const double* Hk = sd.Hm + (size_t)(cj ? d.nx - k : k) * q * q * 2;
    const double sgn = cj ? -1.0 : 1.0;
    double xr = 0, xi = 0;
#pragma unroll 4
    for (int a = 0; a < q; ++a) {
      const double va = sd.vbuf[a];
      xr += Hk[((size_t)a * q + i) * 2] * va;
      xi += sgn * Hk[((size_t)a * q + i) * 2 + 1] * va;
    }
    sd.XH[((size_t)k * q + i) * 2] -= xr;
    sd.XH[((size_t)k * q + i) * 2 + 1] -= xi;
  } else if (t < nm + nI) {
    const int i = (int)(t - nm);
    double acc = 0;
#pragma unroll 4
    for (int a = 0; a < q; ++a) acc += sd.Qm[(size_t)a * nI + i] * sd.vbuf[a];
    sd.yI[(size_t)(d.nx - 1) * nI + i] -= acc;
  }
}

__global__ void __launch_bounds__(kBlockThreads)
k_sd_wall_modes(const TankDev* __restrict__ td, int which, int gate) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sd_wall_modes_body(d, which, (int)blockIdx.x, (int)blockIdx.y);
}

// ------------------------------------------------------------ four-step transforms
// nx = n1 n2, column c = n2 c1 + c2, mode k = k1 + n1 k2, w_N = e^{-2 pi i/N}:
//   g^_k = sum_c2 w_n2^{k2 c2} [ w_nx^{k1 c2} sum_c1 w_n1^{k1 c1} g_{n2 c1 + c2} ]
//   x_c  = Re sum_k1 conj(w_n1)^{k1 c1} [ conj(w_nx)^{k1 c2} sum_k2 conj(w_n2)^{k2 c2} x^_k ] / nx
// Each bracket is a batch of small products on MFMA (16x16x4, real operands,
// complex values as pairs); twiddles come from the nx-point table.

__device__ inline int sd_mod(int64_t a, int n) { return (int)(a % n); }

// pass A (block per c2): FT[k1][c2][j] = w_nx^{k1 c2} sum_c1 w_n1^{k1 c1} g[n2 c1 + c2][j]
template <typename T>
__device__ __forceinline__ void sdf_a_body(const TankDev& d, int which, const T* __restrict__ r, const double* __restrict__ nscale, T* __restrict__ vout, int bx, int by) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const SDData& sd = d.sd[which];
  extern __shared__ double sh[];
  const int q = sd.q, nx = d.nx, nc = d.nc, n1 = sd.fft_n1, n2 = sd.fft_n2;
  const int c2 = bx;
  const int KS = (n1 + 3) / 4, nMT = (n1 + 15) / 16;
  const double rs = sd_in_scale(nscale);
  const int nt = by;   // this workgroup's 16 line unknowns
  double* gl = sh;   // [4 KS][16] line right sides of columns n2 c1 + c2, unknowns 16 nt ..
  for (int t = threadIdx.x; t < 4 * KS * 16; t += blockDim.x) {
    const int c1 = t >> 4, j = 16 * nt + (t & 15);
    double v = 0;
    if (c1 < n1 && j < q) {
      const int c = n2 * c1 + c2, cm = c == 0 ? nx - 1 : c - 1;
      v = (double)r[(int64_t)c * nc + j] * rs;
      if (vout) vout[(int64_t)c * nc + j] = T(v);
      if (sd.wall && c == 0) {
        const double rw = (double)r[(int64_t)nx * nc + j] * rs;
        if (vout) vout[(int64_t)nx * nc + j] = T(rw);
        v += rw;
      }
      v -= sd.TL[(size_t)c * q + j] + sd.TR[(size_t)cm * q + j];
    }
    gl[t] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const SEM_GLOBAL double* twg = gview(d.twid);
  for (int mt = wv; mt < nMT; mt += kWaves) {
    const int k1 = 16 * mt + col, j = 16 * nt + col;
    V4 ar = V4{0, 0, 0, 0}, ai = V4{0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < KS; ++s) {
      const int c1 = 4 * s + grp;
      // (twiddle loaded from a clamped index, then selected: no branch around the load)
      const bool okw = k1 < n1 && c1 < n1;
      const int m = okw ? sd_mod((int64_t)k1 * c1, n1) * n2 : 0;
      const double twr = twg[2 * m], twi = twg[2 * m + 1];
      const T wr = okw ? T(twr) : T(0), wi = okw ? T(twi) : T(0);
      const T b = T(gl[c1 * 16 + col]);
      ar = MF::op(wr, b, ar);
      ai = MF::op(wi, b, ai);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k1o = 16 * mt + MF::row(v, grp);
      if (k1o >= n1 || j >= q) continue;
      const int m = sd_mod((int64_t)k1o * c2, nx);
      const double tr = d.twid[2 * m], ti = d.twid[2 * m + 1];
      const double yr = (double)ar[v], yi = (double)ai[v];
      const size_t o = (((size_t)k1o * n2 + c2) * q + j) * 2;
      sd.FT[o] = yr * tr - yi * ti;
      sd.FT[o + 1] = yr * ti + yi * tr;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sdf_a(const TankDev* __restrict__ td, int which, const T* __restrict__ r, int gate,
        const double* __restrict__ nscale, T* __restrict__ vout) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sdf_a_body<T>(d, which, r, nscale, vout, (int)blockIdx.x, (int)blockIdx.y);
}

// pass B (block per k1): FG[k1 + n1 k2][j] = sum_c2 w_n2^{k2 c2} FT[k1][c2][j]
template <typename T>
__device__ __forceinline__ void sdf_b_body(const TankDev& d, int which, int bx, int by) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const SDData& sd = d.sd[which];
  const int q = sd.q, n1 = sd.fft_n1, n2 = sd.fft_n2;
  const int k1 = bx;
  const int KS = (n2 + 3) / 4, nMT = (n2 + 15) / 16;
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const SEM_GLOBAL double* ftg = gview(sd.FT) + (size_t)k1 * n2 * q * 2;
  const SEM_GLOBAL double* twg = gview(d.twid);
  const int nt = by;   // this workgroup's 16 line unknowns
  for (int mt = wv; mt < nMT; mt += kWaves) {
    const int k2 = 16 * mt + col, j = 16 * nt + col;
    V4 gr = V4{0, 0, 0, 0}, gi = V4{0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < KS; ++s) {
      const int c2 = 4 * s + grp;
      // (operands loaded from clamped indices, then selected)
      const bool okw = k2 < n2 && c2 < n2, okb = c2 < n2 && j < q;
      const int m = okw ? sd_mod((int64_t)k2 * c2, n2) * n1 : 0;
      const double twr = twg[2 * m], twi = twg[2 * m + 1];
      const size_t ob = ((size_t)min(c2, n2 - 1) * q + min(j, q - 1)) * 2;
      const double fr = ftg[ob], fi = ftg[ob + 1];
      const T wr = okw ? T(twr) : T(0), wi = okw ? T(twi) : T(0);
      const T br = okb ? T(fr) : T(0), bi = okb ? T(fi) : T(0);
      gr = MF::op(wr, br, gr);
      gr = MF::op(-wi, bi, gr);
      gi = MF::op(wr, bi, gi);
      gi = MF::op(wi, br, gi);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k2o = 16 * mt + MF::row(v, grp);
      if (k2o >= n2 || j >= q) continue;
      const size_t o = (((size_t)k1 + (size_t)n1 * k2o) * q + j) * 2;
      sd.FG[o] = (double)gr[v];
      sd.FG[o + 1] = (double)gi[v];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sdf_b(const TankDev* __restrict__ td, int which, int gate) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sdf_b_body<T>(d, which, (int)blockIdx.x, (int)blockIdx.y);
}

// per-mode solves x^_k = S^_k^{-1} g^_k (thread per mode and row; each block
// holds 256 / q whole modes and, for walls, adds its share of lines nx-1 and 0)
template <typename T>
__device__ __forceinline__ void sdf_solve_body(const TankDev& d, int which, int bx, int by) {
  const SDData& sd = d.sd[which];
  const int q = sd.q, nx = d.nx;
  const int ml = fft_modes_per_block(q), ns = fft_slots(ml);
  for (int t = threadIdx.x; t < ns * q; t += blockDim.x) {
    const int kk = t / q, i = t - kk * q;
    const int k = fft_mode(bx, kk, ml, nx);
    double xr = 0, xi = 0;
    if (k >= 0) {
      const bool cj = 2 * k > nx;   // stored as the conjugate of mode nx - k
      const SEM_GLOBAL T* S = gview(SdMat<T>::Shat(sd)) + (size_t)(cj ? nx - k : k) * q * q * 2;
      const double sgn = cj ? -1.0 : 1.0;
      const SEM_GLOBAL double* g = gview(sd.FG) + (size_t)k * q * 2;
#pragma unroll 8
      for (int j = 0; j < q; ++j) {
        const double sr = (double)S[((size_t)j * q + i) * 2], si = sgn * (double)S[((size_t)j * q + i) * 2 + 1];
        const double gr = g[2 * j], gi = g[2 * j + 1];
        xr += sr * gr - si * gi;
        xi += sr * gi + si * gr;
      }
      sd.XH[((size_t)k * q + i) * 2] = xr;
      sd.XH[((size_t)k * q + i) * 2 + 1] = xi;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sdf_solve(const TankDev* __restrict__ td, int which, int gate) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sdf_solve_body<T>(d, which, (int)blockIdx.x, (int)blockIdx.y);
}

// pass C (block per k1): FT[c2][k1][j] = conj(w_nx)^{k1 c2} sum_k2 conj(w_n2)^{k2 c2} x^[k1 + n1 k2][j]
template <typename T>
__device__ __forceinline__ void sdf_c_body(const TankDev& d, int which, int bx, int by) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const SDData& sd = d.sd[which];
  const int q = sd.q, nx = d.nx, n1 = sd.fft_n1, n2 = sd.fft_n2;
  const int k1 = bx;
  const int KS = (n2 + 3) / 4, nMT = (n2 + 15) / 16;
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const SEM_GLOBAL double* twg = gview(d.twid);
  const SEM_GLOBAL double* xhg = gview(sd.XH);
  const int nt = by;   // this workgroup's 16 line unknowns
  for (int mt = wv; mt < nMT; mt += kWaves) {
    const int c2 = 16 * mt + col, j = 16 * nt + col;
    V4 ur = V4{0, 0, 0, 0}, ui = V4{0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < KS; ++s) {
      const int k2 = 4 * s + grp;
      // conj(w_n2)^{k2 c2} = (twr, -twi); operands loaded from clamped indices, then selected
      const bool okw = c2 < n2 && k2 < n2, okb = k2 < n2 && j < q;
      const int m = okw ? sd_mod((int64_t)k2 * c2, n2) * n1 : 0;
      const double twr = twg[2 * m], twi = twg[2 * m + 1];
      const size_t o = (((size_t)k1 + (size_t)n1 * min(k2, n2 - 1)) * q + min(j, q - 1)) * 2;
      const double xr = xhg[o], xi = xhg[o + 1];
      const T wr = okw ? T(twr) : T(0), wi = okw ? T(-twi) : T(0);
      const T br = okb ? T(xr) : T(0), bi = okb ? T(xi) : T(0);
      ur = MF::op(wr, br, ur);
      ur = MF::op(-wi, bi, ur);
      ui = MF::op(wr, bi, ui);
      ui = MF::op(wi, br, ui);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c2o = 16 * mt + MF::row(v, grp);
      if (c2o >= n2 || j >= q) continue;
      const int m = sd_mod((int64_t)k1 * c2o, nx);
      const double tr = d.twid[2 * m], ti = -d.twid[2 * m + 1];   // conj(w_nx)^{k1 c2}
      const double a = (double)ur[v], b = (double)ui[v];
      const size_t o = (((size_t)c2o * n1 + k1) * q + j) * 2;
      sd.FT[o] = a * tr - b * ti;
      sd.FT[o + 1] = a * ti + b * tr;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sdf_c(const TankDev* __restrict__ td, int which, int gate) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sdf_c_body<T>(d, which, (int)blockIdx.x, (int)blockIdx.y);
}

// pass D (block per c2): XL[n2 c1 + c2][j] = Re sum_k1 conj(w_n1)^{k1 c1} FT[c2][k1][j] / nx
template <typename T>
__device__ __forceinline__ void sdf_d_body(const TankDev& d, int which, int bx, int by) {
  using MF = Mfma<T>;
  using V4 = typename MF::V4;
  const SDData& sd = d.sd[which];
  const int q = sd.q, nx = d.nx, n1 = sd.fft_n1, n2 = sd.fft_n2;
  const int c2 = bx;
  const int KS = (n1 + 3) / 4, nMT = (n1 + 15) / 16;
  const int lane = threadIdx.x & 63, wv = wave_id(), col = lane & 15, grp = lane >> 4;
  const SEM_GLOBAL double* ftg = gview(sd.FT) + (size_t)c2 * n1 * q * 2;
  const SEM_GLOBAL double* twg = gview(d.twid);
  const double inx = 1.0 / nx;
  const int nt = by;   // this workgroup's 16 line unknowns
  for (int mt = wv; mt < nMT; mt += kWaves) {
    const int c1 = 16 * mt + col, j = 16 * nt + col;
    V4 acc = V4{0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < KS; ++s) {
      const int k1 = 4 * s + grp;
      // Re(conj(w) u) = twr ur + twi ui; operands loaded from clamped indices, then selected
      const bool okw = c1 < n1 && k1 < n1, okb = k1 < n1 && j < q;
      const int m = okw ? sd_mod((int64_t)k1 * c1, n1) * n2 : 0;
      const double twr = twg[2 * m], twi = twg[2 * m + 1];
      const size_t ob = ((size_t)min(k1, n1 - 1) * q + min(j, q - 1)) * 2;
      const double fr = ftg[ob], fi = ftg[ob + 1];
      const T wr = okw ? T(twr) : T(0), wi = okw ? T(twi) : T(0);
      const T br = okb ? T(fr) : T(0), bi = okb ? T(fi) : T(0);
      acc = MF::op(wr, br, acc);
      acc = MF::op(wi, bi, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c1o = 16 * mt + MF::row(v, grp);
      if (c1o >= n1 || j >= q) continue;
      sd.XL[((size_t)n2 * c1o + c2) * q + j] = (double)acc[v] * inx;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_sdf_d(const TankDev* __restrict__ td, int which, int gate) {
  const TankDev& d = *td;
  if (gate && d.ks->done) return;
  sdf_d_body<T>(d, which, (int)blockIdx.x, (int)blockIdx.y);
}

namespace {
// dynamic LDS of the chain's kernels for one tank
struct SdLds {
  size_t cond, modes, back, fa, fsolve, wall;
};
// shapes of a tank's condensation and back-substitution products, alone or
// in a batched launch
// in a batched launch (word: bytes of the arithmetic type)
void sd_shapes(const TankDev& h, const SDData& sd, size_t word, bool batched, SdShape* s1, SdShape* s3) {
  if (!batched) {
    *s1 = sd_shape(h.nx, sd.nMT1);
    *s3 = sd_shape(h.nx, sd.nMT3);
    return;
  }
  *s1 = sd_shape_b(h.nx, sd.nMT1, false, word);
  *s3 = sd_shape_b(h.nx, sd.nMT3, sd_back_dft(h.nx, sd.q, sd.fft_n1, sd.nMT3), word);
}
SdLds sd_lds(const TankDev& h, const SDData& sd, size_t word, bool batched) {
  SdShape s1, s3;
  sd_shapes(h, sd, word, batched, &s1, &s3);
  SdLds l;
  l.cond = sd_cond_stage_bytes(s1.ntw, word, s1.split) + sizeof(int32_t) * sd.nI;
  l.modes = sizeof(double) * (sd_part_words(sd.q) + kModesPerBlockMax * (size_t)sd.q * 2);
  l.back = sizeof(double) * ((16 * (size_t)s3.ntw + 1) * (sd.q + 1) + (s3.split ? kWaves * s3.ntw * 256 : 0));
  l.fa = sd.fft_n1 ? sizeof(double) * 4 * (size_t)((sd.fft_n1 + 3) / 4) * 16 : 0;
  l.fsolve = 0;
  l.wall = 0;
  return l;
}
struct SdGrid {
  int cx, cy, bx, by;
};
// grids of the condensation (cx, cy) and back-substitution (bx, by) products
SdGrid sd_grid(const TankDev& h, const SDData& sd, size_t word, bool batched) {
  SdShape s1, s3;
  sd_shapes(h, sd, word, batched, &s1, &s3);
  const int ct = (h.nx + 15) / 16;
  return SdGrid{(ct + s1.ntw - 1) / s1.ntw, s1.split ? sd.nMT1 : (sd.nMT1 + 3) / 4, (ct + s3.ntw - 1) / s3.ntw,
                s3.split ? sd.nMT3 : (sd.nMT3 + 3) / 4};
}
}  // namespace

// ------------------------------------------------------------ batched chain
// The same kernels over many tanks (one work item per workgroup of a tank's
// own grid).  Input rin; with jn > 0 it is read as w / ||w|| and that
// normalised vector is stored as V_jn on the way.
template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_sd_cond_b(BatchArgs ba, int which, VSel rin, int jn, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  sd_cond_body<T, true>(d, which, bvec<T>(d, rin), jn > 0 ? krylov_norm(d, jn) : nullptr,
                  jn > 0 ? bvec<T>(d, VSel{BV_V, jn}) : nullptr, it_.bx, it_.by);
}
template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_sd_modes_b(BatchArgs ba, int which, VSel rin, int jn, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  sd_modes_any<T, true>(d, which, bvec<T>(d, rin), jn > 0 ? krylov_norm(d, jn) : nullptr,
                  jn > 0 ? bvec<T>(d, VSel{BV_V, jn}) : nullptr, it_.bx, it_.by);
}
template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_sdf_a_b(BatchArgs ba, int which, VSel rin, int jn, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  sdf_a_body<T>(d, which, bvec<T>(d, rin), jn > 0 ? krylov_norm(d, jn) : nullptr,
                jn > 0 ? bvec<T>(d, VSel{BV_V, jn}) : nullptr, it_.bx, it_.by);
}
template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_sd_wall_b(BatchArgs ba, int which, VSel rin, int jn, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  sd_wall_body<T>(d, which, bvec<T>(d, rin), jn > 0 ? krylov_norm(d, jn) : nullptr, it_.bx, it_.by);
}
template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_sd_back_b(BatchArgs ba, int which, VSel zout, int jn, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  sd_back_body<T, true>(d, which, bvec<T>(d, zout), jn > 0 ? bvec<T>(d, VSel{BV_V, jn}) : nullptr, it_.bx, it_.by);
}
#define SEM_SD_PLAIN_B(NAME, BODY)                                                          \
  template <typename T>                                                                     \
  __global__ void __launch_bounds__(kBlockThreads) NAME(BatchArgs ba, int which, int gate) { \
    SEM_BATCH_TANK(ba)                                                                      \
    if (gate && d.ks->done) return;                                                         \
    BODY<T>(d, which, it_.bx, it_.by);                                                      \
  }
SEM_SD_PLAIN_B(k_sd_idft_b, sd_idft_body)
SEM_SD_PLAIN_B(k_sdf_b_b, sdf_b_body)
SEM_SD_PLAIN_B(k_sdf_solve_b, sdf_solve_body)
SEM_SD_PLAIN_B(k_sdf_c_b, sdf_c_body)
SEM_SD_PLAIN_B(k_sdf_d_b, sdf_d_body)
#undef SEM_SD_PLAIN_B
__global__ void __launch_bounds__(kBlockThreads) k_sd_wall_lines_b(BatchArgs ba, int which, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  sd_wall_lines_body(d, which, it_.bx, it_.by);
}
__global__ void __launch_bounds__(kBlockThreads) k_sd_wall_modes_b(BatchArgs ba, int which, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  sd_wall_modes_body(d, which, it_.bx, it_.by);
}

namespace {
void add_grid(BatchStage& st, int tank, int gx, int gy, size_t lds) {
  for (int y = 0; y < gy; ++y)
    for (int x = 0; x < gx; ++x) st.items.push_back(BatchItem{tank, x, y, gx});
  st.lds = std::max(st.lds, lds);
}

// Orders a product's work items so that those reading the same factor rows
// (same tank and M-tile group `by`) sit at positions of the same residue mod
// 8: the chip hands consecutive workgroups to its eight XCDs in turn, so the
// rows are fetched into one XCD's L2 instead of all eight.  Groups go to the
// least loaded XCD; once a residue's queue is empty its positions take items
// of the longest remaining queue.  (Each item writes its own outputs: the
// order does not change any result.)
void xcd_affine(BatchStage& st) {
  constexpr int kXcd = 8;
  std::vector<std::vector<BatchItem>> groups;
  std::map<std::pair<int, int>, size_t> gid;
  for (const BatchItem& it : st.items) {
    auto key = std::make_pair(it.tank, it.by);
    auto f = gid.find(key);
    if (f == gid.end()) {
      f = gid.emplace(key, groups.size()).first;
      groups.emplace_back();
    }
    groups[f->second].push_back(it);
  }
  std::vector<std::vector<BatchItem>> q(kXcd);
  for (const auto& g : groups) {
    size_t best = 0;
    for (size_t k = 1; k < q.size(); ++k)
      if (q[k].size() < q[best].size()) best = k;
    q[best].insert(q[best].end(), g.begin(), g.end());
  }
  std::vector<size_t> head(kXcd, 0);
  std::vector<BatchItem> out;
  out.reserve(st.items.size());
  while (out.size() < st.items.size()) {
    const int r = (int)(out.size() % kXcd);
    int k = r;
    if (head[k] == q[k].size()) {
      size_t rem = 0;
      for (int k2 = 0; k2 < kXcd; ++k2)
        if (q[k2].size() - head[k2] > rem) {
          rem = q[k2].size() - head[k2];
          k = k2;
        }
    }
    out.push_back(q[k][head[k]++]);
  }
  st.items.swap(out);
}
}  // namespace

void plan_sd(const std::vector<TankDev>& tanks, const std::vector<int>& ids, int which, int f32, BatchSD* out) {
  *out = BatchSD{};
  for (int t : ids) {
    const TankDev& h = tanks[t];
    const SDData& sd = h.sd[which];
    const SdLds l = sd_lds(h, sd, f32 ? sizeof(float) : sizeof(double), true);
    const SdGrid g = sd_grid(h, sd, f32 ? sizeof(float) : sizeof(double), true);
    const int ct = (h.nx + 15) / 16;
    add_grid(out->cond, t, g.cx, g.cy, l.cond);
    if (sd.fft_n1) {
      const int nnt = (sd.q + 15) / 16;
      add_grid(out->fa, t, sd.fft_n2, nnt, l.fa);
      add_grid(out->fb, t, sd.fft_n1, nnt, 0);
      add_grid(out->fsolve, t, fft_mode_blocks(h.nx, fft_modes_per_block(sd.q)), 1, l.fsolve);
      add_grid(out->fc, t, sd.fft_n1, nnt, 0);
      add_grid(out->fd, t, sd.fft_n2, nnt, 0);
    } else {
      add_grid(out->modes, t, paired_blocks(h.nx, modes_per_block(h.nx) / 2), 1, l.modes);
      if (!sd_back_dft(h.nx, sd.q, sd.fft_n1, sd.nMT3)) add_grid(out->idft, t, ct, (sd.q + 15) / 16, 0);
    }
    if (sd.wall) {
      add_grid(out->wlines, t, 2 * sd.q, 1, 0);
      add_grid(out->wall, t, sd.q, 1, l.wall);
      const int64_t nm = (int64_t)h.nx * sd.q + sd.nI;
      add_grid(out->wmodes, t, (int)((nm + kBlockThreads - 1) / kBlockThreads), 1, 0);
    }
    add_grid(out->back, t, g.bx, g.by, l.back);
  }
  xcd_affine(out->cond);
  xcd_affine(out->back);
}

template <typename T>
static void sd_b_t(const BatchArgs& a0, const BatchSD& p, int which, VSel rin, VSel zout, int jn, int gate,
                   hipStream_t st) {
  auto go = [&](const BatchStage& s, auto kern, auto... args) {
    if (s.items.empty()) return;
    BatchArgs a = a0;
    a.items = s.dev;
    hipLaunchKernelGGL(kern, dim3((unsigned)s.items.size()), dim3(kBlockThreads), s.lds, st, a, args...);
  };
  // the wall correction needs the modes of the periodic solve; the inverse
  // transforms of the direct and the four-step tanks are independent
  go(p.cond, k_sd_cond_b<T>, which, rin, jn, gate);
  go(p.fa, k_sdf_a_b<T>, which, rin, jn, gate);
  go(p.fb, k_sdf_b_b<T>, which, gate);
  go(p.fsolve, k_sdf_solve_b<T>, which, gate);
  go(p.modes, k_sd_modes_b<T>, which, rin, jn, gate);
  go(p.wlines, k_sd_wall_lines_b, which, gate);
  go(p.wall, k_sd_wall_b<T>, which, rin, jn, gate);
  go(p.wmodes, k_sd_wall_modes_b, which, gate);
  go(p.fc, k_sdf_c_b<T>, which, gate);
  go(p.fd, k_sdf_d_b<T>, which, gate);
  go(p.idft, k_sd_idft_b<T>, which, gate);
  go(p.back, k_sd_back_b<T>, which, zout, jn, gate);
}

void launch_sd_b(const BatchArgs& a, const BatchSD& p, int which, VSel rin, VSel zout, int jn, int gate, int f32,
                 hipStream_t st) {
  if (f32) sd_b_t<float>(a, p, which, rin, zout, jn, gate, st);
  else sd_b_t<double>(a, p, which, rin, zout, jn, gate, st);
}

template <typename T>
static void sd_t(const TankDev& h, const TankDev* d, int which, const T* u, T* y, int gate, const double* nscale,
                 T* vout, hipStream_t st) {
  const SDData& sd = h.sd[which];
  const unsigned ct = (unsigned)((h.nx + 15) / 16);
  const SdLds lds = sd_lds(h, sd, sizeof(T), false);
  const SdGrid g = sd_grid(h, sd, sizeof(T), false);
  const size_t l2 = lds.modes;
  hipLaunchKernelGGL(k_sd_cond<T>, dim3(g.cx, g.cy), dim3(kBlockThreads), lds.cond, st, d, which, u, gate, nscale,
                     vout);
  const int n1 = sd.fft_n1, n2 = sd.fft_n2;
  if (n1) {
    const size_t la = sizeof(double) * 4 * (size_t)((n1 + 3) / 4) * 16;
    const unsigned nnt = (unsigned)((sd.q + 15) / 16);
    hipLaunchKernelGGL(k_sdf_a<T>, dim3(n2, nnt), dim3(kBlockThreads), la, st, d, which, u, gate, nscale, vout);
    hipLaunchKernelGGL(k_sdf_b<T>, dim3(n1, nnt), dim3(kBlockThreads), 0, st, d, which, gate);
    const int ml = fft_modes_per_block(sd.q);
    hipLaunchKernelGGL(k_sdf_solve<T>, dim3(fft_mode_blocks(h.nx, ml)), dim3(kBlockThreads), lds.fsolve, st, d,
                       which, gate);
  } else {
    hipLaunchKernelGGL(k_sd_modes<T>, dim3(paired_blocks(h.nx, modes_per_block(h.nx) / 2)), dim3(kBlockThreads), l2, st, d, which,
                       u, gate, nscale, vout);
  }
  if (sd.wall) {
    hipLaunchKernelGGL(k_sd_wall_lines, dim3(2 * sd.q), dim3(kBlockThreads), 0, st, d, which, gate);
    hipLaunchKernelGGL(k_sd_wall<T>, dim3(sd.q), dim3(kBlockThreads), 0, st, d, which, u, gate, nscale);
    const int64_t nm = (int64_t)h.nx * sd.q + sd.nI;
    hipLaunchKernelGGL(k_sd_wall_modes, dim3((unsigned)((nm + kBlockThreads - 1) / kBlockThreads)),
                       dim3(kBlockThreads), 0, st, d, which, gate);
  }
  if (n1) {
    const unsigned nnt = (unsigned)((sd.q + 15) / 16);
    hipLaunchKernelGGL(k_sdf_c<T>, dim3(n1, nnt), dim3(kBlockThreads), 0, st, d, which, gate);
    hipLaunchKernelGGL(k_sdf_d<T>, dim3(n2, nnt), dim3(kBlockThreads), 0, st, d, which, gate);
  } else if (!sd_back_dft(h.nx, sd.q, sd.fft_n1, sd.nMT3)) {
    hipLaunchKernelGGL(k_sd_idft<T>, dim3(ct, (sd.q + 15) / 16), dim3(kBlockThreads), 0, st, d, which, gate);
  }
  hipLaunchKernelGGL(k_sd_back<T>, dim3(g.bx, g.by), dim3(kBlockThreads), lds.back, st, d, which, y, gate, vout);
}

void launch_sd(const TankDev& h, const TankDev* d, int which, const double* u, double* y, int gate, hipStream_t st,
               const double* nscale, double* vout) {
  sd_t<double>(h, d, which, u, y, gate, nscale, vout, st);
}
void launch_sd(const TankDev& h, const TankDev* d, int which, const float* u, float* y, int gate, hipStream_t st,
               const double* nscale, float* vout) {
  sd_t<float>(h, d, which, u, y, gate, nscale, vout, st);
}

}  // namespace sem
