// HIP kernels (gfx950) of the spectral element free-surface path.
//
// Data layout (one tank):
//   volume vectors [n]: column-major node numbering.  Column c owns nc =
//     P*(P*nz+1) nodes: its left vertical line (nl = P*nz+1 nodes, ordered
//     by sigma) followed by its interior nodes.  The right line of column c is
//     the left line of column c+1 (periodic wrap, or the extra wall line
//     stored at nx*nc).
//   element blocks: workgroup b handles cb consecutive columns (EB = cb*2nz
//     elements, T = ceil(EB/16) MFMA tiles).  Inputs are staged through LDS,
//     element results are summed per node in a fixed order, interior nodes
//     and the block's left line are stored, the contribution to the right
//     line goes to a side buffer and is added by a fix-up pass (two fixed
//     contributions per shared line: results are deterministic).
//   geometric factors G: MFMA tile layout [blk][tile][comp][perm(row)][16].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "launch.hpp"
#include "reduce.hpp"

namespace sem {

// ------------------------------------------------------------ helpers
__device__ inline double block_sum(double v, double* red) {
  // deterministic tree reduction over a 256-thread workgroup
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ inline bool finite(double v) { return v - v == 0.0; }

__device__ inline int64_t right_line_base(const TankDev& d, int c) {
  // global index of the first node of the vertical line at x_c (c in 0..nx)
  if (c < d.nx) return (int64_t)c * d.nc;
  return d.periodic ? 0 : (int64_t)d.nx * d.nc;
}

// precision traits: working type T of vectors and operators, storage type
// of the geometric factors (double, float or bfloat16 bits)
struct BF16 {};
__device__ inline float bf16_to_float(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }
__device__ inline uint16_t float_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t r = 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)((u + r) >> 16);
}
template <typename T, typename GS>
struct Prec;
template <>
struct Prec<double, double> {
  __device__ static const double* Dr(const TankDev& d) { return d.Dr; }
  __device__ static const double* Ds(const TankDev& d) { return d.Ds; }
  __device__ static const double* MDr(const TankDev& d) { return d.MDr; }
  __device__ static const double* MDs(const TankDev& d) { return d.MDs; }
  __device__ static const double* Mref(const TankDev& d) { return d.Mref; }
  __device__ static const double* pre_lap(const TankDev& d) { return d.pre_lap; }
  __device__ static double G(const TankDev& d, int64_t b, int eb, int i, int c) {
    return d.G[tile_index64(d.T, d.NpP, b, eb, i, 3, c)];
  }
};
template <>
struct Prec<float, float> {
  __device__ static const float* Dr(const TankDev& d) { return d.Dr32; }
  __device__ static const float* Ds(const TankDev& d) { return d.Ds32; }
  __device__ static const float* MDr(const TankDev& d) { return d.MDr32; }
  __device__ static const float* MDs(const TankDev& d) { return d.MDs32; }
  __device__ static const float* Mref(const TankDev& d) { return d.Mref32; }
  __device__ static const float* pre_lap(const TankDev& d) { return d.pre_lap32; }
  __device__ static float G(const TankDev& d, int64_t b, int eb, int i, int c) {
    return d.G32[tile_index(d.T, d.NpP, b, eb, i, 3, c)];
  }
};
template <>
struct Prec<float, BF16> : Prec<float, float> {
  __device__ static float G(const TankDev& d, int64_t b, int eb, int i, int c) {
    return bf16_to_float(d.G16[tile_index(d.T, d.NpP, b, eb, i, 3, c)]);
  }
};

// ------------------------------------------------------------ coefficients
// G = |J| Lam K Lam^T and 1/d at every element node (paper Sec. 2).
template <int P>
__device__ __forceinline__ void coef_body(const TankDev& d, const double* __restrict__ eta,
                                          const double* __restrict__ etax, int what, int bx) {
  constexpr int Np = (P + 1) * (P + 2) / 2;
  // Sixteen consecutive lanes take the sixteen elements of one tile at one
  // node, the next sixteen the next node: every store below is then one
  // contiguous run of the tile layout.  Grid: nb * T * Np * 16 threads.
  const int64_t gid = (int64_t)bx * blockDim.x + threadIdx.x;
  const int e16 = (int)(gid & 15);
  const int64_t r = gid >> 4;
  const int m = (int)(r % Np);
  const int64_t g = r / Np;  // tile over the whole tank: b * T + tile
  if (g >= (int64_t)d.nb * d.T) return;
  const int b = (int)(g / d.T);
  const int eb = (int)(g - (int64_t)b * d.T) * 16 + e16;
  if (eb >= d.EB) return;
  const int lc = eb / (2 * d.nz), jt = eb - lc * 2 * d.nz;
  const int c = b * d.cb + lc;
  if (c >= d.nx) return;
  int t = jt & 1;
  const double* lay = d.lay + jt * 8;
  const double* w = d.colw + ((size_t)t * d.NpP + m) * (P + 1);
  double et = 0, ex = 0, hh = 0, hxx = 0;
  for (int k = 0; k <= P; ++k) {
    int s = c * P + k;
    if (s >= d.ns) s -= d.ns;  // periodic wrap
    et += w[k] * eta[s];
    ex += w[k] * (etax ? etax[s] : 0.0);
    hh += w[k] * d.h[s];
    hxx += w[k] * d.hx[s];
  }
  double zeta = d.nodeq[((size_t)t * d.NpP + m) * 2 + 1];
  double sig = lay[5] + zeta * lay[6];
  double dd = et + hh;
  if (!(dd > 0.0)) atomicOr(d.status, finite(dd) ? ST_DOMAIN : ST_NONFINITE);
  double q = (1.0 - sig) * hxx - sig * ex;
  double K00 = dd, K01 = q, K11 = (1.0 + q * q) / dd;
  double l00 = lay[0], l01 = lay[1], l10 = lay[2], l11 = lay[3], J = lay[4];
  // G = J Lam K Lam^T
  double a0 = l00 * K00 + l01 * K01, a1 = l00 * K01 + l01 * K11;
  double b0 = l10 * K00 + l11 * K01, b1 = l10 * K01 + l11 * K11;
  double Grr = J * (a0 * l00 + a1 * l01);
  double Grs = J * (a0 * l10 + a1 * l11);
  double Gss = J * (b0 * l10 + b1 * l11);
  if (what & 2) d.invd[tile_index(d.T, d.NpP, b, eb, m, 1, 0)] = 1.0 / dd;
  if (what & 4) d.sigx[tile_index(d.T, d.NpP, b, eb, m, 1, 0)] = q / dd;
  if (!(what & 1)) return;
  d.G[tile_index64(d.T, d.NpP, b, eb, m, 3, 0)] = Grr;
  d.G[tile_index64(d.T, d.NpP, b, eb, m, 3, 1)] = Grs;
  d.G[tile_index64(d.T, d.NpP, b, eb, m, 3, 2)] = Gss;
  d.G32[tile_index(d.T, d.NpP, b, eb, m, 3, 0)] = (float)Grr;
  d.G32[tile_index(d.T, d.NpP, b, eb, m, 3, 1)] = (float)Grs;
  d.G32[tile_index(d.T, d.NpP, b, eb, m, 3, 2)] = (float)Gss;
  d.G16[tile_index(d.T, d.NpP, b, eb, m, 3, 0)] = float_to_bf16((float)Grr);
  d.G16[tile_index(d.T, d.NpP, b, eb, m, 3, 1)] = float_to_bf16((float)Grs);
  d.G16[tile_index(d.T, d.NpP, b, eb, m, 3, 2)] = float_to_bf16((float)Gss);
}

template <int P>
__global__ void k_coef(const TankDev* __restrict__ td, const double* __restrict__ eta,
                       const double* __restrict__ etax, int what) {
  coef_body<P>(*td, eta, etax, what, blockIdx.x);
}

// ------------------------------------------------------------ gather kernels

// Per block: y_owned = sum over the block's elements of op_e(u_e).
// LDS: region of the input (cb*nc + nl), per-element stage buffers.
template <int P, int OP, typename T = double, typename GS = double>
__device__ __forceinline__ void gather_body(const TankDev& d, const T* __restrict__ u, T* __restrict__ y,
                                            T* __restrict__ side, int flags, int b) {
  using PR = Prec<T, GS>;
  constexpr int Np = (P + 1) * (P + 2) / 2;
  constexpr int NpP = (Np + 15) / 16 * 16;
  extern __shared__ unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int c0 = b * d.cb;
  const int cbb = min(d.cb, d.nx - c0);
  const int nc = d.nc, nl = d.nl;
  const int nreg = cbb * nc + nl;
  const int EBb = cbb * 2 * d.nz;
  T* ureg = lds;                         // [cb*nc + nl]
  T* st1 = ureg + (d.cb * nc + nl);      // [EB][NpP] first stage
  T* st2 = st1 + d.EB * NpP;             // [EB][NpP] second stage
  T* st3 = st2 + d.EB * NpP;             // [EB][NpP] element outputs
  // 1. stage the input region
#pragma unroll 4
  for (int q = threadIdx.x; q < nreg; q += blockDim.x) {
    int lc = q / nc, ql = q - lc * nc;
    int64_t gi;
    if (lc < cbb) gi = (int64_t)(c0 + lc) * nc + ql;
    else gi = (ql < nl) ? right_line_base(d, c0 + cbb) + ql : -1;
    ureg[q] = gi >= 0 ? u[gi] : T(0);
  }
  __syncthreads();
  // 2. per-element work, thread per (element, node)
  const int work = EBb * Np;
  if (OP == OP_STIFF || OP == OP_SZ || OP == OP_SU) {
    // phase 1: derivatives and pointwise flux f_a = sum_b G_ab D_b u
    for (int it = threadIdx.x; it < work; it += blockDim.x) {
      int eb = it / Np, i = it - eb * Np;
      int lc = eb / (2 * d.nz), jt = eb - lc * 2 * d.nz;
      const int32_t* loc = d.elem_loc + jt * NpP;
      T tr = 0, ts = 0;
      const T* Dr = PR::Dr(d);
      const T* Ds = PR::Ds(d);
      for (int k = 0; k < Np; ++k) {
        T uk = ureg[lc * nc + loc[k]];
        tr += Dr[i * NpP + k] * uk;
        ts += Ds[i * NpP + k] * uk;
      }
      if (OP == OP_STIFF) {
        T grr = PR::G(d, b, eb, i, 0);
        T grs = PR::G(d, b, eb, i, 1);
        T gss = PR::G(d, b, eb, i, 2);
        st1[eb * NpP + i] = grr * tr + grs * ts;
        st2[eb * NpP + i] = grs * tr + gss * ts;
      } else if (OP == OP_SZ) {
        const double* lay = d.lay + jt * 8;
        T dsig = T(lay[1]) * tr + T(lay[3]) * ts;
        st1[eb * NpP + i] = dsig * T(d.invd[tile_index(d.T, NpP, b, eb, i, 1, 0)]);
      } else {
        // d phi/dx = d_x Phi + sigma_x d_sigma Phi (chain rule of the sigma-map)
        const double* lay = d.lay + jt * 8;
        T dx = T(lay[0]) * tr + T(lay[2]) * ts;
        T dsig = T(lay[1]) * tr + T(lay[3]) * ts;
        st1[eb * NpP + i] = dx + dsig * T(d.sigx[tile_index(d.T, NpP, b, eb, i, 1, 0)]);
      }
    }
    __syncthreads();
    // phase 2
    for (int it = threadIdx.x; it < work; it += blockDim.x) {
      int eb = it / Np, i = it - eb * Np;
      T acc = 0;
      if (OP == OP_STIFF) {
        const T* MDr = PR::MDr(d);
        const T* MDs = PR::MDs(d);
        for (int k = 0; k < Np; ++k)
          acc += MDr[k * NpP + i] * st1[eb * NpP + k] + MDs[k * NpP + i] * st2[eb * NpP + k];
      } else {
        int jt = eb % (2 * d.nz);
        T J = T(d.lay[jt * 8 + 4]);
        const T* Mr = PR::Mref(d);
        for (int k = 0; k < Np; ++k) acc += Mr[i * NpP + k] * st1[eb * NpP + k];
        acc *= J;
      }
      st3[eb * NpP + i] = acc;
    }
  } else {
    for (int it = threadIdx.x; it < work; it += blockDim.x) {
      int eb = it / Np, i = it - eb * Np;
      int lc = eb / (2 * d.nz), jt = eb - lc * 2 * d.nz;
      const int32_t* loc = d.elem_loc + jt * NpP;
      const T* A;
      T scale = 1;
      if (OP == OP_MASS) {
        A = PR::Mref(d);
        scale = T(d.lay[jt * 8 + 4]);
      } else {
        int c = c0 + lc;
        int cls = d.nclass_col == 1 ? 0 : (c == 0 ? 0 : (c == d.nx - 1 ? 2 : 1));
        if (d.nclass_col == 3 && d.nx == 1) cls = 0;
        const T* base = (OP == OP_PRE_LAP) ? PR::pre_lap(d) : reinterpret_cast<const T*>(d.pre_mass);
        A = base + ((size_t)(cls * 2 * d.nz + jt)) * NpP * NpP;
      }
      T acc = 0;
      for (int k = 0; k < Np; ++k) acc += A[i * NpP + k] * ureg[lc * nc + loc[k]];
      st3[eb * NpP + i] = scale * acc;
    }
  }
  __syncthreads();
  // 3. node sums in a fixed order; store owned nodes, side buffer for the right line
  const T sgn = (flags & F_NEG) ? T(-1) : T(1);
  const int nown = cbb * nc;
  for (int q = threadIdx.x; q < nown + nl; q += blockDim.x) {
    int lc = q / nc, ql = q - lc * nc;
    T acc = 0;
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
          acc += st3[(lc - 1) * 2 * d.nz * NpP + off];
        } else {
          acc += st3[lc * 2 * d.nz * NpP + off];
        }
      }
      acc *= sgn;
      if ((flags & F_MASK_SURF) && d.is_surf_loc[ql]) acc = T(0);
      y[(int64_t)(c0 + lc) * nc + ql] = acc;
    } else {
      // right line: contributions of column cbb-1 through its right-line nodes
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
        acc += st3[(cbb - 1) * 2 * d.nz * NpP + (e & 0x3fffffff)];
      }
      acc *= sgn;
      if ((flags & F_MASK_SURF) && d.is_surf_loc[ql]) acc = T(0);
      side[(size_t)b * nl + ql] = acc;
    }
  }
}

template <int P, int OP, typename T = double, typename GS = double>
__global__ void __launch_bounds__(kBlockThreads)
k_gather(const TankDev* __restrict__ td, const T* __restrict__ u, T* __restrict__ y,
         T* __restrict__ side, int flags) {
  const TankDev& d = *td;
  if ((flags & F_GATE) && d.ks->done) return;
  gather_body<P, OP, T, GS>(d, u, y, side, flags, blockIdx.x);
}

// adds the right-line contributions of each block to the stored left lines
template <typename T>
__device__ __forceinline__ void fixup_body(const TankDev& d, T* __restrict__ y, const T* __restrict__ side, int bx) {
  int gid = bx * blockDim.x + threadIdx.x;
  if (gid >= d.nb * d.nl) return;
  int b = gid / d.nl, ql = gid - b * d.nl;
  // side[b] belongs to the line at x_{c0 + cbb}
  int c0 = b * d.cb;
  int cend = min(c0 + d.cb, d.nx);
  T v = side[(size_t)b * d.nl + ql];
  if (cend < d.nx) {
    y[(int64_t)cend * d.nc + ql] += v;
  } else if (d.periodic) {
    y[ql] += v;
  } else {
    y[(int64_t)d.nx * d.nc + ql] = v;   // the wall line has one contribution
  }
}

template <typename T>
__global__ void k_fixup(const TankDev* __restrict__ td, T* __restrict__ y, const T* __restrict__ side, int flags) {
  const TankDev& d = *td;
  if ((flags & F_GATE) && d.ks->done) return;
  fixup_body<T>(d, y, side, blockIdx.x);
}

// ------------------------------------------------------------ vector kernels
// y = a*x + b*y over [0, n) (optionally masked at surface nodes)
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double bb,
                        double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + bb * y[i];
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

__device__ inline bool is_surface_node(const TankDev& d, int64_t i) {
  int64_t c = i / d.nc;
  int ql = (int)(i - c * d.nc);
  return d.is_surf_loc[ql] != 0;  // the wall line shares the line pattern
}

__global__ void k_mask_surface(const TankDev* __restrict__ td, double* __restrict__ y) {
  const TankDev& d = *td;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.n && is_surface_node(d, i)) y[i] = 0.0;
}

// u = 0 except at the surface nodes, where u = phi_s
__global__ void k_scatter_surface(const TankDev* __restrict__ td, const double* __restrict__ phis,
                                  double* __restrict__ u, int zero_rest) {
  const TankDev& d = *td;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  int64_t c = i / d.nc;
  int ql = (int)(i - c * d.nc);
  if (d.is_surf_loc[ql]) {
    int m;
    if (ql == d.nl - 1) m = 0;
    else {
      m = -1;
      for (int k = 1; k < d.P; ++k)
        if (d.surf_loc[k] == ql) m = k;
    }
    u[i] = phis[c * d.P + m];
  } else if (zero_rest) {
    u[i] = 0.0;
  }
}

__device__ __forceinline__ void gather_surface_body(const TankDev& d, const double* __restrict__ u,
                                                    double* __restrict__ out, int bx) {
  int s = bx * blockDim.x + threadIdx.x;
  if (s >= d.ns) return;
  int c = s / d.P, m = s - c * d.P;
  out[s] = u[(int64_t)c * d.nc + d.surf_loc[m]];
}

__global__ void k_gather_surface(const TankDev* __restrict__ td, const double* __restrict__ u,
                                 double* __restrict__ out) {
  gather_surface_body(*td, u, out, blockIdx.x);
}

// ------------------------------------------------------------ fused reductions
// Partial sums per workgroup (wave butterflies, fixed order), then the last
// workgroup to finish (device-scope counter) adds the partials in block order:
// one launch, deterministic results.
__device__ void givens_update(KrylovState* __restrict__ ks, double* __restrict__ Hbase, int m, int j,
                              double hnorm2, int32_t* __restrict__ status);

// Progress of the current Krylov cycle written to host-visible memory
// (steps done, cycle done, converged) so the host can stop queueing steps
// without synchronising the stream.  A single tank's block also takes the
// scalars the host reports once the solve has converged (scal: residual
// estimate, ||b||, total iterations), written before the word is released.
__device__ inline void publish_progress(const KrylovState* ks, int32_t* mirror, double* scal = nullptr) {
  if (!mirror) return;
  if (scal) {
    scal[0] = ks->resid;
    scal[1] = ks->bnorm;
    scal[2] = (double)ks->iters;
  }
  int32_t v = (ks->j & PROG_STEPS) | (ks->done ? PROG_DONE : 0) | (ks->converged ? PROG_CONV : 0);
  __hip_atomic_store(mirror, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// the scalars of a single tank's progress block (the word, then three doubles)
__device__ inline double* progress_scalars(int32_t* mirror) {
  return mirror ? reinterpret_cast<double*>(mirror) + 1 : nullptr;
}


// The tank sizes the fix-up needs, read once into registers (a loop that
// stores to a vector would otherwise read them again after every store).
struct LineFix {
  int32_t nc = 1, nl = 0, nx = 0, cb = 1, nb = 0, periodic = 0;
  LineFix() = default;
  __device__ explicit LineFix(const TankDev& d)
      : nc(d.nc), nl(d.nl), nx(d.nx), cb(d.cb), nb(d.nb), periodic(d.periodic) {}
};

// Where node i's shared-line contribution is: the side-buffer index (0
// when there is none) and whether it is added (a line shared by two blocks)
// or is the value (the wall line, which has one contribution).  Selects
// only, no branch.
__device__ inline void fix_index(const LineFix& f, int64_t i, int* sidx, bool* add, bool* wall) {
  const int c = (int)(i / f.nc);
  const int ql = (int)(i - (int64_t)c * f.nc);
  const bool line = ql < f.nl;
  const bool wl = line && c == f.nx;
  const bool first = line && !wl && c % f.cb == 0;
  const int blf = c > 0 ? c / f.cb - 1 : (f.periodic ? f.nb - 1 : -1);
  const int bl = wl ? f.nb - 1 : (first ? blf : -1);
  *sidx = (bl >= 0 ? bl : 0) * f.nl + (line ? ql : 0);
  *add = bl >= 0 && !wl;
  *wall = wl;
}
// the fixed-up value from the loaded y[i] and side[sidx]
template <typename T>
__device__ inline T fix_combine(T v, T sv, bool add, bool wall) {
  const T sum = v + (add ? sv : T(0));   // (adding zero leaves v)
  return wall ? sv : sum;
}
// y[i] of an element-kernel output with its shared-line contribution from
// the side buffer added (the fix-up pass, done by the consumer; the same
// addition as the separate pass).  Both loads are issued unconditionally.
template <typename T>
__device__ inline T fixed_value(const LineFix& f, const T* __restrict__ y, const T* __restrict__ side, int64_t i) {
  int sidx;
  bool add, wall;
  fix_index(f, i, &sidx, &add, &wall);
  return fix_combine<T>(y[i], side[sidx], add, wall);
}
template <typename T>
__device__ inline T fixed_value(const TankDev& d, const T* __restrict__ y, const T* __restrict__ side, int64_t i) {
  return fixed_value<T>(LineFix(d), y, side, i);
}

// Workgroup bx: partial products of its chunk into part[bx].  Shared by the
// single-tank kernel (the last workgroup then adds the partials) and the
// batched kernels (a second launch adds them: one device-wide release per
// workgroup is cheap for a few hundred workgroups, not for tens of thousands).
template <typename T>
__device__ __forceinline__ void dots_partial(int64_t n, int nvec, const T* __restrict__ X, int64_t ldx,
                                             T* __restrict__ w, double* __restrict__ part, int ldp, int64_t chunk,
                                             const TankDev* __restrict__ fixd, const T* __restrict__ side, int bx) {
  __shared__ double red[4][kMaxVec];
  const int64_t lo = (int64_t)bx * chunk, hi = min(lo + chunk, n);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // eight vectors per pass, their loads issued together (clamped indices,
  // zero weights past nvec keep the loads unconditional)
  for (int k0 = 0; k0 < nvec; k0 += 8) {
    double sacc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sacc[u] = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      T wt;
      if (fixd && k0 == 0) {
        // w is an operator output whose shared-line contributions are still
        // in the side buffer: the fix-up of this node, kept for the later
        // passes (same thread)
        wt = fixed_value<T>(*fixd, w, side, i);
        const int64_t c = i / fixd->nc;
        if (i - c * fixd->nc < fixd->nl) w[i] = wt;
      } else {
        wt = w[i];
      }
      const double wi = (double)wt;
      T xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = X[(int64_t)min(k0 + u, nvec - 1) * ldx + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) sacc[u] += (double)xv[u] * wi;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double t = wave_sum(sacc[u]);
      if (lane == 0 && k0 + u < nvec) red[wv][k0 + u] = t;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nvec; k += blockDim.x)
    part[(size_t)bx * ldp + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}

// Workgroup bx's part of sum_i v_i^2 over its chunk for values the caller
// forms per node (value(i), which may also store them), in the order of
// dots_partial with X = w: thread-strided sums, wave butterflies, the four
// wave totals in order.
template <typename F>
__device__ __forceinline__ void self_dot_partial(int64_t n, int64_t chunk, int bx, double* __restrict__ part, int ldp,
                                                 F value) {
  __shared__ double red[4];
  const int64_t lo = (int64_t)bx * chunk, hi = min(lo + chunk, n);
  double sacc = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double v = value(i);
    sacc += v * v;
  }
  sacc = wave_sum(sacc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sacc;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)bx * ldp] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_dots_fused(int64_t n, int nvec, const T* __restrict__ X, int64_t ldx, T* __restrict__ w,
             double* __restrict__ part, int ldp, double* __restrict__ out, int64_t chunk,
             int32_t* __restrict__ counter, const KrylovState* __restrict__ gate,
             const TankDev* __restrict__ fixd, const T* __restrict__ side) {
  if (gate && gate->done) return;
  dots_partial<T>(n, nvec, X, ldx, w, part, ldp, chunk, fixd, side, blockIdx.x);
  if (!last_block(counter, gridDim.x)) return;
  dots_reduce(nvec, part, ldp, out, gridDim.x);
  if (threadIdx.x == 0) *counter = 0;
}

// w' = w - sum_{i<=j} h_i V_i, and this workgroup's part of ||w'||^2
// (fixd: w is an operator output whose shared-line contributions are still
// in the side buffer, added as it is read).  A thread takes its entries two
// at a time, their loads requested together (clamped addresses); its sum
// runs over its entries in order.
template <typename T, bool FIX>
__device__ __forceinline__ void orth_partial_t(int64_t n, int j, const T* __restrict__ V,
                                               const double* __restrict__ Hbase, int m, T* __restrict__ w,
                                               double* __restrict__ part, int ldp, int64_t chunk, int bx,
                                               const TankDev* __restrict__ fixd, const T* __restrict__ side) {
  constexpr int U = 2;
  __shared__ double red[4];
  const double* hcol = Hbase + (size_t)j * (m + 1);
  const int64_t lo = (int64_t)bx * chunk, hi = min(lo + chunk, n);
  constexpr bool fix = FIX;
  const LineFix lf = FIX ? LineFix(*fixd) : LineFix();
  double sacc = 0;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (int64_t)U * blockDim.x) {
    // the entries' indices, then all their loads, then the arithmetic
    int64_t ii[U];
    int sidx[U];
    bool add[U], wall[U];
#pragma unroll
    for (int e = 0; e < U; ++e) {
      ii[e] = min(i0 + (int64_t)e * blockDim.x, hi - 1);
      if constexpr (fix) fix_index(lf, ii[e], &sidx[e], &add[e], &wall[e]);
    }
    T wv[U], sv[U];
#pragma unroll
    for (int e = 0; e < U; ++e) {
      wv[e] = w[ii[e]];
      if constexpr (fix) sv[e] = side[sidx[e]];
    }
    double v[U];
#pragma unroll
    for (int e = 0; e < U; ++e) v[e] = fix ? (double)fix_combine<T>(wv[e], sv[e], add[e], wall[e]) : (double)wv[e];
    for (int k0 = 0; k0 <= j; k0 += 8) {
      T vv[U][8];
#pragma unroll
      for (int e = 0; e < U; ++e)
#pragma unroll
        for (int u = 0; u < 8; ++u) vv[e][u] = V[(int64_t)min(k0 + u, j) * n + ii[e]];
      // (h read from clamped indices and the update selected: a branch per
      // vector would wait for each h on its own)
      double hk[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) hk[u] = hcol[min(k0 + u, j)];
#pragma unroll
      for (int e = 0; e < U; ++e)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double t = v[e] - hk[u] * (double)vv[e][u];
          v[e] = k0 + u <= j ? t : v[e];
        }
    }
#pragma unroll
    for (int e = 0; e < U; ++e) {
      if (i0 + (int64_t)e * blockDim.x < hi) {
        const T vt = T(v[e]);
        w[ii[e]] = vt;
        sacc += (double)vt * (double)vt;
      }
    }
  }
  sacc = wave_sum(sacc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sacc;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)bx * ldp] = ((red[0] + red[1]) + red[2]) + red[3];
}
template <typename T>
__device__ __forceinline__ void orth_partial(int64_t n, int j, const T* __restrict__ V,
                                             const double* __restrict__ Hbase, int m, T* __restrict__ w,
                                             double* __restrict__ part, int ldp, int64_t chunk, int bx,
                                             const TankDev* __restrict__ fixd = nullptr,
                                             const T* __restrict__ side = nullptr) {
  if (fixd) orth_partial_t<T, true>(n, j, V, Hbase, m, w, part, ldp, chunk, bx, fixd, side);
  else orth_partial_t<T, false>(n, j, V, Hbase, m, w, part, ldp, chunk, bx, fixd, side);
}

// ||w'||^2 from nblk partials (first wave), then the Givens update of column j
__device__ __forceinline__ void orth_reduce(int j, const double* __restrict__ part, int ldp, int nblk,
                                            KrylovState* __restrict__ ks, double* __restrict__ Hbase, int m,
                                            int32_t* __restrict__ status, int32_t* __restrict__ mirror,
                                            double* __restrict__ smirror = nullptr) {
  if (threadIdx.x < 64) {
    double t = lane_partials(part, ldp, 0, nblk, threadIdx.x);
    t = wave_sum(t);
    if (threadIdx.x == 0) {
      givens_update(ks, Hbase, m, j, t, status);
      publish_progress(ks, mirror, smirror);
    }
  }
}

// w' = w - sum_{i<=j} h_i V_i; ||w'||^2 reduced; Givens update of column j
template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_orth_fused(int64_t n, int j, const T* __restrict__ V, double* __restrict__ Hbase, int m, T* __restrict__ w,
             double* __restrict__ part, int ldp, int64_t chunk, KrylovState* __restrict__ ks,
             int32_t* __restrict__ counter, int32_t* __restrict__ status, int32_t* __restrict__ mirror,
             const TankDev* __restrict__ fixd, const T* __restrict__ side) {
  if (ks->done) return;
  orth_partial<T>(n, j, V, Hbase, m, w, part, ldp, chunk, blockIdx.x, fixd, side);
  if (!last_block(counter, gridDim.x)) return;
  if (threadIdx.x == 0) *counter = 0;
  orth_reduce(j, part, ldp, gridDim.x, ks, Hbase, m, status, mirror, progress_scalars(mirror));
}

// ------------------------------------------------------------ GMRES pieces
// Givens update of Hessenberg column j (one thread).  The column holds
// h_{0..j}; hnorm2 = ||w'||^2.  Sets done/converged and the norm of V_{j+1}.
__device__ void givens_update(KrylovState* __restrict__ ks, double* __restrict__ Hbase, int m, int j,
                              double hnorm2, int32_t* __restrict__ status) {
  if (ks->done) return;
  double* H = Hbase;                       // (m+1) x m, column-major: H[i + j*(m+1)]
  double* cs = Hbase + (m + 1) * m;
  double* sn = cs + m;
  double* g = sn + m;
  double* col = H + (size_t)j * (m + 1);
  double hn = sqrt(fmax(hnorm2, 0.0));
  col[j + 1] = hn;
  // the previous rotations applied to the column in order, the running entry
  // in a register; their operands requested eight at a time from clamped
  // addresses (one round trip per eight rotations, not one per rotation)
  double ci = col[0];
  for (int i0 = 0; i0 < j; i0 += 8) {
    double c8[8], s8[8], h8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = min(i0 + u, j - 1);
      c8[u] = cs[i];
      s8[u] = sn[i];
      h8[u] = col[i + 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (i0 + u < j) {
        const double t = c8[u] * ci + s8[u] * h8[u];
        ci = -s8[u] * ci + c8[u] * h8[u];
        col[i0 + u] = t;
      }
    }
  }
  col[j] = ci;
  double den = hypot(col[j], col[j + 1]);
  if (!(den > 0.0) || !finite(den)) {
    atomicOr(status, finite(den) ? ST_BREAKDOWN : ST_NONFINITE);
    ks->done = 1;
    ks->status |= finite(den) ? ST_BREAKDOWN : ST_NONFINITE;
    return;
  }
  cs[j] = col[j] / den;
  sn[j] = col[j + 1] / den;
  col[j] = den;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  ks->j = j + 1;
  ks->iters += 1;
  ks->resid = fabs(g[j + 1]);
  if (ks->resid <= ks->rtol * ks->bnorm) {
    ks->converged = 1;
    ks->done = 1;
  } else if (j + 1 >= m) {
    ks->done = 1;
  }
  // store the normalisation of V_{j+1}
  g[m + 1 + j] = hn;  // y[] area reused as scratch for the norms
}

// V_{j+1} = w' / hn
template <typename T>
__global__ void k_scale_next(int64_t n, int j, const T* __restrict__ w, T* __restrict__ V,
                             const double* __restrict__ Hbase, int m, const KrylovState* __restrict__ ks) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // independent loads first, then the test
  const double* g = Hbase + (m + 1) * m + 2 * m;
  const double hn = g[m + 1 + j];
  const double wi = (double)w[i];
  if (ks->converged) return;
  if (j + 1 < m + 1) V[(int64_t)(j + 1) * n + i] = (hn > 0.0) ? T(wi / hn) : T(0);
}

// start of a cycle: r is in V_0 (masked); beta = sqrt(rr); V_0 = r/beta; g = (beta, 0, ...)
__device__ void cycle_start(KrylovState* __restrict__ ks, double* __restrict__ Hbase, int m,
                            const double* __restrict__ rr, int first, int32_t* __restrict__ status);

__device__ void cycle_start(KrylovState* __restrict__ ks, double* __restrict__ Hbase, int m,
                            const double* __restrict__ rr, int first, int32_t* __restrict__ status) {
  double beta = sqrt(fmax(rr[0], 0.0));
  if (first) {
    ks->bnorm = sqrt(fmax(rr[1], 0.0));
    if (ks->bnorm == 0.0) ks->bnorm = beta;  // zero right side: relative to the first residual
  }
  if (!finite(beta) || !finite(ks->bnorm)) {
    atomicOr(status, ST_NONFINITE);
    ks->status |= ST_NONFINITE;
    ks->done = 1;
    ks->converged = 0;
    return;
  }
  ks->beta = beta;
  ks->resid = beta;
  ks->j = 0;
  double* g = Hbase + (m + 1) * m + 2 * m;
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = beta;
  if (beta <= ks->rtol * ks->bnorm) {
    ks->converged = 1;
    ks->done = 1;
  } else {
    ks->done = 0;
  }
}

template <typename T>
__global__ void k_scale_v0(int64_t n, T* __restrict__ V, const KrylovState* __restrict__ ks) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || ks->done) return;
  V[i] = T((double)V[i] / ks->beta);
}

// r = b - y (masked at the surface for the Laplace problem)
template <typename T>
__global__ void k_residual(const TankDev* __restrict__ td, int64_t n, const T* __restrict__ bvec,
                           const T* __restrict__ y, T* __restrict__ r, int mask) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T v = bvec[i] - y[i];
  if (mask && is_surface_node(*td, i)) v = T(0);
  r[i] = v;
}

// Start of a Krylov cycle in one launch: r = b - y (y's fix-up folded in,
// masked at the surface) into V_0, ||r||^2 into rr[0], and in the last
// workgroup the cycle start (beta, the Givens right side, convergence at
// once) and its progress word.  The values of the separate residual, inner
// product and cycle-start kernels.
template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_residual_cycle(const TankDev* __restrict__ td, int64_t n, T* __restrict__ bvec, const T* __restrict__ y,
                 const T* __restrict__ side, T* __restrict__ r, int mask, double* __restrict__ part, int ldp,
                 double* __restrict__ rr, int64_t chunk, int32_t* __restrict__ counter, KrylovState* __restrict__ ks,
                 double* __restrict__ Hbase, int m, int first, int32_t* __restrict__ status,
                 int32_t* __restrict__ mirror, const T* __restrict__ bside) {
  const TankDev& d = *td;
  if (bside) {
    // b's own shared-line fix-up (its contributions in bside) in the same
    // pass, kept in b, and ||b||^2 into rr[1] beside ||r||^2 (each sum in the
    // order of the separate fix-up-and-norm kernel)
    __shared__ double red2[2][4];
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(lo + chunk, n);
    double s0 = 0, s1 = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const T bf = fixed_value<T>(d, bvec, bside, i);
      bvec[i] = bf;
      T v = bf - fixed_value<T>(d, y, side, i);
      if (mask && is_surface_node(d, i)) v = T(0);
      r[i] = v;
      const double dv = (double)v, db = (double)bf;
      s0 += dv * dv;
      s1 += db * db;
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if ((threadIdx.x & 63) == 0) {
      red2[0][threadIdx.x >> 6] = s0;
      red2[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      part[(size_t)blockIdx.x * ldp] = ((red2[0][0] + red2[0][1]) + red2[0][2]) + red2[0][3];
      part[(size_t)blockIdx.x * ldp + 1] = ((red2[1][0] + red2[1][1]) + red2[1][2]) + red2[1][3];
    }
  } else {
    self_dot_partial(n, chunk, blockIdx.x, part, ldp, [&](int64_t i) {
      T v = bvec[i] - fixed_value<T>(d, y, side, i);
      if (mask && is_surface_node(d, i)) v = T(0);
      r[i] = v;
      return (double)v;
    });
  }
  if (!last_block(counter, gridDim.x)) return;
  dots_reduce(bside ? 2 : 1, part, ldp, rr, gridDim.x);
  if (bside) __syncthreads();   // rr[1] comes from the second wave
  if (threadIdx.x == 0) {
    *counter = 0;
    if (*status) {
      // a status set before the cycle (a non-positive water column found by
      // the coefficient update, a non-finite value) ends the solve at once
      ks->status |= *status;
      ks->done = 1;
      ks->converged = 0;
    } else {
      cycle_start(ks, Hbase, m, rr, first, status);
    }
    publish_progress(ks, mirror, progress_scalars(mirror));
  }
}

// End of a Krylov cycle in one launch: every workgroup solves the small
// triangular system for y (one thread, the order of the separate solve) and
// then updates its part of x += Z y.
__device__ inline const double* hist_slot(const TankDev& d, int stage, const StageHistory& hs, int back);
__device__ inline int64_t surface_slot(const TankDev& d, int64_t i);

// td set (FP64, the solve's last cycle): the end of the Laplace solve in the
// same pass, the values of k_solve_end (x is the tank's xs)
template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_solve_update(int64_t n, const T* __restrict__ Z, const double* __restrict__ Hbase, int m,
               const KrylovState* __restrict__ ks, T* __restrict__ x, const TankDev* __restrict__ td,
               const double* __restrict__ phis, double* __restrict__ phi, int stage) {
  __shared__ double ys[kMaxRestart];
  // the triangle of H (column k: rows 0 .. k, from index k (k + 1) / 2) and
  // g, staged by the workgroup (every load requested before its store), so
  // that the back-substitution reads LDS instead of one global round trip
  // per entry
  __shared__ double ht[kMaxRestart * (kMaxRestart + 1) / 2];
  __shared__ double gs[kMaxRestart];
  const int jn = ks->j;
  {
    const double* H = Hbase;
    const double* g = Hbase + (m + 1) * m + 2 * m;
    constexpr int kU = 4;
    for (int t0 = threadIdx.x; t0 < jn * jn; t0 += kU * kBlockThreads) {
      double hv[kU];
#pragma unroll
      for (int e = 0; e < kU; ++e) {
        const int t = min(t0 + e * kBlockThreads, jn * jn - 1), k = t / jn, i = t - k * jn;
        hv[e] = H[(size_t)k * (m + 1) + i];
      }
#pragma unroll
      for (int e = 0; e < kU; ++e) {
        const int t = t0 + e * kBlockThreads, k = t / jn, i = t - k * jn;
        if (t < jn * jn && i <= k) ht[k * (k + 1) / 2 + i] = hv[e];
      }
    }
    if ((int)threadIdx.x < jn) gs[threadIdx.x] = g[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = jn - 1; i >= 0; --i) {
      double sacc = gs[i];
      for (int k = i + 1; k < jn; ++k) sacc -= ht[k * (k + 1) / 2 + i] * ys[k];
      ys[i] = sacc / ht[i * (i + 1) / 2 + i];
    }
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = x[i];
  for (int k0 = 0; k0 < jn; k0 += 8) {
    T zz[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) zz[u] = Z[(int64_t)min(k0 + u, jn - 1) * n + i];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < jn) v += ys[k0 + u] * (double)zz[u];
  }
  x[i] = T(v);
  if (td) {
    const TankDev& d = *td;
    const int64_t sl = surface_slot(d, i);
    const double pv = sl >= 0 ? phis[sl] : (double)T(v);
    phi[i] = pv;
    if (stage >= 0) const_cast<double*>(hist_slot(d, stage, *d.hs, 0))[i] = pv - d.pv[i];
  }
}

// r32 = (float)(r * scale)
__global__ void k_to_float(int64_t n, const double* __restrict__ r, double scale, float* __restrict__ r32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r32[i] = (float)(r[i] * scale);
}

// x += scale * x32
__global__ void k_add_float(int64_t n, const float* __restrict__ x32, double scale, double* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += scale * (double)x32[i];
}

// ------------------------------------------------------------ batched Krylov steps
// products of nvec vectors (from X, stride n) with w; out = H column hcol,
// or the tank's scalars from index sidx when hcol < 0
template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_dots_b(BatchArgs ba, int nvec, VSel X, VSel w, int fix, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  dots_partial<T>(d.n, nvec, bvec<T>(d, X), d.n, bvec<T>(d, w), d.part, d.m + 2, dot_chunk(d.n),
                  fix ? &d : nullptr, fix ? reinterpret_cast<const T*>(d.side) : nullptr, it_.bx);
}

// one workgroup per tank: out = H column hcol, or the scalars from sidx when hcol < 0
__global__ void __launch_bounds__(kBlockThreads) k_dots_sum_b(BatchArgs ba, int nvec, int hcol, int sidx, int gate) {
  SEM_BATCH_TANK(ba)
  if (gate && d.ks->done) return;
  double* out = hcol >= 0 ? d.H + (size_t)hcol * (d.m + 1) : d.scal + sidx;
  dots_reduce(nvec, d.part, d.m + 2, out, dot_nchunk(d.n));
}

// the products of a stiffness output (before its fix-up) with V_0 ..
// V_{nvec-1}, per stiffness block as the single-tank stiffness launch forms
// them: item (tank, first block bx, blocks by)
template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_dots_blocks_b(BatchArgs ba, int nvec) {
  SEM_BATCH_TANK(ba)
  if (d.ks->done) return;
  const T* y = bvec<T>(d, VSel{BV_W, 0});
  const T* V = bvec<T>(d, VSel{BV_V, 0});
  for (int b = it_.bx; b < min(it_.bx + it_.by, d.nb); ++b)
    block_dots_part<T>(d.cb, d.nx, d.nc, d.nl, d.periodic, y, reinterpret_cast<const T*>(d.side), V, d.n, nvec,
                       d.part, d.m + 2, b);
}

// one workgroup per tank: the products' sums from the per-block partials
// into H column hcol
__global__ void __launch_bounds__(kBlockThreads) k_dots_sum_blocks_b(BatchArgs ba, int nvec, int hcol) {
  SEM_BATCH_TANK(ba)
  if (d.ks->done) return;
  dots_reduce(nvec, d.part, d.m + 2, d.H + (size_t)hcol * (d.m + 1), d.nb);
}

// fix: w's shared-line contributions are still in the side buffer
template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_orth_b(BatchArgs ba, int j, int fix) {
  SEM_BATCH_TANK(ba)
  if (d.ks->done) return;
  orth_partial<T>(d.n, j, bvec<T>(d, VSel{BV_V, 0}), d.H, d.m, bvec<T>(d, VSel{BV_W, 0}), d.part, d.m + 2,
                  dot_chunk(d.n), it_.bx, fix ? &d : nullptr, fix ? reinterpret_cast<const T*>(d.side) : nullptr);
}

__global__ void __launch_bounds__(kBlockThreads) k_orth_sum_b(BatchArgs ba, int j) {
  SEM_BATCH_TANK(ba)
  if (d.ks->done) return;
  orth_reduce(j, d.part, d.m + 2, dot_nchunk(d.n), d.ks, d.H, d.m, d.status, d.prog);
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_fixup_b(BatchArgs ba, VSel y, int flags) {
  SEM_BATCH_TANK(ba)
  if ((flags & F_GATE) && d.ks->done) return;
  fixup_body<T>(d, bvec<T>(d, y), reinterpret_cast<const T*>(d.side), it_.bx);
}

template <typename T>
// (ysel = BV_NONE: y = A x for x = 0, exactly zero, is not read)
__global__ void __launch_bounds__(kBlockThreads) k_residual_b(BatchArgs ba, VSel bsel, VSel ysel, VSel rsel) {
  SEM_BATCH_TANK(ba)
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const T* bv = bvec<T>(d, bsel);
  T v = bv[i];
  if (ysel.kind != BV_NONE) v -= bvec<T>(d, ysel)[i];
  if (is_surface_node(d, i)) v = T(0);
  bvec<T>(d, rsel)[i] = v;
}

// a tank whose status word is already set (e.g. a non-positive water column
// found by the coefficient update) ends its solve at once
__global__ void k_cycle_start_b(BatchArgs ba, int first) {
  SEM_BATCH_TANK(ba)
  if (threadIdx.x != 0) return;
  if (*d.status) {
    d.ks->done = 1;
    d.ks->converged = 0;
    d.ks->status |= *d.status;
  } else {
    cycle_start(d.ks, d.H, d.m, d.scal, first, d.status);
  }
  publish_progress(d.ks, d.prog);
}

// fresh Krylov state (including the reductions' completion counter)
// rtol_t (optional): a tolerance per tank
__global__ void k_ks_init_b(BatchArgs ba, double rtol, const double* __restrict__ rtol_t) {
  SEM_BATCH_TANK(ba)
  if (threadIdx.x != 0) return;
  KrylovState k{};
  k.rtol = rtol_t ? rtol_t[it_.tank] : rtol;
  *d.ks = k;
}

__global__ void k_status_clear_b(BatchArgs ba, int) {
  SEM_BATCH_TANK(ba)
  if (threadIdx.x == 0) *d.status = 0;
}

// end of a solve: unconverged tanks get the no-convergence bit; the Krylov
// states and status words are copied to host-visible memory
__global__ void k_state_out_b(BatchArgs ba, KrylovState* __restrict__ ks_out, int32_t* __restrict__ st_out,
                              int mark_noconv) {
  SEM_BATCH_TANK(ba)
  if (threadIdx.x != 0) return;
  const KrylovState k = *d.ks;
  int32_t w = *d.status;
  if (mark_noconv && !k.converged && !w) {
    w |= ST_NOCONV;
    *d.status = w;
  }
  ks_out[it_.tank] = k;
  st_out[it_.tank] = w;
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_scale_v0_b(BatchArgs ba, int) {
  SEM_BATCH_TANK(ba)
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= d.n || d.ks->done) return;
  T* V = bvec<T>(d, VSel{BV_V, 0});
  V[i] = T((double)V[i] / d.ks->beta);
}

__global__ void k_solve_y_b(BatchArgs ba, int) {
  SEM_BATCH_TANK(ba)
  if (threadIdx.x != 0) return;
  const int m = d.m;
  const int jn = d.ks->j;
  const double* H = d.H;
  const double* g = d.H + (m + 1) * m + 2 * m;
  double* y = d.H + (m + 1) * m + 2 * m + (m + 1) + m;
  for (int i = jn - 1; i >= 0; --i) {
    double sacc = g[i];
    for (int k = i + 1; k < jn; ++k) sacc -= H[(size_t)k * (m + 1) + i] * y[k];
    y[i] = sacc / H[(size_t)i * (m + 1) + i];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_update_x_b(BatchArgs ba, VSel xsel) {
  SEM_BATCH_TANK(ba)
  const int64_t n = d.n;
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = d.m;
  const double* y = d.H + (m + 1) * m + 2 * m + (m + 1) + m;
  const T* Z = bvec<T>(d, VSel{BV_Z, 0});
  T* x = bvec<T>(d, xsel);
  const int jn = d.ks->j;
  double v = x[i];
  for (int k0 = 0; k0 < jn; k0 += 8) {
    T zz[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) zz[u] = Z[(int64_t)min(k0 + u, jn - 1) * n + i];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < jn) v += y[k0 + u] * (double)zz[u];
  }
  x[i] = T(v);
}

// the tank's scalar idx to host-visible memory
__global__ void k_scal_out_b(BatchArgs ba, int idx, double* __restrict__ out) {
  SEM_BATCH_TANK(ba)
  if (threadIdx.x == 0) out[it_.tank] = d.scal[idx];
}

// refinement: b32 = (float)(tmp * scale[tank]), x32 = 0
__global__ void __launch_bounds__(kBlockThreads) k_to_float_b(BatchArgs ba, const double* __restrict__ scale) {
  SEM_BATCH_TANK(ba)
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  d.b32[i] = (float)(d.tmp[i] * scale[it_.tank]);
  d.x32[i] = 0.0f;
}

// refinement: xs += scale[tank] * x32
__global__ void __launch_bounds__(kBlockThreads) k_add_float_b(BatchArgs ba, const double* __restrict__ scale) {
  SEM_BATCH_TANK(ba)
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  d.xs[i] += scale[it_.tank] * (double)d.x32[i];
}

__global__ void k_status_or_b(BatchArgs ba, int bits) {
  SEM_BATCH_TANK(ba)
  if (threadIdx.x == 0) atomicOr(d.status, bits);
}

// surface value of node i (x-ordered surface array phis), or -1 when i is
// not a surface node
__device__ inline int64_t surface_slot(const TankDev& d, int64_t i) {
  const int64_t c = i / d.nc;
  const int ql = (int)(i - c * d.nc);
  if (!d.is_surf_loc[ql]) return -1;
  int m = 0;
  if (ql != d.nl - 1) {
    for (int k = 1; k < d.P; ++k)
      if (d.surf_loc[k] == ql) m = k;
  }
  return c * d.P + m;
}

// u = [0; phi~] (the lift's input) in the tank's tmp vector, and the start
// vector xs = guess (masked at the surface) or 0
__global__ void __launch_bounds__(kBlockThreads)
k_lift_in_b(BatchArgs ba, const double* const* __restrict__ phis, const double* const* __restrict__ guess) {
  SEM_BATCH_TANK(ba)
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int64_t sl = surface_slot(d, i);
  const double* ps = phis[it_.tank];
  const double* gs = guess ? guess[it_.tank] : nullptr;
  d.tmp[i] = sl >= 0 ? ps[sl] : 0.0;
  d.xs[i] = (sl >= 0 || !gs) ? 0.0 : gs[i];
}

// Phi = xs with the surface values put back
__global__ void __launch_bounds__(kBlockThreads)
k_solution_out_b(BatchArgs ba, const double* const* __restrict__ phis, double* const* __restrict__ phi) {
  SEM_BATCH_TANK(ba)
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int64_t sl = surface_slot(d, i);
  phi[it_.tank][i] = sl >= 0 ? phis[it_.tank][sl] : d.xs[i];
}

// ------------------------------------------------------------ stage predictor
// Initial guess of RK4 stage k's Laplace solve.  The solve starts from the
// previous stage's solution p; the guess adds the change from the previous
// stage to stage k, extrapolated over the last steps (the same stage of
// steps n-1, n-2, ...: D1, D2, ...) by the polynomial through the available
// depth q: sum_m (-1)^(m+1) C(q, m) D_m (D1; 2 D1 - D2; 3 D1 - 3 D2 + D3;
// ...).  Stage 0's change in a step needs the last stage of the step before,
// so its record starts one step later.  Only the starting vector changes;
// the solve's stopping test does not.
__device__ inline int predict_depth(const StageHistory& hs, int stage, int maxdepth, double dt) {
  if (hs.dt != dt) return 0;
  const int dep = stage == 0 ? hs.valid - 1 : hs.valid;
  return max(0, min(dep, maxdepth));
}
// the record of stage k, `back` steps before the current one (0: the current step's slot)
__device__ inline const double* hist_slot(const TankDev& d, int stage, const StageHistory& hs, int back) {
  const int r = (hs.slot - back + kHistSteps) % kHistSteps;
  return d.hist + ((size_t)stage * kHistSteps + (size_t)r) * d.n;
}

// the extrapolated change at node i for depth dep >= 1 (terms added in the
// order m = 1, 2, ...; the records are loaded together)
__device__ inline double predict_increment(const TankDev& d, const StageHistory& hs, int stage, int dep, int64_t i) {
  // signed binomial weights (-1)^(m+1) C(q, m), row q - 1
  constexpr double kW[kHistSteps][kHistSteps] = {{1, 0, 0, 0, 0, 0},         {2, -1, 0, 0, 0, 0},
                                                  {3, -3, 1, 0, 0, 0},        {4, -6, 4, -1, 0, 0},
                                                  {5, -10, 10, -5, 1, 0},     {6, -15, 20, -15, 6, -1}};
  double dm[kHistSteps];
#pragma unroll
  for (int m = 0; m < kHistSteps; ++m) dm[m] = m < dep ? hist_slot(d, stage, hs, m + 1)[i] : 0.0;
  double e = dm[0] * kW[dep - 1][0];
#pragma unroll
  for (int m = 1; m < kHistSteps; ++m)
    if (m < dep) e += kW[dep - 1][m] * dm[m];
  return e;
}

__device__ __forceinline__ void predict_body(const TankDev& d, int stage, int maxdepth, double dt,
                                             double* __restrict__ ws, int64_t i) {
  const StageHistory hs = *d.hs;
  const int dep = predict_depth(hs, stage, maxdepth, dt);
  const double p = ws[i];
  d.pv[i] = p;
  if (dep > 0) ws[i] = p + predict_increment(d, hs, stage, dep, i);
}

// after stage k's solve: its change from the starting vector, into this step's slot
__device__ __forceinline__ void history_body(const TankDev& d, int stage, const double* __restrict__ ws, int64_t i) {
  double* slot = const_cast<double*>(hist_slot(d, stage, *d.hs, 0));
  slot[i] = ws[i] - d.pv[i];
}

// Start of a single-tank Laplace solve, one pass: u = [0; phi~] (the lift's
// input); the start vector xs = 0 at the surface and elsewhere the warm-start
// vector ws (none: 0), plus the extrapolated change when stage >= 0 (ws
// itself is kept as the stage's starting vector); the Krylov state reset
// (init_ks).  Values as the separate passes give them.
__global__ void __launch_bounds__(kBlockThreads)
k_solve_begin(const TankDev* __restrict__ td, const double* __restrict__ phis, double* __restrict__ u,
              const double* __restrict__ ws, int stage, int maxdepth, double dt, double rtol, int init_ks) {
  const TankDev& d = *td;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (init_ks && i == 0) {
    KrylovState k0{};
    k0.rtol = rtol;
    *d.ks = k0;
  }
  if (i >= d.n) return;
  const int64_t sl = surface_slot(d, i);
  u[i] = sl >= 0 ? phis[sl] : 0.0;
  double g = 0.0;
  if (ws) {
    const double p = ws[i];
    g = p;
    if (stage >= 0) {
      const StageHistory hs = *d.hs;
      const int dep = predict_depth(hs, stage, maxdepth, dt);
      d.pv[i] = p;
      if (dep > 0) g = p + predict_increment(d, hs, stage, dep, i);
    }
  }
  d.xs[i] = sl >= 0 ? 0.0 : g;
}

// End of a single-tank Laplace solve: Phi = xs with the surface values put
// back; for a stage solve (stage >= 0) the change from the stage's starting
// vector into this step's record.
__global__ void __launch_bounds__(kBlockThreads)
k_solve_end(const TankDev* __restrict__ td, const double* __restrict__ phis, double* __restrict__ phi, int stage) {
  const TankDev& d = *td;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int64_t sl = surface_slot(d, i);
  const double v = sl >= 0 ? phis[sl] : d.xs[i];
  phi[i] = v;
  if (stage >= 0) const_cast<double*>(hist_slot(d, stage, *d.hs, 0))[i] = v - d.pv[i];
}

__global__ void __launch_bounds__(kBlockThreads)
k_predict_b(BatchArgs ba, int stage, int maxdepth, const double* __restrict__ dt, int table) {
  SEM_BATCH_TANK(ba)
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  predict_body(d, stage, maxdepth, dt[it_.tank], const_cast<double*>(ba.ptrs[(size_t)table * ba.count + it_.tank]), i);
}

__global__ void __launch_bounds__(kBlockThreads) k_history_b(BatchArgs ba, int stage, int table) {
  SEM_BATCH_TANK(ba)
  const int64_t i = (int64_t)it_.bx * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  history_body(d, stage, ba.ptrs[(size_t)table * ba.count + it_.tank], i);
}

// ------------------------------------------------------------ 1D surface work
// One workgroup per tank.  1D element e (column) holds surface nodes
// e*P + k, k = 0..P (wrapped when periodic).
__device__ inline int s_index(const TankDev& d, int e, int k) {
  int s = e * d.P + k;
  return s >= d.ns ? s - d.ns : s;
}

// ------------------------------------------------------------ 1D projections as exact rows
// y = A x for A = M'^{-1} S_x or M'^{-1}.  Periodic: A is block-circulant,
// given by its first block-row [P][nx P]: y[eP + a] = sum_j row[a][j]
// x[(eP + j) mod nx P], j within the row's decay band (circ_band elements
// each side, below rounding beyond).  Walls: the same rows for the nodes
// farther than the band from both walls, explicit rows for the others.  One
// wavefront per output node: lanes stride over j, then a butterfly sum
// (fixed order).  x1/y1, when given, is a second vector with the same operator.
__device__ __forceinline__ void circ_body(const TankDev& d, int which, const double* __restrict__ x0,
                                          double* __restrict__ y0, const double* __restrict__ x1,
                                          double* __restrict__ y1, int bx) {
  const int s = bx * (kBlockThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= d.ns) return;
  const int P = d.P, ns = d.ns;
  const int e = s / P, a = s - e * P;
  double acc0 = 0, acc1 = 0;
  int rr = -1, t0 = 0;   // walls: explicit row near a wall and its window start
  if (!d.periodic) {
    if (s < d.wall_nl) {
      rr = s;
    } else if (s >= ns - d.wall_nr) {
      rr = d.wall_nl + (s - (ns - d.wall_nr));
      t0 = ns - d.wall_wd;
    }
  }
  if (rr >= 0) {
    const double* row = d.wrows + ((size_t)(which == 0 ? 0 : 1) * (d.wall_nl + d.wall_nr) + rr) * d.wall_wd;
    for (int t = lane; t < d.wall_wd; t += 64) {
      const double r = row[t];
      acc0 += r * x0[t0 + t];
      if (x1) acc1 += r * x1[t0 + t];
    }
  } else {
    // the periodic row (nodes per row: nxp = nx P); its band: elements
    // nx - band .. nx - 1, 0 .. band (or the whole row).  With walls the
    // node is at least band + 1 elements from both walls: no wrap.
    const int nxp = d.nx * P;
    const double* row = (which == 0 ? d.Rrow : d.Brow) + (size_t)a * ns;
    const int base = e * P;
    const bool all = 2 * d.circ_band + 1 >= d.nx;
    const int span = all ? nxp : (2 * d.circ_band + 1) * P;
    const int j0 = all ? 0 : (d.nx - d.circ_band) * P;
    for (int t = lane; t < span; t += 64) {
      int j = j0 + t;
      if (j >= nxp) j -= nxp;
      int src = d.periodic ? base + j : base - d.circ_band * P + t;
      if (src >= nxp && d.periodic) src -= nxp;
      double r = row[j];
      acc0 += r * x0[src];
      if (x1) acc1 += r * x1[src];
    }
  }
  acc0 = wave_sum(acc0);
  if (x1) acc1 = wave_sum(acc1);
  if (lane == 0) {
    y0[s] = acc0;
    if (x1) y1[s] = acc1;
  }
}

__global__ void __launch_bounds__(kBlockThreads)
k_circ_apply(const TankDev* __restrict__ td, int which, const double* __restrict__ x0, double* __restrict__ y0,
             const double* __restrict__ x1, double* __restrict__ y1) {
  circ_body(*td, which, x0, y0, x1, y1, blockIdx.x);
}

// Over-integrated element right-hand sides (Secs. 3.1.1, 3.3): loc[e][i][2]
// = J_e (I^T M_f F)_i for F_eta and F_phi.  One wavefront per element: the
// fluxes at the P_f+1 fine nodes, their mass-weighted sums, then the
// projection back onto the P+1 element nodes.
__device__ __forceinline__ void fs_local_body(const TankDev& d, const double* __restrict__ eta,
                                              const double* __restrict__ etax, const double* __restrict__ phix,
                                              const double* __restrict__ ws, double* __restrict__ loc, int bx) {
  constexpr int kW = kBlockThreads / 64;
  __shared__ double fl[kW][2][64];
  __shared__ double mf[kW][2][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e = bx * kW + wv;
  const bool live = e < d.nx;
  const int P = d.P, nf = d.Pf + 1;
  if (live && lane < nf) {
    double et = 0, ex = 0, px = 0, ww = 0;
    for (int k = 0; k <= P; ++k) {
      double Ik = d.Ifine[lane * (P + 1) + k];
      int s = e * P + k;
      if (s >= d.ns) s -= d.ns;
      et += Ik * eta[s];
      ex += Ik * etax[s];
      px += Ik * phix[s];
      ww += Ik * ws[s];
    }
    fl[wv][0][lane] = -ex * px + ww * (1.0 + ex * ex);
    fl[wv][1][lane] = -d.g * et - 0.5 * (px * px - ww * ww * (1.0 + ex * ex));
  }
  __syncthreads();
  if (live && lane < nf) {
    double se = 0, sp = 0;
    for (int b = 0; b < nf; ++b) {
      double m = d.Mfine[lane * nf + b];
      se += m * fl[wv][0][b];
      sp += m * fl[wv][1][b];
    }
    mf[wv][0][lane] = se;
    mf[wv][1][lane] = sp;
  }
  __syncthreads();
  if (live && lane <= P) {
    double ae = 0, ap = 0;
    for (int a = 0; a < nf; ++a) {
      double I = d.Ifine[a * (P + 1) + lane];
      ae += I * mf[wv][0][a];
      ap += I * mf[wv][1][a];
    }
    const double J = 0.5 * d.dX;
    const size_t it = (size_t)e * (P + 1) + lane;
    loc[it * 2 + 0] = J * ae;
    loc[it * 2 + 1] = J * ap;
  }
}

__global__ void __launch_bounds__(kBlockThreads)
k_fs_local(const TankDev* __restrict__ td, const double* __restrict__ eta, const double* __restrict__ etax,
           const double* __restrict__ phix, const double* __restrict__ ws, double* __restrict__ loc) {
  fs_local_body(*td, eta, etax, phix, ws, loc, blockIdx.x);
}

// node sums of the element right-hand sides (left element first)
__device__ __forceinline__ void fs_gather_body(const TankDev& d, const double* __restrict__ loc,
                                               double* __restrict__ re, double* __restrict__ rp, int bx) {
  const int s = bx * blockDim.x + threadIdx.x;
  if (s >= d.ns) return;
  const int P = d.P;
  const int e = s / P, k = s - e * P;
  double ae = 0, ap = 0;
  if (e < d.nx) {
    ae = loc[((size_t)e * (P + 1) + k) * 2 + 0];
    ap = loc[((size_t)e * (P + 1) + k) * 2 + 1];
  }
  if (k == 0) {
    int ep = e - 1;
    if (ep < 0 && d.periodic) ep = d.nx - 1;
    if (ep >= 0) {
      ae += loc[((size_t)ep * (P + 1) + P) * 2 + 0];
      ap += loc[((size_t)ep * (P + 1) + P) * 2 + 1];
    }
  }
  re[s] = ae;
  rp[s] = ap;
}

__global__ void k_fs_gather(const TankDev* __restrict__ td, const double* __restrict__ loc,
                            double* __restrict__ re, double* __restrict__ rp) {
  fs_gather_body(*td, loc, re, rp, blockIdx.x);
}

// ------------------------------------------------------------ RK4 + filter
// stage: ye = y0e + a*dt*ke, yp = y0p + a*dt*kp ; acc += w * k
__global__ void k_rk4_stage(int ns, double adt, double wgt, int first, const double* __restrict__ y0e,
                            const double* __restrict__ y0p, const double* __restrict__ ke,
                            const double* __restrict__ kp, double* __restrict__ ye, double* __restrict__ yp,
                            double* __restrict__ acce, double* __restrict__ accp) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  double a = ke[s], bq = kp[s];
  acce[s] = (first ? 0.0 : acce[s]) + wgt * a;
  accp[s] = (first ? 0.0 : accp[s]) + wgt * bq;
  ye[s] = y0e[s] + adt * a;
  yp[s] = y0p[s] + adt * bq;
}

// y = y0 + dt*acc, then the element filter on interior nodes; writes the
// caller's arrays only when the status word is clean (transactional step).
template <int P>
__device__ __forceinline__ void rk4_final_body(const TankDev& d, double dt, const double* __restrict__ acce,
                                               const double* __restrict__ accp, double* __restrict__ eta,
                                               double* __restrict__ phi, int use_filter) {
  double* ne = d.s1d + 13 * (size_t)d.ns;
  double* np_ = d.s1d + 14 * (size_t)d.ns;
  for (int s = threadIdx.x; s < d.ns; s += blockDim.x) {
    ne[s] = eta[s] + dt * acce[s];
    np_[s] = phi[s] + dt * accp[s];
  }
  __syncthreads();
  // filtered values into the scratch pair, then a block-wide validity check,
  // then the write-back (all or nothing)
  double* fe = d.s1d + 15 * (size_t)d.ns;
  double* fp = d.s1d + 11 * (size_t)d.ns;
  __shared__ double red[kBlockThreads];
  double bad = 0.0;
  for (int s = threadIdx.x; s < d.ns; s += blockDim.x) {
    double ve = ne[s], vp = np_[s];
    int e = s / P, k = s - e * P;
    if (use_filter && k > 0) {
      ve = 0;
      vp = 0;
      for (int q = 0; q <= P; ++q) {
        double f = d.Filt[k * (P + 1) + q];
        ve += f * ne[s_index(d, e, q)];
        vp += f * np_[s_index(d, e, q)];
      }
    }
    if (!finite(ve) || !finite(vp)) bad = 1.0;
    fe[s] = ve;
    fp[s] = vp;
  }
  bad = block_sum(bad, red);
  if (bad > 0.0) {
    if (threadIdx.x == 0) atomicOr(d.status, ST_NONFINITE);
    return;
  }
  if (*d.status != 0) return;
  for (int s = threadIdx.x; s < d.ns; s += blockDim.x) {
    eta[s] = fe[s];
    phi[s] = fp[s];
  }
  if (threadIdx.x == 0) {   // the step is complete: its stage record counts
    StageHistory& hs = *d.hs;
    hs.valid = hs.dt == dt ? min(hs.valid + 1, 64) : 1;
    hs.slot = (hs.slot + 1) % kHistSteps;
    hs.dt = dt;
  }
}

template <int P>
__global__ void __launch_bounds__(kBlockThreads)
k_rk4_final(const TankDev* __restrict__ td, double dt, const double* __restrict__ acce,
            const double* __restrict__ accp, double* __restrict__ eta, double* __restrict__ phi,
            int use_filter) {
  rk4_final_body<P>(*td, dt, acce, accp, eta, phi, use_filter);
}

// ------------------------------------------------------------ batched stage kernels
// The per-stage work of the RK4 step around the Laplace solve, over many
// tanks per launch (the single-tank bodies on each tank's own data).
__global__ void __launch_bounds__(kBlockThreads)
k_circ_apply_b(BatchArgs ba, int which, SSel x0, SSel y0, SSel x1, SSel y1) {
  SEM_BATCH_TANK(ba)
  circ_body(d, which, svec(ba, d, it_.tank, x0), svec(ba, d, it_.tank, y0), svec(ba, d, it_.tank, x1),
            svec(ba, d, it_.tank, y1), it_.bx);
}

// M'^-1 applied to the free-surface node sums kept in s1d rows 11 and 12
__global__ void __launch_bounds__(kBlockThreads) k_circ_apply_s1d_b(BatchArgs ba, SSel y0, SSel y1) {
  SEM_BATCH_TANK(ba)
  circ_body(d, 1, d.s1d + 11 * (size_t)d.ns, svec(ba, d, it_.tank, y0), d.s1d + 12 * (size_t)d.ns,
            svec(ba, d, it_.tank, y1), it_.bx);
}

template <int P>
__global__ void __launch_bounds__(kBlockThreads) k_coef_b(BatchArgs ba, SSel eta, SSel etax, int what) {
  SEM_BATCH_TANK(ba)
  coef_body<P>(d, svec(ba, d, it_.tank, eta), svec(ba, d, it_.tank, etax), what, it_.bx);
}

__global__ void __launch_bounds__(kBlockThreads) k_gather_surface_b(BatchArgs ba, VSel u, SSel out) {
  SEM_BATCH_TANK(ba)
  gather_surface_body(d, bvec<double>(d, u), svec(ba, d, it_.tank, out), it_.bx);
}

// element right sides into s1d (the single-tank kernels' scratch)
__global__ void __launch_bounds__(kBlockThreads)
k_fs_local_b(BatchArgs ba, SSel eta, SSel etax, SSel phix, SSel ws) {
  SEM_BATCH_TANK(ba)
  fs_local_body(d, svec(ba, d, it_.tank, eta), svec(ba, d, it_.tank, etax), svec(ba, d, it_.tank, phix),
                svec(ba, d, it_.tank, ws), d.s1d + 5 * (size_t)d.ns, it_.bx);
}

__global__ void __launch_bounds__(kBlockThreads) k_fs_gather_b(BatchArgs ba, int) {
  SEM_BATCH_TANK(ba)
  fs_gather_body(d, d.s1d + 5 * (size_t)d.ns, d.s1d + 11 * (size_t)d.ns, d.s1d + 12 * (size_t)d.ns, it_.bx);
}

// stage update with each tank's own step: ye = y0e + c dt ke, ... (as k_rk4_stage)
__global__ void __launch_bounds__(kBlockThreads)
k_rk4_stage_b(BatchArgs ba, const double* __restrict__ dt, double c, double wgt, int first, SSel y0e, SSel y0p) {
  SEM_BATCH_TANK(ba)
  const int s = it_.bx * blockDim.x + threadIdx.x;
  if (s >= d.ns) return;
  const size_t ns = d.ns;
  const double adt = c * dt[it_.tank];
  const double* ke = d.rk + 5 * ns;
  const double* kp = d.rk + 6 * ns;
  double* acce = d.rk + 7 * ns;
  double* accp = d.rk + 8 * ns;
  const double a = ke[s], bq = kp[s];
  acce[s] = (first ? 0.0 : acce[s]) + wgt * a;
  accp[s] = (first ? 0.0 : accp[s]) + wgt * bq;
  d.rk[s] = svec(ba, d, it_.tank, y0e)[s] + adt * a;
  d.rk[ns + s] = svec(ba, d, it_.tank, y0p)[s] + adt * bq;
}

template <int P>
__global__ void __launch_bounds__(kBlockThreads)
k_rk4_final_b(BatchArgs ba, const double* __restrict__ dt, SSel eta, SSel phi) {
  SEM_BATCH_TANK(ba)
  const size_t ns = d.ns;
  rk4_final_body<P>(d, dt[it_.tank], d.rk + 7 * ns, d.rk + 8 * ns, svec(ba, d, it_.tank, eta),
                    svec(ba, d, it_.tank, phi), d.use_filter);
}

// ------------------------------------------------------------ launchers
#define SEM_P_CASE(V, ...) \
  case V: {                \
    constexpr int PP = V;  \
    __VA_ARGS__;           \
  } break;
#define SEM_P_SWITCH(P, ...)              \
  switch (P) {                            \
    SEM_P_CASE(1, __VA_ARGS__)            \
    SEM_P_CASE(2, __VA_ARGS__)            \
    SEM_P_CASE(3, __VA_ARGS__)            \
    SEM_P_CASE(4, __VA_ARGS__)            \
    SEM_P_CASE(5, __VA_ARGS__)            \
    SEM_P_CASE(6, __VA_ARGS__)            \
    SEM_P_CASE(7, __VA_ARGS__)            \
    SEM_P_CASE(8, __VA_ARGS__)            \
    default: break;                       \
  }

static inline unsigned nblk(int64_t n, int t = kBlockThreads) { return (unsigned)((n + t - 1) / t); }

size_t gather_lds_bytes(const TankDev& h, size_t word) {
  return word * ((size_t)h.cb * h.nc + h.nl + 3 * (size_t)h.EB * h.NpP);
}

void launch_coef(const TankDev& h, const TankDev* d, const double* eta, const double* etax, int what,
                 hipStream_t st) {
  int64_t total = (int64_t)h.nb * h.T * h.Np * 16;
  SEM_P_SWITCH(h.P, hipLaunchKernelGGL(k_coef<PP>, dim3(nblk(total)), dim3(kBlockThreads), 0, st, d, eta, etax, what));
}

// element kernel only (no line fix-up)
template <typename T, typename GS>
static void gather_kernel(const TankDev& h, const TankDev* d, int op, const T* u, T* y, T* side, int flags,
                          hipStream_t st) {
  size_t lds = gather_lds_bytes(h, sizeof(T));
  dim3 g(h.nb), b(kBlockThreads);
#define SEM_G(OPV) SEM_P_SWITCH(h.P, hipLaunchKernelGGL((k_gather<PP, OPV, T, GS>), g, b, lds, st, d, u, y, side, flags))
  if (sizeof(T) == sizeof(double)) {
    switch (op) {
      case OP_STIFF: SEM_G(OP_STIFF); break;
      case OP_MASS: SEM_G(OP_MASS); break;
      case OP_PRE_LAP: SEM_G(OP_PRE_LAP); break;
      case OP_PRE_MASS: SEM_G(OP_PRE_MASS); break;
      case OP_SZ: SEM_G(OP_SZ); break;
      case OP_SU: SEM_G(OP_SU); break;
    }
  } else {
    switch (op) {
      case OP_STIFF: SEM_G(OP_STIFF); break;
      case OP_PRE_LAP: SEM_G(OP_PRE_LAP); break;
    }
  }
#undef SEM_G
}

static void stiff_mfma(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, int flags,
                       int gstore, hipStream_t st) {
  launch_stiff_mfma(h, d, u, y, side, flags, st);
}
static void stiff_mfma(const TankDev& h, const TankDev* d, const float* u, float* y, float* side, int flags,
                       int gstore, hipStream_t st) {
  launch_stiff_mfma(h, d, u, y, side, flags, gstore, st);
}

template <typename T, typename GS>
static void gather_full(const TankDev& h, const TankDev* d, int op, const T* u, T* y, T* side, int flags,
                        hipStream_t st) {
  if ((op == OP_PRE_LAP || op == OP_PRE_MASS) && h.pre_kind == 1) {
    if (op == OP_PRE_LAP || sizeof(T) == sizeof(double)) {
      launch_sd(h, d, op == OP_PRE_LAP ? 0 : 1, u, y, (flags & F_GATE) ? 1 : 0, st);
      return;
    }
  }
  bool done = false;
  if constexpr (sizeof(T) == sizeof(double)) {
    if (op == OP_SZ && h.use_mfma && flags == 0) {
      launch_sz_mfma(h, d, u, y, side, st);
      done = true;
    }
  }
  if (done) {
  } else if (op == OP_STIFF && h.use_mfma) {
    stiff_mfma(h, d, u, y, side, flags, sizeof(GS) == 1 ? 2 : 1, st);
  } else {
    gather_kernel<T, GS>(h, d, op, u, y, side, flags, st);
  }
  if (!(flags & F_NOFIX))
    hipLaunchKernelGGL(k_fixup<T>, dim3(nblk((int64_t)h.nb * h.nl)), dim3(kBlockThreads), 0, st, d, y, side, flags);
}

void launch_fixup(const TankDev& h, const TankDev* d, double* y, double* side, int flags, hipStream_t st) {
  hipLaunchKernelGGL(k_fixup<double>, dim3(nblk((int64_t)h.nb * h.nl)), dim3(kBlockThreads), 0, st, d, y, side, flags);
}
void launch_fixup(const TankDev& h, const TankDev* d, float* y, float* side, int flags, hipStream_t st) {
  hipLaunchKernelGGL(k_fixup<float>, dim3(nblk((int64_t)h.nb * h.nl)), dim3(kBlockThreads), 0, st, d, y, side, flags);
}

void launch_gather(const TankDev& h, const TankDev* d, int op, const double* u, double* y, double* side,
                   int flags, hipStream_t st) {
  gather_full<double, double>(h, d, op, u, y, side, flags, st);
}
void launch_gather(const TankDev& h, const TankDev* d, int op, const float* u, float* y, float* side, int flags,
                   int gstore, hipStream_t st) {
  if (gstore == 2) gather_full<float, BF16>(h, d, op, u, y, side, flags, st);
  else gather_full<float, float>(h, d, op, u, y, side, flags, st);
}

// element kernel of an operator without the line fix-up (timing support);
// prec 0 = FP64, 1 = FP32, 2 = FP32 with bfloat16 factors
void launch_gather_only(const TankDev& h, const TankDev* d, int op, int prec, const void* u, void* y, void* side,
                        hipStream_t st) {
  if (prec == 0) {
    if ((op == OP_PRE_LAP || op == OP_PRE_MASS) && h.pre_kind == 1)
      launch_sd(h, d, op == OP_PRE_LAP ? 0 : 1, (const double*)u, (double*)y, 0, st);
    else if (op == OP_STIFF && h.use_mfma) launch_stiff_mfma(h, d, (const double*)u, (double*)y, (double*)side, 0, st);
    else gather_kernel<double, double>(h, d, op, (const double*)u, (double*)y, (double*)side, 0, st);
  } else {
    if (op == OP_PRE_LAP && h.pre_kind == 1) launch_sd(h, d, 0, (const float*)u, (float*)y, 0, st);
    else if (op == OP_STIFF && h.use_mfma)
      launch_stiff_mfma(h, d, (const float*)u, (float*)y, (float*)side, 0, prec == 2 ? 2 : 1, st);
    else if (prec == 2) gather_kernel<float, BF16>(h, d, op, (const float*)u, (float*)y, (float*)side, 0, st);
    else gather_kernel<float, float>(h, d, op, (const float*)u, (float*)y, (float*)side, 0, st);
  }
}

void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, a, x, b, y);
}
void launch_fill(int64_t n, double v, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, v, y);
}
void launch_solve_begin(const TankDev& h, const TankDev* d, const double* phis, double* u, const double* ws,
                        int stage, int maxdepth, double dt, double rtol, int init_ks, hipStream_t st) {
  hipLaunchKernelGGL(k_solve_begin, dim3(nblk(h.n)), dim3(kBlockThreads), 0, st, d, phis, u, ws, stage, maxdepth, dt,
                     rtol, init_ks);
}
void launch_solve_end(const TankDev& h, const TankDev* d, const double* phis, double* phi, int stage, hipStream_t st) {
  hipLaunchKernelGGL(k_solve_end, dim3(nblk(h.n)), dim3(kBlockThreads), 0, st, d, phis, phi, stage);
}
void launch_mask_surface(const TankDev& h, const TankDev* d, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_mask_surface, dim3(nblk(h.n)), dim3(kBlockThreads), 0, st, d, y);
}
void launch_scatter_surface(const TankDev& h, const TankDev* d, const double* phis, double* u, int zero_rest,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_surface, dim3(nblk(h.n)), dim3(kBlockThreads), 0, st, d, phis, u, zero_rest);
}
void launch_gather_surface(const TankDev& h, const TankDev* d, const double* u, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_surface, dim3(nblk(h.ns)), dim3(kBlockThreads), 0, st, d, u, out);
}

// chunking of [0, n) for the reductions (the device side's dot_chunk)
void dot_layout(int64_t n, int* nchunk, int64_t* chunk) {
  *chunk = dot_chunk(n);
  *nchunk = dot_nchunk(n);
}

template <typename T>
static void dots_t(int64_t n, int nvec, const T* X, int64_t ldx, const T* w, double* part, int ldp, double* out,
                   int32_t* counter, const KrylovState* gate, const TankDev* fixd, const T* side, hipStream_t st) {
  int nc;
  int64_t chunk;
  dot_layout(n, &nc, &chunk);
  hipLaunchKernelGGL(k_dots_fused<T>, dim3(nc), dim3(kBlockThreads), 0, st, n, nvec, X, ldx, const_cast<T*>(w), part,
                     ldp, out, chunk, counter, gate, fixd, side);
}
void launch_dots(int64_t n, int nvec, const double* X, int64_t ldx, const double* w, double* part, int ldp,
                 double* out, int32_t* counter, const KrylovState* gate, hipStream_t st, const TankDev* fixd,
                 const double* side) {
  dots_t<double>(n, nvec, X, ldx, w, part, ldp, out, counter, gate, fixd, side, st);
}
void launch_dots(int64_t n, int nvec, const float* X, int64_t ldx, const float* w, double* part, int ldp,
                 double* out, int32_t* counter, const KrylovState* gate, hipStream_t st, const TankDev* fixd,
                 const float* side) {
  dots_t<float>(n, nvec, X, ldx, w, part, ldp, out, counter, gate, fixd, side, st);
}

template <typename T>
static void orth_t(int64_t n, int j, const T* V, double* H, int m, T* w, double* part, int ldp, KrylovState* ks,
                   int32_t* counter, int32_t* status, int32_t* mirror, hipStream_t st, const TankDev* fixd,
                   const T* side) {
  int nc;
  int64_t chunk;
  dot_layout(n, &nc, &chunk);
  hipLaunchKernelGGL(k_orth_fused<T>, dim3(nc), dim3(kBlockThreads), 0, st, n, j, V, H, m, w, part, ldp, chunk, ks,
                     counter, status, mirror, fixd, side);
}
void launch_orth_givens(int64_t n, int j, const double* V, double* H, int m, double* w, double* part, int ldp,
                        KrylovState* ks, int32_t* counter, int32_t* status, int32_t* mirror, hipStream_t st,
                        const TankDev* fixd, const double* side) {
  orth_t<double>(n, j, V, H, m, w, part, ldp, ks, counter, status, mirror, st, fixd, side);
}
void launch_orth_givens(int64_t n, int j, const float* V, double* H, int m, float* w, double* part, int ldp,
                        KrylovState* ks, int32_t* counter, int32_t* status, int32_t* mirror, hipStream_t st,
                        const TankDev* fixd, const float* side) {
  orth_t<float>(n, j, V, H, m, w, part, ldp, ks, counter, status, mirror, st, fixd, side);
}

void launch_scale_next(int64_t n, int j, const double* w, double* V, const double* H, int m,
                       const KrylovState* ks, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_next<double>, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, j, w, V, H, m, ks);
}
void launch_scale_next(int64_t n, int j, const float* w, float* V, const double* H, int m,
                       const KrylovState* ks, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_next<float>, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, j, w, V, H, m, ks);
}
void launch_solve_update_fused(int64_t n, const double* Z, double* H, int m, KrylovState* ks, double* x,
                               hipStream_t st, const TankDev* d, const double* phis, double* phi, int stage) {
  hipLaunchKernelGGL(k_solve_update<double>, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, Z, H, m, ks, x, d, phis,
                     phi, stage);
}
void launch_solve_update_fused(int64_t n, const float* Z, double* H, int m, KrylovState* ks, float* x,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_solve_update<float>, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, Z, H, m, ks, x,
                     (const TankDev*)nullptr, (const double*)nullptr, (double*)nullptr, -1);
}
template <typename T>
static void residual_cycle_t(const TankDev* d, int64_t n, const T* b, const T* y, const T* side, T* r, int mask,
                             double* part, int ldp, double* rr, int32_t* counter, KrylovState* ks, double* H, int m,
                             int first, int32_t* status, int32_t* mirror, hipStream_t st, const T* bside) {
  int nc;
  int64_t chunk;
  dot_layout(n, &nc, &chunk);
  hipLaunchKernelGGL(k_residual_cycle<T>, dim3(nc), dim3(kBlockThreads), 0, st, d, n, const_cast<T*>(b), y, side, r,
                     mask, part, ldp, rr, chunk, counter, ks, H, m, first, status, mirror, bside);
  hipLaunchKernelGGL(k_scale_v0<T>, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, r, ks);
}
void launch_residual_cycle(const TankDev& h, const TankDev* d, int64_t n, const double* b, const double* y,
                           const double* side, double* r, int mask, double* part, int ldp, double* rr,
                           int32_t* counter, KrylovState* ks, double* H, int m, int first, int32_t* status,
                           int32_t* mirror, hipStream_t st, const double* bside) {
  residual_cycle_t<double>(d, n, b, y, side, r, mask, part, ldp, rr, counter, ks, H, m, first, status, mirror, st,
                           bside);
}
void launch_residual_cycle(const TankDev& h, const TankDev* d, int64_t n, const float* b, const float* y,
                           const float* side, float* r, int mask, double* part, int ldp, double* rr,
                           int32_t* counter, KrylovState* ks, double* H, int m, int first, int32_t* status,
                           int32_t* mirror, hipStream_t st) {
  residual_cycle_t<float>(d, n, b, y, side, r, mask, part, ldp, rr, counter, ks, H, m, first, status, mirror, st,
                          (const float*)nullptr);
}
void launch_residual(const TankDev& h, const TankDev* d, int64_t n, const double* b, const double* y, double* r,
                     int mask, hipStream_t st) {
  hipLaunchKernelGGL(k_residual<double>, dim3(nblk(n)), dim3(kBlockThreads), 0, st, d, n, b, y, r, mask);
}
void launch_residual(const TankDev& h, const TankDev* d, int64_t n, const float* b, const float* y, float* r,
                     int mask, hipStream_t st) {
  hipLaunchKernelGGL(k_residual<float>, dim3(nblk(n)), dim3(kBlockThreads), 0, st, d, n, b, y, r, mask);
}
// ------------------------------------------------------------ batched launchers
static bool batch_args(const BatchArgs& a0, const BatchStage& p, BatchArgs* a) {
  if (p.items.empty()) return false;
  *a = a0;
  a->items = p.dev;
  return true;
}
#define SEM_BLAUNCH(P, KERN, ...)                                                                              \
  do {                                                                                                       \
    BatchArgs a_;                                                                                            \
    if (batch_args(a0, P, &a_))                                                                              \
      hipLaunchKernelGGL(KERN, dim3((unsigned)(P).items.size()), dim3(kBlockThreads), 0, st, a_, __VA_ARGS__); \
  } while (0)

void launch_dots_b(const BatchArgs& a0, const BatchStage& p, const BatchStage& per_tank, int nvec, VSel X, VSel w,
                   int hcol, int sidx, int fix, int gate, int f32, hipStream_t st) {
  if (f32) SEM_BLAUNCH(p, k_dots_b<float>, nvec, X, w, fix, gate);
  else SEM_BLAUNCH(p, k_dots_b<double>, nvec, X, w, fix, gate);
  SEM_BLAUNCH(per_tank, k_dots_sum_b, nvec, hcol, sidx, gate);
}
void launch_orth_b(const BatchArgs& a0, const BatchStage& p, const BatchStage& per_tank, int j, int f32,
                   hipStream_t st, int fix) {
  if (f32) SEM_BLAUNCH(p, k_orth_b<float>, j, fix);
  else SEM_BLAUNCH(p, k_orth_b<double>, j, fix);
  SEM_BLAUNCH(per_tank, k_orth_sum_b, j);
}
void launch_dots_blocks_b(const BatchArgs& a0, const BatchStage& p, const BatchStage& per_tank, int nvec, int hcol,
                          int f32, hipStream_t st) {
  if (f32) SEM_BLAUNCH(p, k_dots_blocks_b<float>, nvec);
  else SEM_BLAUNCH(p, k_dots_blocks_b<double>, nvec);
  SEM_BLAUNCH(per_tank, k_dots_sum_blocks_b, nvec, hcol);
}
void launch_fixup_b(const BatchArgs& a0, const BatchStage& p, VSel y, int flags, int f32, hipStream_t st) {
  if (f32) SEM_BLAUNCH(p, k_fixup_b<float>, y, flags);
  else SEM_BLAUNCH(p, k_fixup_b<double>, y, flags);
}
void launch_predict_b(const BatchArgs& a0, const BatchStage& vec, int stage, int maxdepth, const double* dt, int table,
                      hipStream_t st) {
  SEM_BLAUNCH(vec, k_predict_b, stage, maxdepth, dt, table);
}
void launch_history_b(const BatchArgs& a0, const BatchStage& vec, int stage, int table, hipStream_t st) {
  SEM_BLAUNCH(vec, k_history_b, stage, table);
}
void launch_residual_b(const BatchArgs& a0, const BatchStage& p, VSel b, VSel y, VSel r, int f32, hipStream_t st) {
  if (f32) SEM_BLAUNCH(p, k_residual_b<float>, b, y, r);
  else SEM_BLAUNCH(p, k_residual_b<double>, b, y, r);
}
void launch_cycle_start_b(const BatchArgs& a0, const BatchStage& per_tank, const BatchStage& vec, int first, int f32,
                          hipStream_t st) {
  SEM_BLAUNCH(per_tank, k_cycle_start_b, first);
  if (f32) SEM_BLAUNCH(vec, k_scale_v0_b<float>, 0);
  else SEM_BLAUNCH(vec, k_scale_v0_b<double>, 0);
}
void launch_solve_update_b(const BatchArgs& a0, const BatchStage& per_tank, const BatchStage& vec, VSel x, int f32,
                           hipStream_t st) {
  SEM_BLAUNCH(per_tank, k_solve_y_b, 0);
  if (f32) SEM_BLAUNCH(vec, k_update_x_b<float>, x);
  else SEM_BLAUNCH(vec, k_update_x_b<double>, x);
}
void launch_ks_init_b(const BatchArgs& a0, const BatchStage& per_tank, double rtol, const double* rtol_t,
                      hipStream_t st) {
  SEM_BLAUNCH(per_tank, k_ks_init_b, rtol, rtol_t);
}
void launch_status_clear_b(const BatchArgs& a0, const BatchStage& per_tank, hipStream_t st) {
  SEM_BLAUNCH(per_tank, k_status_clear_b, 0);
}
void launch_state_out_b(const BatchArgs& a0, const BatchStage& per_tank, KrylovState* ks_out, int32_t* st_out,
                        int mark_noconv, hipStream_t st) {
  SEM_BLAUNCH(per_tank, k_state_out_b, ks_out, st_out, mark_noconv);
}
void launch_scal_out_b(const BatchArgs& a0, const BatchStage& per_tank, int idx, double* out, hipStream_t st) {
  SEM_BLAUNCH(per_tank, k_scal_out_b, idx, out);
}
void launch_to_float_b(const BatchArgs& a0, const BatchStage& vec, const double* scale, hipStream_t st) {
  SEM_BLAUNCH(vec, k_to_float_b, scale);
}
void launch_add_float_b(const BatchArgs& a0, const BatchStage& vec, const double* scale, hipStream_t st) {
  SEM_BLAUNCH(vec, k_add_float_b, scale);
}
void launch_status_or_b(const BatchArgs& a0, const BatchStage& per_tank, int bits, hipStream_t st) {
  SEM_BLAUNCH(per_tank, k_status_or_b, bits);
}
void launch_lift_in_b(const BatchArgs& a0, const BatchStage& vec, const double* const* phis,
                      const double* const* guess, hipStream_t st) {
  SEM_BLAUNCH(vec, k_lift_in_b, phis, guess);
}
void launch_solution_out_b(const BatchArgs& a0, const BatchStage& vec, const double* const* phis, double* const* phi,
                           hipStream_t st) {
  SEM_BLAUNCH(vec, k_solution_out_b, phis, phi);
}
#undef SEM_BLAUNCH

void launch_to_float(int64_t n, const double* r, double scale, float* r32, hipStream_t st) {
  hipLaunchKernelGGL(k_to_float, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, r, scale, r32);
}
void launch_add_float(int64_t n, const float* x32, double scale, double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_add_float, dim3(nblk(n)), dim3(kBlockThreads), 0, st, n, x32, scale, x);
}
void launch_fill_f(int64_t n, float* y, hipStream_t st) { hipMemsetAsync(y, 0, n * sizeof(float), st); }

// Krylov state of a fresh solve: everything zero (the reductions' completion
// counter included) except the tolerance
__global__ void k_ks_reset(KrylovState* ks, double rtol) {
  if (threadIdx.x == 0) {
    KrylovState z{};
    z.rtol = rtol;
    *ks = z;
  }
}
void launch_ks_reset(KrylovState* ks, double rtol, hipStream_t st) {
  hipLaunchKernelGGL(k_ks_reset, dim3(1), dim3(64), 0, st, ks, rtol);
}

void launch_recover_dx(const TankDev& h, const TankDev* d, const double* in0, double* out0, const double* in1,
                       double* out1, hipStream_t st) {
  hipLaunchKernelGGL(k_circ_apply, dim3(nblk(h.ns, kBlockThreads / 64)), dim3(kBlockThreads), 0, st, d, 0, in0, out0,
                     in1, out1);
}
void launch_fs_rhs(const TankDev& h, const TankDev* d, const double* eta, const double* etax, const double* phix,
                   const double* ws, double* et, double* pt, hipStream_t st) {
  launch_fs_rhs_into(h, d, eta, etax, phix, ws, et, pt, h.s1d + 5 * (size_t)h.ns, h.s1d + 11 * (size_t)h.ns,
                     h.s1d + 12 * (size_t)h.ns, st);
}
void launch_fs_rhs_into(const TankDev& h, const TankDev* d, const double* eta, const double* etax,
                        const double* phix, const double* ws, double* et, double* pt, double* loc, double* re,
                        double* rp, hipStream_t st) {
  hipLaunchKernelGGL(k_fs_local, dim3(nblk(h.nx, kBlockThreads / 64)), dim3(kBlockThreads), 0, st, d, eta, etax,
                     phix, ws, loc);
  hipLaunchKernelGGL(k_fs_gather, dim3(nblk(h.ns)), dim3(kBlockThreads), 0, st, d, loc, re, rp);
  hipLaunchKernelGGL(k_circ_apply, dim3(nblk(h.ns, kBlockThreads / 64)), dim3(kBlockThreads), 0, st, d, 1, re, et, rp,
                     pt);
}
// Relaxation-zone source of Sec. 2.2 added to a stage's slopes:
// k += w (q_a - q) / tau for q = eta and phi~ at the stage state.
__global__ void k_relax(int ns, double inv_tau, const double* __restrict__ w, const double* __restrict__ qae,
                        const double* __restrict__ qap, const double* __restrict__ se, const double* __restrict__ sp,
                        double* __restrict__ ke, double* __restrict__ kp) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const double a = w[s] * inv_tau;
  ke[s] += a * (qae[s] - se[s]);
  kp[s] += a * (qap[s] - sp[s]);
}
void launch_relax(int ns, double inv_tau, const double* w, const double* qae, const double* qap, const double* se,
                  const double* sp, double* ke, double* kp, hipStream_t st) {
  hipLaunchKernelGGL(k_relax, dim3(nblk(ns)), dim3(kBlockThreads), 0, st, ns, inv_tau, w, qae, qap, se, sp, ke, kp);
}

void launch_rk4_stage(int ns, double adt, double wgt, int first, const double* y0e, const double* y0p,
                      const double* ke, const double* kp, double* ye, double* yp, double* acce, double* accp,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_rk4_stage, dim3(nblk(ns)), dim3(kBlockThreads), 0, st, ns, adt, wgt, first, y0e, y0p, ke, kp,
                     ye, yp, acce, accp);
}
void launch_rk4_final(const TankDev& h, const TankDev* d, double dt, const double* acce, const double* accp,
                      double* eta, double* phi, int use_filter, hipStream_t st) {
  SEM_P_SWITCH(h.P, hipLaunchKernelGGL(k_rk4_final<PP>, dim3(1), dim3(kBlockThreads), 0, st, d, dt, acce, accp, eta, phi, use_filter));
}

// ------------------------------------------------------------ batched stage launchers
void plan_stage(const std::vector<TankDev>& tanks, const std::vector<int>& ids, BatchStagePlan* out) {
  *out = BatchStagePlan{};
  for (int t : ids) {
    const TankDev& h = tanks[t];
    auto add = [&](BatchStage& s, int gx, size_t lds) {
      for (int x = 0; x < gx; ++x) s.items.push_back(BatchItem{t, x, 0, gx});
      s.lds = std::max(s.lds, lds);
    };
    const int P = h.P;
    add(out->coef[P], (int)nblk((int64_t)h.nb * h.T * h.Np * 16), 0);
    add(out->final_[P], 1, 0);
    add(out->surf, (int)nblk(h.ns), 0);
    if (h.circ1d) {
      add(out->circ, (int)nblk(h.ns, kBlockThreads / 64), 0);
      add(out->fsl, (int)nblk(h.nx, kBlockThreads / 64), 0);
      add(out->fsg, (int)nblk(h.ns), 0);
    }
  }
}

#define SEM_BL(ST, KERN, ...)                                                                                   \
  do {                                                                                                        \
    BatchArgs a_;                                                                                             \
    if (batch_args(a0, ST, &a_))                                                                              \
      hipLaunchKernelGGL(KERN, dim3((unsigned)(ST).items.size()), dim3(kBlockThreads), (ST).lds, st, a_,       \
                         __VA_ARGS__);                                                                         \
  } while (0)

void launch_recover_dx_b(const BatchArgs& a0, const BatchStagePlan& p, SSel in0, SSel out0, SSel in1, SSel out1,
                         hipStream_t st) {
  SEM_BL(p.circ, k_circ_apply_b, 0, in0, out0, in1, out1);
}
void launch_coef_b(const BatchArgs& a0, const BatchStagePlan& p, SSel eta, SSel etax, int what, hipStream_t st) {
  for (int P = 1; P <= kMaxOrder; ++P) SEM_P_SWITCH(P, SEM_BL(p.coef[PP], k_coef_b<PP>, eta, etax, what));
}
void launch_gather_surface_b(const BatchArgs& a0, const BatchStagePlan& p, VSel u, SSel out, hipStream_t st) {
  SEM_BL(p.surf, k_gather_surface_b, u, out);
}
void launch_fs_rhs_b(const BatchArgs& a0, const BatchStagePlan& p, SSel eta, SSel etax, SSel phix, SSel ws,
                     SSel et, SSel pt, hipStream_t st) {
  SEM_BL(p.fsl, k_fs_local_b, eta, etax, phix, ws);
  SEM_BL(p.fsg, k_fs_gather_b, 0);
  SEM_BL(p.circ, k_circ_apply_s1d_b, et, pt);   // M'^-1 of the node sums
}
void launch_rk4_stage_b(const BatchArgs& a0, const BatchStagePlan& p, const double* dt, double c, double wgt,
                        int first, SSel y0e, SSel y0p, hipStream_t st) {
  SEM_BL(p.surf, k_rk4_stage_b, dt, c, wgt, first, y0e, y0p);
}
void launch_rk4_final_b(const BatchArgs& a0, const BatchStagePlan& p, const double* dt, SSel eta, SSel phi,
                        hipStream_t st) {
  for (int P = 1; P <= kMaxOrder; ++P) SEM_P_SWITCH(P, SEM_BL(p.final_[PP], k_rk4_final_b<PP>, dt, eta, phi));
}
#undef SEM_BL

}  // namespace sem
