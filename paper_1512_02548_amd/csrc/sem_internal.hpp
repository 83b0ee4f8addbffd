// Internal data structures shared by the host driver and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sem {

constexpr int kMaxOrder = 8;
constexpr int kMaxContrib = 8;      // element contributions to one column-local node
constexpr int kBlockThreads = 256;
constexpr int kMaxRestart = 64;     // GMRES restart length limit
constexpr int kMaxVec = kMaxRestart + 1;
constexpr int kMaxLayers = 256;     // sigma layers (nz) at most
// Fourier modes per workgroup of the direct-transform mode solves: 8 for
// short tanks (more workgroups), 16 from nx > 128 on (full 16-row MFMA tiles,
// each workgroup's pass over the columns shared by more modes)
constexpr int kModesPerBlockMax = 16;
__host__ __device__ inline int modes_per_block(int nx) { return nx <= 128 ? 8 : 16; }

// Mode solves take mode k together with its conjugate partner nx - k (both
// use the one stored inverse symbol): a workgroup of `pairs` pairs has
// k = pairs bx + h in slot h and nx - k in slot pairs + h (-1: empty slot;
// modes 0 and nx/2 have no partner).
__host__ __device__ inline int paired_mode(int bx, int slot, int pairs, int nx) {
  const int h = slot < pairs ? slot : slot - pairs;
  const int k = pairs * bx + h;
  if (2 * k > nx) return -1;
  if (slot < pairs) return k;
  return (k == 0 || 2 * k == nx) ? -1 : nx - k;
}
__host__ __device__ inline int paired_blocks(int nx, int pairs) { return (nx / 2) / pairs + 1; }
// the four-step path's mode solve: up to ml = 256 / q modes per workgroup
// (paired when ml >= 2, one mode per workgroup otherwise)
__host__ __device__ inline int fft_modes_per_block(int q) { return q >= 256 ? 1 : 256 / q; }
__host__ __device__ inline int fft_slots(int ml) { return ml < 2 ? 1 : 2 * (ml / 2); }
__host__ __device__ inline int fft_mode(int bx, int slot, int ml, int nx) {
  if (ml < 2) return bx < nx ? bx : -1;
  return paired_mode(bx, slot, ml / 2, nx);
}
__host__ __device__ inline int fft_mode_blocks(int nx, int ml) { return ml < 2 ? nx : paired_blocks(nx, ml / 2); }

// status bits accumulated on the device
enum : int32_t {
  ST_DOMAIN = 1,
  ST_NOCONV = 2,
  ST_BREAKDOWN = 4,
  ST_NONFINITE = 8,
};

// Krylov state of one solve, resident in the workspace.
// Record of the RK4 stepper's stage solutions, for the initial guesses of
// the stage Laplace solves: the ring slot of the next step, the number of
// consecutive completed steps with step size dt since the last reset (a
// different step size starts the record again).
struct StageHistory {
  int32_t slot;
  int32_t valid;
  double dt;
};
constexpr int kHistSteps = 6;       // past steps kept per stage

struct KrylovState {
  double bnorm;       // ||b||
  double beta;        // ||r0|| of the current cycle
  double resid;       // current residual estimate |g_{j+1}|
  double rtol;
  int32_t j;          // columns completed in the current cycle
  int32_t done;       // 1 when the cycle ended (converged or restart)
  int32_t converged;  // 1 when rtol met
  int32_t iters;      // total iterations
  int32_t status;
  int32_t pad[3];
};

// Exact inverse of a column-coupled operator on a periodic tank: the interior
// nodes of every column are condensed onto the vertical lines, the resulting
// block-circulant line system is diagonalised by a DFT along x.  Dense
// factors are stored in MFMA fragment order: element (M-tile mt, K-step s,
// lane l) is A[16 mt + l%16][4 s + l/16], zero padded.
struct SDData {
  int32_t nI, q;                  // interior unknowns per column, unknowns per line
  int32_t zero_surface;           // 1: surface nodes are Dirichlet (set to 0)
  int32_t M1;                     // nI + 2q rows of the condensation factor
  int32_t nMT1, KS1;              // its M-tiles and K-steps
  int32_t nMT3, KS3;              // of the back-substitution factor
  const int32_t* I_idx;           // [nI] column-local indices of the interior unknowns
  const double* A1;               // fragments of [A_II^-1; A_LI A_II^-1; A_RI A_II^-1]  (M1 x nI)
  const double* C3;               // fragments of A_II^-1 [A_IL | A_IR]                    (nI x 2q)
  const double* Shat;             // [nx/2+1][q][q][2] inverse line symbol per Fourier mode k <= nx/2,
                                  // column-major (mode nx - k is the conjugate of mode k)
  const float* A1_32;
  const float* C3_32;
  const float* Shat32;
  double* yI;                     // [nx][nI] interior solves
  double* TL;                     // [nx][q]
  double* TR;                     // [nx][q]
  double* XH;                     // [nx][q][2] modal line solution
  // tanks with walls: correction for the jump v between the wall line nx and
  // line 0 of the periodic solve (Schur complement on the wall line)
  int32_t wall, pad2;
  const double* Wv;               // [q][3q + nI] v from [r_wall; x_{nx-1}; x_0; y_I(nx-1)], row-major
  const double* Hm;               // [nx/2+1][q][q][2] modal response to v, column-major per mode
                                  // (mode nx - k is the conjugate of mode k)
  const double* Qm;               // [q][nI] interior response of the last column, column-major
  double* vbuf;                   // [q] v
  double* WP;                     // [2][q] lines nx-1 and 0 of the periodic solve
  int32_t pad5;
  // long tanks: the transforms along x as four-step FFTs, nx = n1 n2
  int32_t fft_n1, fft_n2;         // 0: direct DFT products
  int32_t pad3;
  double* FT;                     // [nx][q][2] intermediate of the two-step transforms
  double* FG;                     // [nx][q][2] transformed line right sides
  double* XL;                     // [nx][q] line solution
};

// Everything a kernel needs about one tank; lives in device memory at the
// start of the tank's workspace.  Pointers are device addresses.
struct TankDev {
  // sizes
  int32_t P, Np, NpP, nx, nz, periodic, nl, nc, n, ns, E;
  int32_t cb, nb, T, EB;          // columns per block, blocks, tiles per block, elems per block (cb*2nz)
  int32_t m;                      // GMRES restart length
  int32_t Pf;
  double L, dX, g;
  // reference operators (padded to NpP, row-major)
  const double* Dr;               // NpP x NpP
  const double* Ds;
  const double* MDr;              // M Dr
  const double* MDs;
  const double* Mref;             // M
  const float* Dr32;
  const float* Ds32;
  const float* MDr32;
  const float* MDs32;
  const float* Mref32;
  const double* opf;              // [4 NpP^2] stiffness operators in MFMA fragment order (FP64 rows)
  const float* opf32;             // the same for the FP32 accumulator row map
  const double* opf_sz;           // [4 NpP^2] S_z operators: stage 1 as opf, stage 2 M (second block zero)
  // mesh tables
  const int32_t* elem_loc;        // [2nz][NpP] column-local node (< nc + nl), -1 = padding
  const int32_t* acc_cnt;         // [nc] number of contributions
  const int32_t* acc_ent;         // [nc][kMaxContrib]: bit 30 = previous column, low bits e_in_col*NpP + m
  const int32_t* surf_loc;        // [P] column-local index of the surface nodes of a column
  const int32_t* is_surf_loc;     // [nc + nl] 1 if the column-local node lies on sigma = 1
  const uint16_t* acc_pk;         // [nc][kMaxContrib]: offset in the element outputs (e_in_col (NpP+1) + m) | prev << 15
  const uint16_t* acc_cm;         // [nc]: count | surface << 4
  const double* lay;              // [2nz][8]: Lam_rx, Lam_rs(sig), Lam_sx, Lam_ss, J, sigma_j, dsigma_j, 0
  const double* nodeq;            // [2][NpP][2]: xi, zeta of each reference node in the unit quad
  const double* colw;             // [2][NpP][P+1]: column interpolation weights at xi
  const double* pre_lap;          // [nclass][NpP][NpP] W C^{-1} W (free nodes), zero padded
  const double* pre_mass;         // [nclass][NpP][NpP]
  const float* pre_lap32;
  int32_t nclass_col;             // 1 (periodic) or 3 (walls: first, interior, last)
  int32_t pre_kind;               // 0 element-block Jacobi, 1 exact inverses (line Schur + DFT)
  const double* twid;             // [nx][2] exp(-2 pi i m / nx)
  int32_t use_mfma;               // stiffness apply on matrix cores (1) or the reference kernel (0)
  int32_t pad1;
  // exact inverses by line condensation + DFT (periodic tanks): [0] the
  // still-water Laplace operator on the free nodes, [1] the 2D mass matrix
  SDData sd[2];
  // 1D surface operators (P+1)^2 etc.
  const double* M1;
  const double* S1;               // M1 D1
  const double* Ifine;            // (Pf+1) x (P+1)
  const double* Mfine;            // (Pf+1) x (Pf+1)
  const double* Filt;             // (P+1) x (P+1)
  int32_t circ1d;                 // periodic: M'^{-1} and M'^{-1} S_x applied as block-circulant rows
  int32_t circ_band;              // ... over the elements within this distance of the diagonal (all if 2 band + 1 >= nx)
  const double* Brow;             // [P][ns] first block-row of M'^{-1}
  const double* Rrow;             // [P][ns] first block-row of M'^{-1} S_x
  // walls: rows of M'^{-1} S_x (table 0) and M'^{-1} (table 1) within a few
  // decay lengths of the walls, exact, over a window of wall_wd nodes from
  // the wall ([2][wall_nl + wall_nr][wall_wd]); the other rows are the
  // periodic block-rows above
  const double* wrows;
  int32_t wall_nl, wall_nr, wall_wd, pad6;
  const double* h;                // [ns]
  const double* hx;               // [ns]
  // dynamic fields
  double* G;                      // [nb][T][3][NpP][16]
  float* G32;
  uint16_t* G16;                  // bfloat16 copy of G (same layout)
  double* invd;                   // [nb][T][NpP][16]
  double* sigx;                   // d sigma/dx at the element nodes, same layout (kinematics)
  int32_t* status;                // one word
  KrylovState* ks;
  double* H;                      // (m+1) x m Hessenberg, then cs[m], sn[m], g[m+1], y[m]
  double* part;                   // [nb][m+2] block partial sums
  double* V;                      // (m+1) x n
  double* Zb;                     // m x n
  double* w;                      // n
  double* b;                      // n
  double* tmp;                    // n
  double* xs;                     // n  solution accumulator
  double* wmass;                  // n  warm start of the mass solve
  double* side;                   // [4][nb][nl] line contributions of assembled outputs
  double* s1d;                    // [16][ns] 1D work arrays
  // FP32 inner-solve storage
  float* V32;
  float* Z32;
  float* w32;
  float* x32;
  float* b32;
  double* scal;                   // [64] small scalars (norms of the current solve)
  int32_t* prog;                  // progress word of the running Krylov cycle (host-visible), or null
  double* rk;                     // [9][ns] RK4 stage arrays: eta, phi, eta_x, phi_x, w~, slopes (2), sums (2)
  int32_t use_filter;             // the modal filter is on
  int32_t pad4;
  double* hist;                   // [4 stages][kHistSteps][n] stage-solution differences
  double* pv;                     // n: a stage's starting vector before extrapolation
  StageHistory* hs;
};

// ------------------------------------------------------------ batched launches
// Many tanks advance together: every launch of a batched Krylov step covers
// the workgroups of all tanks, listed in a table.  A work item names the tank
// and the block coordinates inside that tank's own grid, plus the x extent of
// that grid (the completion counters of the fused reductions count to it).
struct BatchItem {
  int32_t tank, bx, by, nbx;
};

// Arguments common to every batched launch.
struct BatchArgs {
  const TankDev* tanks;     // [count] copies of the tanks' descriptors
  const int32_t* live;      // [count] 1 while the tank takes part in the current solve
  const BatchItem* items;   // the launch's work items, one per workgroup
  const double* const* ptrs;   // [tables][count] the caller's per-tank surface and volume arrays
  int32_t count;
  int32_t pad;
};

// A surface array of a tank: one of its RK4 stage arrays (rk + k ns), or the
// caller's array from pointer table k.
enum : int32_t { SS_RK = 0, SS_PT = 1 };
struct SSel {
  int32_t kind, k;
};
__host__ __device__ inline double* svec(const BatchArgs& ba, const TankDev& d, int tank, SSel s) {
  return s.kind == SS_RK ? d.rk + (size_t)s.k * d.ns : const_cast<double*>(ba.ptrs[(size_t)s.k * ba.count + tank]);
}

// Start of every batched kernel: the workgroup reads its work item, returns
// unless its tank takes part in the solve, and then runs the single-tank code
// on that tank's own workspace (d).
#define SEM_BATCH_TANK(ba)                        \
  const BatchItem it_ = (ba).items[blockIdx.x];  \
  if (!(ba).live[it_.tank]) return;              \
  const TankDev& d = (ba).tanks[it_.tank];

// A vector of a tank's own workspace, named per launch.
enum : int32_t { BV_NONE = 0, BV_V, BV_Z, BV_W, BV_B, BV_XS, BV_TMP, BV_WMASS };
struct VSel {
  int32_t kind, col;        // col: column of V or Z
};

template <typename T>
__host__ __device__ inline T* bvec(const TankDev& d, VSel s);
template <>
__host__ __device__ inline double* bvec<double>(const TankDev& d, VSel s) {
  switch (s.kind) {
    case BV_V: return d.V + (int64_t)s.col * d.n;
    case BV_Z: return d.Zb + (int64_t)s.col * d.n;
    case BV_W: return d.w;
    case BV_B: return d.b;
    case BV_XS: return d.xs;
    case BV_TMP: return d.tmp;
    case BV_WMASS: return d.wmass;
    default: return nullptr;
  }
}
template <>
__host__ __device__ inline float* bvec<float>(const TankDev& d, VSel s) {
  switch (s.kind) {
    case BV_V: return d.V32 + (int64_t)s.col * d.n;
    case BV_Z: return d.Z32 + (int64_t)s.col * d.n;
    case BV_W: return d.w32;
    case BV_B: return d.b32;
    case BV_XS: return d.x32;
    default: return nullptr;
  }
}

// The norm of the Krylov vector V_j (j >= 1), kept in the scratch area after
// the Givens rotations and the right side of the tank's least-squares problem.
__host__ __device__ inline double* krylov_norm(const TankDev& d, int j) {
  const int m = d.m;
  return d.H + (size_t)(m + 1) * m + 2 * m + (m + 1) + (j - 1);
}

// Chunking of the fused reductions: at most 256 workgroups of >= 512 entries
// (1024 workgroups measured slower on the 2048-column tank: the last
// workgroup's pass over the partials grows with their count).
constexpr int64_t kDotMaxChunks = 256;
__host__ __device__ inline int64_t dot_chunk(int64_t n) {
  const int64_t c = (n + kDotMaxChunks - 1) / kDotMaxChunks;
  return c < 512 ? 512 : c;
}
__host__ __device__ inline int dot_nchunk(int64_t n) {
  const int64_t k = (n + dot_chunk(n) - 1) / dot_chunk(n);
  return k < 1 ? 1 : (int)k;
}

// Index of the element-node value of component c in the MFMA tile layout.
// FP32 copies: row order perm(m) = 16(m/16) + 4(m%4) + (m%16)/4 (the FP32
// 16x16x4 accumulator holds rows 4(lane/16)+v); FP64 copies keep the natural
// row order (the FP64 16x16x4 accumulator holds rows 4v+lane/16), see
// tile_index64.  Either way one (component, M-tile, v) load is 64 contiguous
// values.
__host__ __device__ inline int64_t tile_index(int T, int NpP, int64_t blk, int eb, int m, int ncomp,
                                              int c) {
  int tile = eb >> 4, e = eb & 15;
  int perm = (m >> 4) * 16 + (m & 3) * 4 + ((m & 15) >> 2);
  return (((blk * T + tile) * ncomp + c) * (int64_t)NpP + perm) * 16 + e;
}

__host__ __device__ inline int64_t tile_index64(int T, int NpP, int64_t blk, int eb, int m, int ncomp, int c) {
  int tile = eb >> 4, e = eb & 15;
  return (((blk * T + tile) * ncomp + c) * (int64_t)NpP + m) * 16 + e;
}

}  // namespace sem
