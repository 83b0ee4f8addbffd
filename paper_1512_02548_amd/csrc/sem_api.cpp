// C ABI of the library (include/sem.h): host-side mesh construction, workspace
// layout, and the drivers that sequence the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstring>
#include <map>
#include <type_traits>
#include <memory>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sem.h"
#include "host_refelem.hpp"
#include "launch.hpp"
#include "mesh.hpp"
#include "sem_internal.hpp"

using namespace sem;

// ------------------------------------------------------------ error state
static thread_local std::string g_err;
sem_status sem::fail(sem_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
extern "C" const char* sem_last_error(void) { return g_err.c_str(); }

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

template <class T>
static size_t put(sem_mesh* M, const char* name, const std::vector<T>& v) {
  size_t o = M->ws_bytes;
  Upload u;
  u.off = o;
  u.data.resize(v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(u.data.data(), v.data(), u.data.size());
  M->uploads.push_back(std::move(u));
  M->off[name] = o;
  M->ws_bytes = align256(o + v.size() * sizeof(T));
  return o;
}

static size_t reserve(sem_mesh* M, const char* name, size_t bytes) {
  size_t o = M->ws_bytes;
  M->off[name] = o;
  M->ws_bytes = align256(o + bytes);
  return o;
}

// pad an Np x Np matrix to NpP x NpP
static std::vector<double> pad(const Mat& A, int Np, int NpP) {
  std::vector<double> out((size_t)NpP * NpP, 0.0);
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) out[(size_t)i * NpP + j] = A[(size_t)i * Np + j];
  return out;
}
static std::vector<float> tof(const std::vector<double>& v) {
  std::vector<float> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
  return o;
}

// Runs f(0 .. n-1) on the host's hardware threads.
template <class F>
static void parallel_for(int n, F&& f) {
  int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
  nt = std::min(nt, std::max(1, n));
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int i = next++; i < n; i = next++) f(i);
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

// Build column template, tables, preconditioner blocks and the workspace layout.
static sem_status build_mesh(sem_mesh* M) {
  const int P = M->P, nz = M->nz, nx = M->nx;
  RefTri ref(P);
  Ref1D r1(P);
  M->Np = ref.Np;
  M->NpP = (ref.Np + 15) / 16 * 16;
  const int Np = M->Np, NpP = M->NpP;
  M->nl = P * nz + 1;
  M->nc = P * M->nl;
  const int nl = M->nl, nc = M->nc;
  M->n = (int64_t)nx * nc + (M->periodic ? 0 : nl);
  M->ns = (int64_t)nx * P + (M->periodic ? 0 : 1);
  M->E = (int64_t)2 * nx * nz;
  const double dX = M->L / nx;
  std::vector<double> sl(nz + 1);
  if (M->slev.empty())
    for (int j = 0; j <= nz; ++j) sl[j] = double(j) / nz;
  else
    sl = M->slev;

  // reference-node positions in the unit quad per triangle type:
  // lower (t=0): A=(0,0) B=(1,0) C=(1,1); upper (t=1): A=(0,0) B=(1,1) C=(0,1)
  std::vector<double> nodeq((size_t)2 * NpP * 2, 0.0);
  for (int t = 0; t < 2; ++t)
    for (int k = 0; k < Np; ++k) {
      double a = 0.5 * (1 + ref.r[k]), bb = 0.5 * (1 + ref.s[k]);
      double xi = t == 0 ? a + bb : a;
      double ze = t == 0 ? bb : a + bb;
      nodeq[((size_t)t * NpP + k) * 2 + 0] = xi;
      nodeq[((size_t)t * NpP + k) * 2 + 1] = ze;
    }
  // column-local numbering: left line by sigma, then interior in first-appearance order
  const double tol = 1e-9;
  std::vector<double> line_sig;
  for (int j = 0; j < nz; ++j)
    for (int t = 0; t < 2; ++t)
      for (int k = 0; k < Np; ++k) {
        double xi = nodeq[((size_t)t * NpP + k) * 2], ze = nodeq[((size_t)t * NpP + k) * 2 + 1];
        if (std::fabs(xi) < tol) line_sig.push_back(sl[j] + ze * (sl[j + 1] - sl[j]));
      }
  std::sort(line_sig.begin(), line_sig.end());
  std::vector<double> uniq;
  for (double v : line_sig)
    if (uniq.empty() || std::fabs(v - uniq.back()) > tol) uniq.push_back(v);
  if ((int)uniq.size() != nl) return fail(SEM_E_INVAL, "column template: unexpected line node count");
  auto line_index = [&](double sg) {
    for (int q = 0; q < nl; ++q)
      if (std::fabs(uniq[q] - sg) < tol) return q;
    return -1;
  };
  struct IP { double xi, sg; };
  std::vector<IP> interior;
  M->elem_loc.assign((size_t)2 * nz * NpP, -1);
  for (int j = 0; j < nz; ++j)
    for (int t = 0; t < 2; ++t)
      for (int k = 0; k < Np; ++k) {
        double xi = nodeq[((size_t)t * NpP + k) * 2], ze = nodeq[((size_t)t * NpP + k) * 2 + 1];
        double sg = sl[j] + ze * (sl[j + 1] - sl[j]);
        int loc;
        if (std::fabs(xi) < tol) loc = line_index(sg);
        else if (std::fabs(xi - 1.0) < tol) loc = nc + line_index(sg);
        else {
          loc = -1;
          for (size_t q = 0; q < interior.size(); ++q)
            if (std::fabs(interior[q].xi - xi) < tol && std::fabs(interior[q].sg - sg) < tol) loc = nl + (int)q;
          if (loc < 0) {
            interior.push_back({xi, sg});
            loc = nl + (int)interior.size() - 1;
          }
        }
        if (loc < 0) return fail(SEM_E_INVAL, "column template: node identification failed");
        M->elem_loc[(size_t)(j * 2 + t) * NpP + k] = loc;
      }
  if ((int)interior.size() + nl != nc) return fail(SEM_E_INVAL, "column template: unexpected interior count");
  // column-local coordinates
  std::vector<double> cx(nc + nl), cs(nc + nl);
  for (int q = 0; q < nl; ++q) {
    cx[q] = 0.0;
    cs[q] = uniq[q];
    cx[nc + q] = 1.0;
    cs[nc + q] = uniq[q];
  }
  for (size_t q = 0; q < interior.size(); ++q) {
    cx[nl + q] = interior[q].xi;
    cs[nl + q] = interior[q].sg;
  }
  M->is_surf_loc.assign(nc + nl, 0);
  for (int q = 0; q < nc + nl; ++q) M->is_surf_loc[q] = std::fabs(cs[q] - 1.0) < tol ? 1 : 0;
  // surface nodes of a column, ordered by x: left-line top first
  std::vector<std::pair<double, int>> sv;
  for (int q = 0; q < nc; ++q)
    if (M->is_surf_loc[q]) sv.push_back({cx[q], q});
  std::sort(sv.begin(), sv.end());
  if ((int)sv.size() != P) return fail(SEM_E_INVAL, "column template: surface count");
  M->surf_loc.resize(P);
  for (int k = 0; k < P; ++k) M->surf_loc[k] = sv[k].second;
  // accumulation table: contributions to column-local node q < nc
  M->acc_cnt.assign(nc, 0);
  M->acc_ent.assign((size_t)nc * kMaxContrib, 0);
  auto add = [&](int q, int code) -> bool {
    if (M->acc_cnt[q] >= kMaxContrib) return false;
    M->acc_ent[(size_t)q * kMaxContrib + M->acc_cnt[q]++] = code;
    return true;
  };
  for (int q = 0; q < nc; ++q) {
    for (int e = 0; e < 2 * nz; ++e)
      for (int k = 0; k < Np; ++k)
        if (M->elem_loc[(size_t)e * NpP + k] == q && !add(q, e * NpP + k))
          return fail(SEM_E_INVAL, "accumulation table overflow");
    if (q < nl)
      for (int e = 0; e < 2 * nz; ++e)
        for (int k = 0; k < Np; ++k)
          if (M->elem_loc[(size_t)e * NpP + k] == nc + q && !add(q, (1 << 30) | (e * NpP + k)))
            return fail(SEM_E_INVAL, "accumulation table overflow");
  }
  // the same table packed for the matrix-core stiffness kernels: per node
  // kMaxContrib 16-bit entries, the contribution's offset in the kernel's
  // element outputs (element-in-column x (NpP + 1) + node, below 2^15 for
  // nz <= 256) | previous column << 15, and one word count | surface << 4
  M->acc_pk.assign((size_t)nc * kMaxContrib, 0);
  M->acc_cm.assign(nc, 0);
  for (int q = 0; q < nc; ++q) {
    for (int k = 0; k < M->acc_cnt[q]; ++k) {
      const int e = M->acc_ent[(size_t)q * kMaxContrib + k];
      const int off = e & 0x3fffffff;
      const int pos = (off / NpP) * (NpP + 1) + off % NpP;
      if (pos >= (1 << 15)) return fail(SEM_E_INVAL, "packed accumulation table overflow");
      M->acc_pk[(size_t)q * kMaxContrib + k] = (uint16_t)(pos | (((e >> 30) & 1) << 15));
    }
    M->acc_cm[q] = (uint16_t)(M->acc_cnt[q] | (M->is_surf_loc[q] << 4));
  }
  // global coordinates
  M->node_x.assign(M->n, 0.0);
  M->node_sig.assign(M->n, 0.0);
  for (int c = 0; c < nx; ++c)
    for (int q = 0; q < nc; ++q) {
      M->node_x[(size_t)c * nc + q] = (c + cx[q]) * dX;
      M->node_sig[(size_t)c * nc + q] = cs[q];
    }
  if (!M->periodic)
    for (int q = 0; q < nl; ++q) {
      M->node_x[(size_t)nx * nc + q] = M->L;
      M->node_sig[(size_t)nx * nc + q] = cs[q];
    }
  M->surf_nodes.resize(M->ns);
  for (int c = 0; c < nx; ++c)
    for (int k = 0; k < P; ++k) M->surf_nodes[(size_t)c * P + k] = (int64_t)c * nc + M->surf_loc[k];
  if (!M->periodic) M->surf_nodes[M->ns - 1] = (int64_t)nx * nc + nl - 1;

  // per-layer geometry: Lam = d(r,s)/d(x,sigma), J
  std::vector<double> lay((size_t)2 * nz * 8, 0.0);
  for (int j = 0; j < nz; ++j) {
    double ds = sl[j + 1] - sl[j];
    for (int t = 0; t < 2; ++t) {
      // d(x,sig)/d(r,s) = [[(B-A)/2, (C-A)/2]] in physical units
      double bx = dX, bs = t == 0 ? 0.0 : ds;      // B - A
      double cxv = t == 0 ? dX : 0.0, csv = ds;    // C - A
      double a00 = bx / 2, a01 = cxv / 2, a10 = bs / 2, a11 = csv / 2;
      double det = a00 * a11 - a01 * a10;
      double* L = &lay[(size_t)(j * 2 + t) * 8];
      L[0] = a11 / det;   // dr/dx
      L[1] = -a01 / det;  // dr/dsig
      L[2] = -a10 / det;  // ds/dx
      L[3] = a00 / det;   // ds/dsig
      L[4] = det;         // |J|
      L[5] = sl[j];
      L[6] = ds;
    }
  }
  // column interpolation weights
  std::vector<double> colw((size_t)2 * NpP * (P + 1), 0.0);
  for (int t = 0; t < 2; ++t)
    for (int k = 0; k < Np; ++k) {
      Mat I = r1.interp_to({2.0 * nodeq[((size_t)t * NpP + k) * 2] - 1.0});
      for (int q = 0; q <= P; ++q) colw[((size_t)t * NpP + k) * (P + 1) + q] = I[q];
    }
  // block decomposition: a workgroup takes cb whole columns.  Up to four
  // 16-element MFMA tiles per workgroup (one per wavefront) while the tank
  // still gives at least 512 workgroups (two per CU); small tanks use one
  // tile per workgroup for parallelism.  Both element kernels must fit their
  // LDS (64 KiB): the reference kernel stages three element buffers, the
  // matrix-core kernel the operators (when they fit in 40 KiB), the element
  // table and one output buffer.
  {
    const int per_col = 2 * nz;
    const double tiles_total = (double)nx * per_col / 16.0;
    const int tt = M->tiles_req > 0 ? M->tiles_req : std::max(1, std::min(4, (int)(tiles_total / 512.0)));
    auto lds_ok = [&](int cb) {
      const size_t EB = (size_t)cb * per_col, T = (EB + 15) / 16;
      const size_t region = (size_t)cb * nc + nl;
      const size_t ref = (region + 3 * EB * NpP) * sizeof(double);
      const size_t ops = 4 * (size_t)NpP * NpP * sizeof(double);
      // (the seventh- and eighth-order FP64 operators, 72 KiB, sit in LDS
      // beside a block of at most 64 KiB; smaller operators count towards it)
      const size_t mfma = (ops <= 40 * 1024 ? ops : 0) + (size_t)per_col * NpP * 4 + 32 + region * sizeof(double) +
                          T * 16 * (NpP + 1) * sizeof(double);
      return ref <= 65536 && mfma <= 65536;
    };
    int cb = std::max(1, (16 * tt) / per_col);
    while (cb > 1 && !lds_ok(cb)) --cb;
    M->cb = std::min(cb, nx);
  }
  M->nb = (nx + M->cb - 1) / M->cb;
  M->EB = M->cb * 2 * nz;
  M->T = (M->EB + 15) / 16;

  // ---- preconditioner blocks from the still-water flat-bed operator at the mean depth
  double h0 = 0;
  for (double v : M->h) h0 += v;
  h0 /= (double)M->h.size();
  M->nclass_col = M->periodic ? 1 : 3;
  Mat MDr = matmul(ref.M, ref.Dr, Np, Np, Np), MDs = matmul(ref.M, ref.Ds, Np, Np, Np);
  auto elem_matrix = [&](int jt, bool mass) {
    const double* L = &lay[(size_t)jt * 8];
    Mat A((size_t)Np * Np, 0.0);
    if (mass) {
      for (size_t i = 0; i < A.size(); ++i) A[i] = L[4] * ref.M[i];
      return A;
    }
    double K00 = h0, K11 = 1.0 / h0;
    double grr = L[4] * (L[0] * L[0] * K00 + L[1] * L[1] * K11);
    double grs = L[4] * (L[0] * L[2] * K00 + L[1] * L[3] * K11);
    double gss = L[4] * (L[2] * L[2] * K00 + L[3] * L[3] * K11);
    // sum_ab G_ab D_a^T M D_b with constant G
    Mat DrT = transpose(ref.Dr, Np, Np), DsT = transpose(ref.Ds, Np, Np);
    Mat t1 = matmul(DrT, MDr, Np, Np, Np), t2 = matmul(DrT, MDs, Np, Np, Np);
    Mat t3 = matmul(DsT, MDr, Np, Np, Np), t4 = matmul(DsT, MDs, Np, Np, Np);
    for (size_t i = 0; i < A.size(); ++i) A[i] = grr * t1[i] + grs * (t2[i] + t3[i]) + gss * t4[i];
    return A;
  };
  // global node id of (column c, elem jt, node k)
  auto gnode = [&](int c, int jt, int k) -> int64_t {
    int loc = M->elem_loc[(size_t)jt * NpP + k];
    if (loc < nc) return (int64_t)c * nc + loc;
    int c2 = c + 1;
    if (c2 == nx) return M->periodic ? (int64_t)(loc - nc) : (int64_t)nx * nc + (loc - nc);
    return (int64_t)c2 * nc + (loc - nc);
  };
  // multiplicities (elements per node) of one column neighbourhood are enough; compute globally
  std::vector<int> mult(M->n, 0);
  for (int c = 0; c < nx; ++c)
    for (int jt = 0; jt < 2 * nz; ++jt)
      for (int k = 0; k < Np; ++k) mult[gnode(c, jt, k)]++;
  auto surf_global = [&](int64_t gi) {
    int64_t c = gi / nc;
    return M->is_surf_loc[gi - c * nc] != 0;
  };
  const int ncls = M->nclass_col * 2 * nz;
  std::vector<double> pre_lap((size_t)ncls * NpP * NpP, 0.0), pre_mass((size_t)ncls * NpP * NpP, 0.0);
  for (int cc = 0; cc < M->nclass_col; ++cc) {
    int crep = M->periodic ? 0 : (cc == 0 ? 0 : (cc == 2 ? nx - 1 : 1));
    if (!M->periodic && cc == 1 && nx < 3) continue;
    if (!M->periodic && cc == 2 && nx < 2) continue;
    std::set<int> cols;
    for (int dc = -1; dc <= 1; ++dc) {
      int c = crep + dc;
      if (M->periodic) c = ((c % nx) + nx) % nx;
      else if (c < 0 || c >= nx) continue;
      cols.insert(c);
    }
    for (int mass = 0; mass < 2; ++mass) {
      // assemble the patch
      std::map<int64_t, int> lid;
      for (int c : cols)
        for (int jt = 0; jt < 2 * nz; ++jt)
          for (int k = 0; k < Np; ++k) {
            int64_t gi = gnode(c, jt, k);
            if (!lid.count(gi)) {
              int id = (int)lid.size();
              lid[gi] = id;
            }
          }
      int nloc = (int)lid.size();
      Mat Ap((size_t)nloc * nloc, 0.0);
      for (int c : cols)
        for (int jt = 0; jt < 2 * nz; ++jt) {
          Mat Ae = elem_matrix(jt, mass != 0);
          for (int a = 0; a < Np; ++a)
            for (int b = 0; b < Np; ++b)
              Ap[(size_t)lid[gnode(c, jt, a)] * nloc + lid[gnode(c, jt, b)]] += Ae[(size_t)a * Np + b];
        }
      for (int jt = 0; jt < 2 * nz; ++jt) {
        std::vector<int> keep;
        for (int k = 0; k < Np; ++k)
          if (mass || !surf_global(gnode(crep, jt, k))) keep.push_back(k);
        int nk = (int)keep.size();
        Mat C((size_t)nk * nk);
        for (int a = 0; a < nk; ++a)
          for (int b = 0; b < nk; ++b)
            C[(size_t)a * nk + b] = Ap[(size_t)lid[gnode(crep, jt, keep[a])] * nloc + lid[gnode(crep, jt, keep[b])]];
        if (!invert(C, nk)) return fail(SEM_E_INVAL, "singular preconditioner block");
        std::vector<double>& dst = mass ? pre_mass : pre_lap;
        double* blk = &dst[(size_t)(cc * 2 * nz + jt) * NpP * NpP];
        for (int a = 0; a < nk; ++a)
          for (int b = 0; b < nk; ++b) {
            double wa = 1.0 / std::sqrt((double)mult[gnode(crep, jt, keep[a])]);
            double wb = 1.0 / std::sqrt((double)mult[gnode(crep, jt, keep[b])]);
            blk[(size_t)keep[a] * NpP + keep[b]] = wa * C[(size_t)a * nk + b] * wb;
          }
      }
    }
  }
  // ---- exact inverses for periodic tanks: column interiors condensed onto the
  // vertical lines, line system diagonalised by a DFT in x.  [0] still-water
  // Laplace operator on the free nodes (preconditioner), [1] 2D mass matrix.
  struct SDHost {
    int nI = 0, q = 0, M1 = 0, nMT1 = 0, KS1 = 0, nMT3 = 0, KS3 = 0, wall = 0;
    std::vector<int32_t> I_idx;
    std::vector<double> A1, C3, Shat;   // fragment-ordered factors, per-mode inverses
    std::vector<double> Wv, Hm, Qm;   // wall-line correction (tanks with walls)
  } sdh[2];
  // MFMA fragment order of a rows x cols row-major matrix: [M-tile][K-step][lane]
  auto fragments = [](const Mat& A, int rows, int cols, int* nmt, int* ks) {
    *nmt = (rows + 15) / 16;
    *ks = (cols + 3) / 4;
    std::vector<double> f((size_t)*nmt * *ks * 64, 0.0);
    for (int mt = 0; mt < *nmt; ++mt)
      for (int st = 0; st < *ks; ++st)
        for (int l = 0; l < 64; ++l) {
          int r = 16 * mt + l % 16, c = 4 * st + l / 16;
          if (r < rows && c < cols) f[((size_t)mt * *ks + st) * 64 + l] = A[(size_t)r * cols + c];
        }
    return f;
  };
  std::vector<double> twid;
  // exact inverses need the interior right sides of 16 columns in LDS (64 KiB)
  M->pre_kind = ((M->periodic || nx >= 2) && (size_t)((nc - nl + 3) / 4) * 4 * 16 * sizeof(double) <= 65536) ? 1 : 0;
  if (M->pre_kind == 1) {
    const int nloc = nc + nl;
    for (int which = 0; which < 2; ++which) {
      const bool lap = which == 0;
      SDHost& H = sdh[which];
      Mat A0c((size_t)nloc * nloc, 0.0);
      for (int jt = 0; jt < 2 * nz; ++jt) {
        Mat Ae = elem_matrix(jt, !lap);
        for (int a = 0; a < Np; ++a)
          for (int b = 0; b < Np; ++b)
            A0c[(size_t)M->elem_loc[(size_t)jt * NpP + a] * nloc + M->elem_loc[(size_t)jt * NpP + b]] +=
                Ae[(size_t)a * Np + b];
      }
      // line unknowns: sigma-ordered line nodes (the surface node is Dirichlet for the Laplace problem)
      const int q = lap ? nl - 1 : nl;
      for (int loc = nl; loc < nc; ++loc)
        if (!lap || !M->is_surf_loc[loc]) H.I_idx.push_back(loc);
      const int nI = (int)H.I_idx.size();
      H.q = q;
      H.nI = nI;
      std::vector<int> Gam(2 * q);
      for (int a = 0; a < q; ++a) {
        Gam[a] = a;
        Gam[q + a] = nc + a;
      }
      Mat Ainv((size_t)nI * nI, 0.0);
      for (int i = 0; i < nI; ++i)
        for (int j = 0; j < nI; ++j) Ainv[(size_t)i * nI + j] = A0c[(size_t)H.I_idx[i] * nloc + H.I_idx[j]];
      if (!invert(Ainv, nI)) return fail(SEM_E_INVAL, "singular column interior block");
      // line-interior couplings A_GI (2q x nI, lines left then right) and A_IG (nI x 2q)
      Mat AGI((size_t)2 * q * nI), AIG((size_t)nI * 2 * q);
      for (int a = 0; a < 2 * q; ++a)
        for (int i = 0; i < nI; ++i) {
          AGI[(size_t)a * nI + i] = A0c[(size_t)Gam[a] * nloc + H.I_idx[i]];
          AIG[(size_t)i * 2 * q + a] = A0c[(size_t)H.I_idx[i] * nloc + Gam[a]];
        }
      // condensation factor [A_II^-1; A_GI A_II^-1] and back-substitution factor A_II^-1 A_IG
      {
        Mat GA = matmul(AGI, Ainv, 2 * q, nI, nI);
        Mat A1((size_t)(nI + 2 * q) * nI);
        std::copy(Ainv.begin(), Ainv.end(), A1.begin());
        std::copy(GA.begin(), GA.end(), A1.begin() + (size_t)nI * nI);
        H.M1 = nI + 2 * q;
        H.A1 = fragments(A1, H.M1, nI, &H.nMT1, &H.KS1);
        Mat C = matmul(Ainv, AIG, nI, nI, 2 * q);
        H.C3 = fragments(C, nI, 2 * q, &H.nMT3, &H.KS3);
      }
      // Schur complement of the column on its two lines: S = A_GG - A_GI A_II^-1 A_IG
      Mat W = matmul(Ainv, AIG, nI, nI, 2 * q);   // nI x 2q
      Mat SW = matmul(AGI, W, 2 * q, nI, 2 * q);
      Mat S((size_t)4 * q * q);
      for (int a = 0; a < 2 * q; ++a)
        for (int b = 0; b < 2 * q; ++b)
          S[(size_t)a * 2 * q + b] = A0c[(size_t)Gam[a] * nloc + Gam[b]] - SW[(size_t)a * 2 * q + b];
      auto Sblk = [&](int A, int B, int a, int b) { return S[(size_t)(A * q + a) * 2 * q + B * q + b]; };
      // per-mode symbol S_LL + S_RR + S_LR e^{i k} + S_RL e^{-i k}, inverted;
      // the symbol of mode nx-k is the conjugate of mode k's (S is real)
      using cd = std::complex<double>;
      const int nk = nx / 2 + 1;
      std::vector<cd> Sinv((size_t)nk * q * q);
      std::atomic<bool> singular{false};
      parallel_for(nk, [&](int k) {
        double kap = 2.0 * M_PI * k / nx;
        cd ep(std::cos(kap), std::sin(kap)), em = std::conj(ep);
        std::vector<cd> Ak((size_t)q * q);
        cd* Ik = Sinv.data() + (size_t)k * q * q;
        for (int a = 0; a < q; ++a)
          for (int b = 0; b < q; ++b) {
            Ak[(size_t)a * q + b] = Sblk(0, 0, a, b) + Sblk(1, 1, a, b) + Sblk(0, 1, a, b) * ep + Sblk(1, 0, a, b) * em;
            Ik[(size_t)a * q + b] = a == b ? 1.0 : 0.0;
          }
        // complex Gauss-Jordan with partial pivoting
        for (int cc = 0; cc < q; ++cc) {
          int piv = cc;
          for (int rr = cc + 1; rr < q; ++rr)
            if (std::abs(Ak[(size_t)rr * q + cc]) > std::abs(Ak[(size_t)piv * q + cc])) piv = rr;
          if (std::abs(Ak[(size_t)piv * q + cc]) == 0.0) {
            singular = true;
            return;
          }
          if (piv != cc)
            for (int j = 0; j < q; ++j) {
              std::swap(Ak[(size_t)cc * q + j], Ak[(size_t)piv * q + j]);
              std::swap(Ik[(size_t)cc * q + j], Ik[(size_t)piv * q + j]);
            }
          cd inv = 1.0 / Ak[(size_t)cc * q + cc];
          for (int j = 0; j < q; ++j) {
            Ak[(size_t)cc * q + j] *= inv;
            Ik[(size_t)cc * q + j] *= inv;
          }
          for (int rr = 0; rr < q; ++rr) {
            if (rr == cc) continue;
            cd f = Ak[(size_t)rr * q + cc];
            if (f == 0.0) continue;
            for (int j = 0; j < q; ++j) {
              Ak[(size_t)rr * q + j] -= f * Ak[(size_t)cc * q + j];
              Ik[(size_t)rr * q + j] -= f * Ik[(size_t)cc * q + j];
            }
          }
        }
      });
      if (singular) return fail(SEM_E_INVAL, "singular line symbol");
      auto sinv = [&](int k, int a, int b) -> cd {
        if (k < nk) return Sinv[((size_t)k * q + a) * q + b];
        return std::conj(Sinv[((size_t)(nx - k) * q + a) * q + b]);
      };
      // modes k > nx/2 are the conjugates of modes nx - k: only 0..nx/2 are kept
      H.Shat.assign((size_t)nk * q * q * 2, 0.0);
      for (int k = 0; k < nk; ++k)
        for (int a = 0; a < q; ++a)
          for (int b = 0; b < q; ++b) {
            cd v = sinv(k, a, b);
            H.Shat[(((size_t)k * q + a) * q + b) * 2] = v.real();
            H.Shat[(((size_t)k * q + a) * q + b) * 2 + 1] = v.imag();
          }
      if (!M->periodic) {
        // Walls: the walled operator A_w is the periodic one A_p (line nx
        // identified with line 0) plus the jump v between lines nx and 0.
        // In the basis u = E u_p + F v (E copies line 0 onto line nx, F puts
        // v on line nx):  [A_p B12; B21 C] [u_p; v] = [E^T r; F^T r], solved
        // through the Schur complement Sc = C - B21 A_p^-1 B12 (q x q).  B12,
        // B21 and C are blocks of the last column's matrix (its right line is
        // line nx); A_p^-1 restricted to that column and line 0 follows from
        // the line Green's function G(d) = (1/nx) sum_k e^{i th_k d} S^_k^-1.
        H.wall = 1;
        auto A0 = [&](int r, int c) { return A0c[(size_t)r * nloc + c]; };
        Mat G0((size_t)q * q, 0.0), Gp((size_t)q * q, 0.0), Gm((size_t)q * q, 0.0);
        for (int k = 0; k < nx; ++k) {
          double th = 2.0 * M_PI * k / nx;
          cd e1(std::cos(th), std::sin(th));
          for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) {
              cd v = sinv(k, a, b);
              G0[(size_t)a * q + b] += v.real();
              Gp[(size_t)a * q + b] += (e1 * v).real();
              Gm[(size_t)a * q + b] += (std::conj(e1) * v).real();
            }
        }
        for (size_t t = 0; t < G0.size(); ++t) {
          G0[t] /= nx;
          Gp[t] /= nx;
          Gm[t] /= nx;
        }
        Mat B12L((size_t)q * q), B12R((size_t)q * q), B12I((size_t)nI * q);
        Mat B21L((size_t)q * q), B21R((size_t)q * q), B21I((size_t)q * nI);
        for (int a = 0; a < q; ++a)
          for (int j = 0; j < q; ++j) {
            B12L[(size_t)a * q + j] = A0(Gam[a], Gam[q + j]);
            B12R[(size_t)a * q + j] = A0(Gam[q + a], Gam[q + j]);
            B21L[(size_t)j * q + a] = A0(Gam[q + j], Gam[a]);
            B21R[(size_t)j * q + a] = A0(Gam[q + j], Gam[q + a]);
          }
        for (int i = 0; i < nI; ++i)
          for (int j = 0; j < q; ++j) {
            B12I[(size_t)i * q + j] = A0(H.I_idx[i], Gam[q + j]);
            B21I[(size_t)j * nI + i] = A0(Gam[q + j], H.I_idx[i]);
          }
        auto mv = [](const Mat& A, const std::vector<double>& x, int rows, int cols) {
          std::vector<double> y(rows, 0.0);
          for (int r = 0; r < rows; ++r) {
            double t = 0;
            for (int c = 0; c < cols; ++c) t += A[(size_t)r * cols + c] * x[c];
            y[r] = t;
          }
          return y;
        };
        Mat ALI((size_t)q * nI), ARI((size_t)q * nI), AIL((size_t)nI * q), AIR((size_t)nI * q);
        for (int a = 0; a < q; ++a)
          for (int i = 0; i < nI; ++i) {
            ALI[(size_t)a * nI + i] = AGI[(size_t)a * nI + i];
            ARI[(size_t)a * nI + i] = AGI[(size_t)(q + a) * nI + i];
            AIL[(size_t)i * q + a] = AIG[(size_t)i * 2 * q + a];
            AIR[(size_t)i * q + a] = AIG[(size_t)i * 2 * q + q + a];
          }
        Mat Sc = B12R;   // C = the right line's own block
        for (int j = 0; j < q; ++j) {
          std::vector<double> rL(q), rI(nI), rR(q);
          for (int a = 0; a < q; ++a) {
            rL[a] = B12L[(size_t)a * q + j];
            rR[a] = B12R[(size_t)a * q + j];
          }
          for (int i = 0; i < nI; ++i) rI[i] = B12I[(size_t)i * q + j];
          std::vector<double> y = mv(Ainv, rI, nI, nI);
          std::vector<double> gL = mv(ALI, y, q, nI), gR = mv(ARI, y, q, nI);
          for (int a = 0; a < q; ++a) {
            gL[a] = rL[a] - gL[a];
            gR[a] = rR[a] - gR[a];
          }
          std::vector<double> xL = mv(G0, gL, q, q), t1 = mv(Gm, gR, q, q);
          std::vector<double> xR = mv(Gp, gL, q, q), t2 = mv(G0, gR, q, q);
          for (int a = 0; a < q; ++a) {
            xL[a] += t1[a];
            xR[a] += t2[a];
          }
          std::vector<double> u1 = mv(AIL, xL, nI, q), u2 = mv(AIR, xR, nI, q);
          for (int i = 0; i < nI; ++i) u1[i] += u2[i];
          std::vector<double> u3 = mv(Ainv, u1, nI, nI);
          std::vector<double> xI(nI);
          for (int i = 0; i < nI; ++i) xI[i] = y[i] - u3[i];
          std::vector<double> c1 = mv(B21L, xL, q, q), c2 = mv(B21I, xI, q, nI), c3 = mv(B21R, xR, q, q);
          for (int a = 0; a < q; ++a) Sc[(size_t)a * q + j] -= c1[a] + c2[a] + c3[a];
        }
        if (!invert(Sc, q)) return fail(SEM_E_INVAL, "singular wall Schur complement");
        Mat Q = matmul(Ainv, B12I, nI, nI, q);                // nI x q
        Mat PhiL = B12L, PhiR = B12R;
        {
          Mat LQ = matmul(ALI, Q, q, nI, q), RQ = matmul(ARI, Q, q, nI, q);
          for (size_t t = 0; t < PhiL.size(); ++t) {
            PhiL[t] -= LQ[t];
            PhiR[t] -= RQ[t];
          }
        }
        // v = Sc^-1 (r_w - B21 y) with y on the last column from the first
        // solve: lines nx-1 and 0 (x_a, x_b) and interior y_I - C_L x_a - C_R x_b.
        // Folded into one row-major q x (3q + nI) matrix acting on
        // [r_w; x_a; x_b; y_I]:  [Sc^-1 | -Sc^-1 (B21L - B21I C_L) | -Sc^-1 (B21R - B21I C_R) | -Sc^-1 B21I]
        {
          Mat CL((size_t)nI * q), CR((size_t)nI * q);
          for (int i = 0; i < nI; ++i)
            for (int a = 0; a < q; ++a) {
              CL[(size_t)i * q + a] = W[(size_t)i * 2 * q + a];
              CR[(size_t)i * q + a] = W[(size_t)i * 2 * q + q + a];
            }
          Mat BL = matmul(B21I, CL, q, nI, q), BR = matmul(B21I, CR, q, nI, q);
          for (size_t t = 0; t < BL.size(); ++t) {
            BL[t] = B21L[t] - BL[t];
            BR[t] = B21R[t] - BR[t];
          }
          Mat V2 = matmul(Sc, BL, q, q, q), V3 = matmul(Sc, BR, q, q, q), V4 = matmul(Sc, B21I, q, q, nI);
          const int np = 3 * q + nI;
          H.Wv.assign((size_t)q * np, 0.0);
          for (int a = 0; a < q; ++a) {
            for (int b = 0; b < q; ++b) {
              H.Wv[(size_t)a * np + b] = Sc[(size_t)a * q + b];
              H.Wv[(size_t)a * np + q + b] = -V2[(size_t)a * q + b];
              H.Wv[(size_t)a * np + 2 * q + b] = -V3[(size_t)a * q + b];
            }
            for (int i = 0; i < nI; ++i) H.Wv[(size_t)a * np + 3 * q + i] = -V4[(size_t)a * nI + i];
          }
        }
        // y_I of the last column -= Q v  (column-major: threads over the interior rows)
        H.Qm.assign((size_t)q * nI, 0.0);
        for (int i = 0; i < nI; ++i)
          for (int a = 0; a < q; ++a) H.Qm[(size_t)a * nI + i] = Q[(size_t)i * q + a];
        // H_k = S^_k^-1 (e^{i th_k} Phi_L + Phi_R), column-major per mode
        // modes k > nx/2 are the conjugates of modes nx - k: only 0..nx/2 are kept
        H.Hm.assign((size_t)nk * q * q * 2, 0.0);
        parallel_for(nk, [&](int k) {
          double th = 2.0 * M_PI * k / nx;
          cd e1(std::cos(th), std::sin(th));
          for (int i = 0; i < q; ++i)
            for (int a = 0; a < q; ++a) {
              cd t = 0;
              for (int b = 0; b < q; ++b)
                t += sinv(k, i, b) * (e1 * PhiL[(size_t)b * q + a] + PhiR[(size_t)b * q + a]);
              H.Hm[(((size_t)k * q + a) * q + i) * 2] = t.real();
              H.Hm[(((size_t)k * q + a) * q + i) * 2 + 1] = t.imag();
            }
        });
      }
    }
    // long tanks: transforms along x as two passes of n1- and n2-point
    // products (nx = n1 n2, n1 the largest divisor with 8 <= n1 <= sqrt(nx))
    M->fft_n1 = M->fft_n2 = 0;
    if (nx >= 256) {
      for (int a = (int)std::sqrt((double)nx); a >= 8; --a)
        if (nx % a == 0) {
          M->fft_n1 = a;
          M->fft_n2 = nx / a;
          break;
        }
    }
    twid.resize((size_t)2 * nx);
    for (int mm = 0; mm < nx; ++mm) {
      twid[2 * mm] = std::cos(2.0 * M_PI * mm / nx);
      twid[2 * mm + 1] = -std::sin(2.0 * M_PI * mm / nx);
    }
  }
  for (int w = 0; w < 2; ++w) {
    M->sd_nI[w] = sdh[w].nI;
    M->sd_q[w] = sdh[w].q;
    M->sd_M1[w] = sdh[w].M1;
    M->sd_nMT1[w] = sdh[w].nMT1;
    M->sd_KS1[w] = sdh[w].KS1;
    M->sd_nMT3[w] = sdh[w].nMT3;
    M->sd_KS3[w] = sdh[w].KS3;
    M->sd_wall[w] = sdh[w].wall;
  }
  // ---- 1D operators
  const int P1 = P + 1;
  Mat S1 = matmul(r1.M, r1.D, P1, P1, P1);
  Ref1D rf(M->Pf);
  Mat If = r1.interp_to(rf.r);
  Mat Filt = filter_matrix(P, M->ic, M->sf);
  // 1D projections applied as exact rows: first block-rows of M'^{-1} and
  // M'^{-1} S_x from the block symbol of the periodic operators (blocks of
  // the P nodes e*P..e*P+P-1 of element e).  With walls these are the rows of
  // every node farther than the rows' decay band from both walls; the rows
  // near the walls follow below from the walled M'.
  std::vector<double> Brow, Rrow, wrows;
  M->circ1d = 1;
  if (M->circ1d) {
    using cd = std::complex<double>;
    const int ns1 = (int)M->ns;
    const double Je = 0.5 * dX;
    // A(0), A(+1), A(-1) blocks of M' and S_x
    Mat Dm((size_t)P * P, 0.0), Um((size_t)P * P, 0.0), Lm((size_t)P * P, 0.0);
    Mat Ds_((size_t)P * P, 0.0), Us((size_t)P * P, 0.0), Ls((size_t)P * P, 0.0);
    for (int a = 0; a <= P; ++a)
      for (int b = 0; b <= P; ++b) {
        double mv = Je * r1.M[(size_t)a * P1 + b], sv = S1[(size_t)a * P1 + b];
        // element e holds nodes eP+a; a = P is node 0 of block e+1
        int ba = a == P ? 1 : 0, ia = a == P ? 0 : a;
        int bb = b == P ? 1 : 0, ib = b == P ? 0 : b;
        int off = bb - ba;   // block offset of the column relative to the row
        Mat& Mt = off == 0 ? Dm : (off == 1 ? Um : Lm);
        Mat& St = off == 0 ? Ds_ : (off == 1 ? Us : Ls);
        Mt[(size_t)ia * P + ib] += mv;
        St[(size_t)ia * P + ib] += sv;
      }
    std::vector<cd> Bk((size_t)nx * P * P), Rk((size_t)nx * P * P);
    for (int k = 0; k < nx; ++k) {
      double kap = 2.0 * M_PI * k / nx;
      cd ep(std::cos(kap), std::sin(kap)), em = std::conj(ep);
      std::vector<cd> C((size_t)P * P), Sx((size_t)P * P), I((size_t)P * P, 0.0);
      for (int i = 0; i < P * P; ++i) {
        C[i] = Dm[i] + Um[i] * ep + Lm[i] * em;
        Sx[i] = Ds_[i] + Us[i] * ep + Ls[i] * em;
      }
      for (int a = 0; a < P; ++a) I[(size_t)a * P + a] = 1.0;
      for (int cc = 0; cc < P; ++cc) {
        int piv = cc;
        for (int rr = cc + 1; rr < P; ++rr)
          if (std::abs(C[(size_t)rr * P + cc]) > std::abs(C[(size_t)piv * P + cc])) piv = rr;
        if (piv != cc)
          for (int j = 0; j < P; ++j) {
            std::swap(C[(size_t)cc * P + j], C[(size_t)piv * P + j]);
            std::swap(I[(size_t)cc * P + j], I[(size_t)piv * P + j]);
          }
        cd inv = 1.0 / C[(size_t)cc * P + cc];
        for (int j = 0; j < P; ++j) {
          C[(size_t)cc * P + j] *= inv;
          I[(size_t)cc * P + j] *= inv;
        }
        for (int rr = 0; rr < P; ++rr) {
          if (rr == cc) continue;
          cd f = C[(size_t)rr * P + cc];
          for (int j = 0; j < P; ++j) {
            C[(size_t)rr * P + j] -= f * C[(size_t)cc * P + j];
            I[(size_t)rr * P + j] -= f * I[(size_t)cc * P + j];
          }
        }
      }
      for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) {
          Bk[((size_t)k * P + a) * P + b] = I[(size_t)a * P + b];
          cd acc = 0;
          for (int c2 = 0; c2 < P; ++c2) acc += I[(size_t)a * P + c2] * Sx[(size_t)c2 * P + b];
          Rk[((size_t)k * P + a) * P + b] = acc;
        }
    }
    Brow.assign((size_t)P * ns1, 0.0);
    Rrow.assign((size_t)P * ns1, 0.0);
    std::vector<cd> tw(nx);
    for (int mm = 0; mm < nx; ++mm) tw[mm] = cd(std::cos(-2.0 * M_PI * mm / nx), std::sin(-2.0 * M_PI * mm / nx));
    for (int dd = 0; dd < nx; ++dd)
      for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) {
          cd sb = 0, sr = 0;
          int idx = 0;   // (k dd) mod nx
          for (int k = 0; k < nx; ++k, idx = (idx + dd) % nx) {
            const cd& e = tw[idx];
            sb += Bk[((size_t)k * P + a) * P + b] * e;
            sr += Rk[((size_t)k * P + a) * P + b] * e;
          }
          Brow[(size_t)a * ns1 + dd * P + b] = sb.real() / nx;
          Rrow[(size_t)a * ns1 + dd * P + b] = sr.real() / nx;
        }
    // The rows decay geometrically away from the diagonal (about a decade per
    // element): the applies skip the elements farther than `circ_band`, where
    // every entry is below 1e-15 of its row's largest and the first skipped
    // ones, four elements further out, below ~1e-19 (under the rounding of
    // the sums themselves).  Short tanks keep every element.
    int reach = 0;
    for (const std::vector<double>* R : {&Brow, &Rrow})
      for (int a = 0; a < P; ++a) {
        double mx = 0;
        for (int j = 0; j < ns1; ++j) mx = std::max(mx, std::fabs((*R)[(size_t)a * ns1 + j]));
        for (int j = 0; j < ns1; ++j) {
          const int dd = j / P, dist = std::min(dd, nx - dd);
          if (std::fabs((*R)[(size_t)a * ns1 + j]) > 1e-15 * mx) reach = std::max(reach, dist);
        }
      }
    M->circ_band = std::min(reach + 4, nx);   // elements on each side; 2 band + 1 >= nx: all
    if (!M->periodic) {
      // Walled M' (banded, half-bandwidth P) and S_x, assembled from the
      // element matrices; rows of M'^{-1} from a banded Cholesky factor
      // (M' e_s solves; M' is symmetric), rows of M'^{-1} S_x as S_x^T
      // applied to them.  Rows of the nodes in the W elements next to each
      // wall are kept explicitly over the window of nodes they reach.
      const int band = M->circ_band, W = band + 2;
      const bool all = 2 * W + 1 >= nx;
      M->wall_nl = all ? ns1 : W * P;
      M->wall_nr = all ? 0 : W * P + 1;
      M->wall_wd = all ? ns1 : std::min(ns1, (W + band + 1) * P + 1);
      const int hb = P;
      std::vector<double> Mb((size_t)ns1 * (hb + 1), 0.0);   // Mb[i][k] = M'(i, i - k)
      std::vector<double> Sd((size_t)ns1 * (2 * hb + 1), 0.0);   // Sd[i][hb + j - i] = S_x(i, j)
      for (int e = 0; e < nx; ++e)
        for (int a = 0; a <= P; ++a)
          for (int b = 0; b <= P; ++b) {
            const int i = e * P + a, j = e * P + b;
            if (j <= i) Mb[(size_t)i * (hb + 1) + (i - j)] += Je * r1.M[(size_t)a * P1 + b];
            Sd[(size_t)i * (2 * hb + 1) + hb + j - i] += S1[(size_t)a * P1 + b];
          }
      std::vector<double> Lb((size_t)ns1 * (hb + 1), 0.0);   // Cholesky factor, same band layout
      for (int i = 0; i < ns1; ++i)
        for (int j = std::max(0, i - hb); j <= i; ++j) {
          double sum = Mb[(size_t)i * (hb + 1) + (i - j)];
          for (int k = std::max(0, i - hb); k < j; ++k)
            sum -= Lb[(size_t)i * (hb + 1) + (i - k)] * Lb[(size_t)j * (hb + 1) + (j - k)];
          if (i == j) {
            if (!(sum > 0)) return fail(SEM_E_INVAL, "internal: 1D mass matrix not positive definite");
            Lb[(size_t)i * (hb + 1)] = std::sqrt(sum);
          } else {
            Lb[(size_t)i * (hb + 1) + (i - j)] = sum / Lb[(size_t)j * (hb + 1)];
          }
        }
      const int nr = M->wall_nl + M->wall_nr, wd = M->wall_wd;
      wrows.assign((size_t)2 * nr * wd, 0.0);
      std::vector<double> z(ns1), y(ns1);
      for (int rr = 0; rr < nr; ++rr) {
        const int srow = rr < M->wall_nl ? rr : ns1 - M->wall_nr + (rr - M->wall_nl);
        const int t0 = rr < M->wall_nl ? 0 : ns1 - wd;
        // M' z = e_srow: L y = e, L^T z = y
        for (int i = 0; i < ns1; ++i) {
          double sum = i == srow ? 1.0 : 0.0;
          for (int k = std::max(0, i - hb); k < i; ++k) sum -= Lb[(size_t)i * (hb + 1) + (i - k)] * y[k];
          y[i] = sum / Lb[(size_t)i * (hb + 1)];
        }
        for (int i = ns1 - 1; i >= 0; --i) {
          double sum = y[i];
          for (int k = i + 1; k <= std::min(ns1 - 1, i + hb); ++k) sum -= Lb[(size_t)k * (hb + 1) + (k - i)] * z[k];
          z[i] = sum / Lb[(size_t)i * (hb + 1)];
        }
        for (int t = 0; t < wd; ++t) {
          const int j = t0 + t;
          // (S_x^T z)_j = sum_i S_x(i, j) z_i over |i - j| <= hb
          double r = 0;
          for (int i = std::max(0, j - hb); i <= std::min(ns1 - 1, j + hb); ++i)
            r += Sd[(size_t)i * (2 * hb + 1) + hb + j - i] * z[i];
          wrows[((size_t)0 * nr + rr) * wd + t] = r;
          wrows[((size_t)1 * nr + rr) * wd + t] = z[j];
        }
      }
    }
  }

  // ---- workspace layout: constants
  M->ws_bytes = 0;
  M->uploads.clear();
  reserve(M, "tank", sizeof(TankDev));
  reserve(M, "scal", 64 * sizeof(double));
  std::vector<double> Drp = pad(ref.Dr, Np, NpP), Dsp = pad(ref.Ds, Np, NpP);
  std::vector<double> MDrp = pad(MDr, Np, NpP), MDsp = pad(MDs, Np, NpP), Mp = pad(ref.M, Np, NpP);
  put(M, "Dr", Drp);
  put(M, "Ds", Dsp);
  put(M, "MDr", MDrp);
  put(M, "MDs", MDsp);
  put(M, "M", Mp);
  put(M, "Dr32", tof(Drp));
  put(M, "Ds32", tof(Dsp));
  put(M, "MDr32", tof(MDrp));
  put(M, "MDs32", tof(MDsp));
  put(M, "M32", tof(Mp));
  // Operators of the matrix-core stiffness kernel in MFMA fragment order.
  // Stage 1 (A = [Dr; Ds], 16x4 A tiles): [mt][s][op][lane] holds
  // D_op[16 mt + l%16][4 s + l/16].  Stage 2 (A = (M D_op)^T): [mt][v][mo][op][lane]
  // holds (M D_op)[16 mt + row(v, l/16)][16 mo + l%16], with the accumulator
  // row map of the instruction: 4v + g for FP64, 4g + v for FP32.
  {
    const int MTt = NpP / 16, KSt = NpP / 4;
    const std::vector<double> zero((size_t)NpP * NpP, 0.0);
    auto frag = [&](bool fp64, bool sz = false) {
      std::vector<double> f((size_t)4 * NpP * NpP, 0.0);
      const std::vector<double>* D1[2] = {&Drp, &Dsp};
      const std::vector<double>* D2[2] = {sz ? &Mp : &MDrp, sz ? &zero : &MDsp};
      size_t o = 0;
      for (int mt = 0; mt < MTt; ++mt)
        for (int st = 0; st < KSt; ++st)
          for (int w = 0; w < 2; ++w)
            for (int l = 0; l < 64; ++l) f[o++] = (*D1[w])[(size_t)(16 * mt + l % 16) * NpP + 4 * st + l / 16];
      for (int mt = 0; mt < MTt; ++mt)
        for (int v = 0; v < 4; ++v)
          for (int mo = 0; mo < MTt; ++mo)
            for (int w = 0; w < 2; ++w)
              for (int l = 0; l < 64; ++l) {
                const int g = l / 16;
                const int row = fp64 ? 4 * v + g : 4 * g + v;
                f[o++] = (*D2[w])[(size_t)(16 * mt + row) * NpP + 16 * mo + l % 16];
              }
      return f;
    };
    put(M, "opf", frag(true));
    put(M, "opf32", tof(frag(false)));
    // S_z (w~ recovery): the same stage 1; stage 2 applies M (symmetric)
    put(M, "opf_sz", frag(true, true));
  }
  put(M, "elem_loc", M->elem_loc);
  put(M, "acc_cnt", M->acc_cnt);
  put(M, "acc_ent", M->acc_ent);
  put(M, "acc_pk", M->acc_pk);
  put(M, "acc_cm", M->acc_cm);
  put(M, "surf_loc", M->surf_loc);
  put(M, "is_surf_loc", M->is_surf_loc);
  put(M, "lay", lay);
  put(M, "nodeq", nodeq);
  put(M, "colw", colw);
  put(M, "pre_lap", pre_lap);
  put(M, "pre_mass", pre_mass);
  put(M, "pre_lap32", tof(pre_lap));
  put(M, "M1", r1.M);
  put(M, "S1", S1);
  put(M, "Ifine", If);
  put(M, "Mfine", rf.M);
  put(M, "Filt", Filt);
  put(M, "Brow", Brow);
  put(M, "Rrow", Rrow);
  if (wrows.empty()) wrows.assign(1, 0.0);
  put(M, "wrows", wrows);
  put(M, "h", M->h);
  put(M, "hx", M->hx);
  put(M, "twid", twid);
  for (int w = 0; w < 2; ++w) {
    std::string p = w == 0 ? "sd0_" : "sd1_";
    SDHost& H = sdh[w];
    put(M, (p + "I_idx").c_str(), H.I_idx);
    // the per-mode inverses are uploaded column-major
    {
      std::vector<double> St(H.Shat.size());
      const size_t qq = (size_t)H.q * H.q;
      const size_t nks = H.Shat.size() / (2 * std::max<size_t>(qq, 1));
      for (size_t k = 0; k < nks; ++k)
        for (int a = 0; a < H.q; ++a)
          for (int b = 0; b < H.q; ++b)
            for (int ri = 0; ri < 2; ++ri)
              St[((k * qq) + (size_t)b * H.q + a) * 2 + ri] = H.Shat[((k * qq) + (size_t)a * H.q + b) * 2 + ri];
      H.Shat.swap(St);
    }
    put(M, (p + "A1").c_str(), H.A1);
    put(M, (p + "C3").c_str(), H.C3);
    put(M, (p + "Shat").c_str(), H.Shat);
    put(M, (p + "A1_32").c_str(), tof(H.A1));
    put(M, (p + "C3_32").c_str(), tof(H.C3));
    put(M, (p + "Shat32").c_str(), tof(H.Shat));
    put(M, (p + "Wv").c_str(), H.Wv);
    put(M, (p + "Hm").c_str(), H.Hm);
    put(M, (p + "Qm").c_str(), H.Qm);
    reserve(M, (p + "vbuf").c_str(), (size_t)std::max(1, H.q) * sizeof(double));
    reserve(M, (p + "WP").c_str(), (size_t)2 * std::max(1, H.q) * sizeof(double));
    const size_t lbytes = (size_t)nx * std::max(1, H.q) * sizeof(double);
    const size_t fbytes = M->fft_n1 ? lbytes : 8;
    reserve(M, (p + "FT").c_str(), 2 * fbytes);
    reserve(M, (p + "FG").c_str(), 2 * fbytes);
    reserve(M, (p + "XL").c_str(), lbytes);
    reserve(M, (p + "yI").c_str(), (size_t)nx * std::max(1, H.nI) * sizeof(double));
    reserve(M, (p + "TL").c_str(), (size_t)nx * std::max(1, H.q) * sizeof(double));
    reserve(M, (p + "TR").c_str(), (size_t)nx * std::max(1, H.q) * sizeof(double));
    reserve(M, (p + "XH").c_str(), (size_t)nx * std::max(1, H.q) * 2 * sizeof(double));
  }
  // dynamic
  const int m = M->m;
  const size_t n = (size_t)M->n, ns1 = (size_t)M->ns;
  const size_t tiles = (size_t)M->nb * M->T * 16 * NpP;
  int nchunk;
  int64_t chunk;
  dot_layout(M->n, &nchunk, &chunk);
  const int ldp = m + 2;
  reserve(M, "G", tiles * 3 * sizeof(double));
  reserve(M, "probe", 512 * sizeof(double));
  reserve(M, "G32", tiles * 3 * sizeof(float));
  reserve(M, "G16", tiles * 3 * sizeof(uint16_t));
  reserve(M, "invd", tiles * sizeof(double));
  reserve(M, "sigx", tiles * sizeof(double));
  reserve(M, "status", 64);
  reserve(M, "ks", sizeof(KrylovState));
  reserve(M, "H", ((size_t)(m + 1) * m + 5 * m + 1) * sizeof(double));
  reserve(M, "part", (size_t)std::max<int64_t>(nchunk, M->nb) * ldp * sizeof(double));
  reserve(M, "V", (size_t)(m + 1) * n * sizeof(double));
  reserve(M, "Z", (size_t)m * n * sizeof(double));
  reserve(M, "w", n * sizeof(double));
  reserve(M, "b", n * sizeof(double));
  reserve(M, "tmp", n * sizeof(double));
  reserve(M, "xs", n * sizeof(double));
  reserve(M, "wmass", n * sizeof(double));
  reserve(M, "side", (size_t)4 * M->nb * nl * sizeof(double));
  reserve(M, "s1d", 16 * ns1 * sizeof(double));
  reserve(M, "rk", 16 * ns1 * sizeof(double));
  reserve(M, "hist", (size_t)4 * kHistSteps * n * sizeof(double));
  reserve(M, "pv", n * sizeof(double));
  reserve(M, "hs", sizeof(StageHistory));
  reserve(M, "V32", (size_t)(m + 1) * n * sizeof(float));
  reserve(M, "Z32", (size_t)m * n * sizeof(float));
  reserve(M, "w32", n * sizeof(float));
  reserve(M, "x32", n * sizeof(float));
  reserve(M, "b32", n * sizeof(float));
  return SEM_OK;
}

extern "C" sem_status sem_mesh_create(const sem_mesh_desc* desc, sem_mesh** out) {
  if (!desc || !out) return fail(SEM_E_INVAL, "null argument");
  *out = nullptr;
  if (desc->nx < 1 || desc->nz < 1) return fail(SEM_E_INVAL, "nx and nz must be >= 1");
  if (desc->nz > kMaxLayers) return fail(SEM_E_INVAL, "nz must be <= 256");
  if (desc->order < 1 || desc->order > kMaxOrder) return fail(SEM_E_INVAL, "order must be in 1..8");
  if (!(desc->length > 0)) return fail(SEM_E_INVAL, "length must be positive");
  if (desc->periodic && desc->nx < 2) return fail(SEM_E_INVAL, "a periodic tank needs nx >= 2");
  if (desc->filter_ic < 2 || desc->filter_ic > desc->order + 1)
    return fail(SEM_E_INVAL, "filter_ic must be in 2..order+1 (vertex modes are never filtered)");
  if (desc->overint_order < desc->order || desc->overint_order > 32)
    return fail(SEM_E_INVAL, "overint_order must be in order..32");
  if (!desc->h || !desc->h_x) return fail(SEM_E_INVAL, "h and h_x are required");
  std::unique_ptr<sem_mesh> M(new (std::nothrow) sem_mesh());
  if (!M) return fail(SEM_E_NOMEM, "host allocation failed");
  M->nx = desc->nx;
  M->nz = desc->nz;
  M->P = desc->order;
  M->periodic = desc->periodic ? 1 : 0;
  M->L = desc->length;
  M->g = desc->g;
  M->ic = desc->filter_ic;
  M->sf = desc->filter_sigma;
  M->Pf = desc->overint_order;
  M->m = desc->restart > 0 ? desc->restart : 30;
  if (desc->variant < 0 || desc->variant > 1) return fail(SEM_E_INVAL, "variant must be 0 or 1");
  M->variant = desc->variant;
  if (desc->tiles_per_block < 0 || desc->tiles_per_block > 4) return fail(SEM_E_INVAL, "tiles_per_block must be in 0..4");
  M->tiles_req = desc->tiles_per_block;
  if (M->m > kMaxRestart) return fail(SEM_E_INVAL, "restart must be <= 64");
  int64_t ns = (int64_t)M->nx * M->P + (M->periodic ? 0 : 1);
  M->h.assign(desc->h, desc->h + ns);
  M->hx.assign(desc->h_x, desc->h_x + ns);
  for (double v : M->h)
    if (!(v > 0)) return fail(SEM_E_INVAL, "still-water depth must be positive");
  if (desc->sigma_levels) {
    M->slev.assign(desc->sigma_levels, desc->sigma_levels + M->nz + 1);
    if (M->slev[0] != 0.0 || M->slev[M->nz] != 1.0) return fail(SEM_E_INVAL, "sigma_levels must run from 0 to 1");
    for (int j = 0; j < M->nz; ++j)
      if (!(M->slev[j + 1] > M->slev[j])) return fail(SEM_E_INVAL, "sigma_levels must increase");
  }
  sem_status s;
  try {
    s = build_mesh(M.get());
  } catch (const std::exception& e) {
    return fail(SEM_E_INVAL, e.what());
  }
  if (s != SEM_OK) return s;
  *out = M.release();
  return SEM_OK;
}

extern "C" sem_status sem_mesh_query(const sem_mesh* M, sem_mesh_info* out) {
  if (!M || !out) return fail(SEM_E_INVAL, "null argument");
  out->n = M->n;
  out->ns = M->ns;
  out->n_free = M->n - M->ns;
  out->n_elem = M->E;
  out->np = M->Np;
  out->nblocks = M->nb;
  out->workspace_bytes = M->ws_bytes;
  return SEM_OK;
}

extern "C" sem_status sem_mesh_node_coords(const sem_mesh* M, double* x, double* sg) {
  if (!M || !x || !sg) return fail(SEM_E_INVAL, "null argument");
  std::memcpy(x, M->node_x.data(), M->n * sizeof(double));
  std::memcpy(sg, M->node_sig.data(), M->n * sizeof(double));
  return SEM_OK;
}

extern "C" sem_status sem_mesh_surface_nodes(const sem_mesh* M, int64_t* idx) {
  if (!M || !idx) return fail(SEM_E_INVAL, "null argument");
  std::memcpy(idx, M->surf_nodes.data(), M->ns * sizeof(int64_t));
  return SEM_OK;
}

extern "C" void sem_mesh_destroy(sem_mesh* M) { delete M; }

extern "C" sem_status sem_reference_operators(int32_t P, int32_t Pf, int32_t ic, double sigma_f, double* r,
                                              double* s, double* Dr, double* Ds, double* Mm, double* F,
                                              double* I, double* Mf) {
  if (P < 1 || P > 10 || Pf < P || Pf > 32) return fail(SEM_E_INVAL, "need 1 <= P <= 10 and P <= Pf <= 32");
  if (ic < 2) return fail(SEM_E_INVAL, "filter cut-off must leave the vertex modes alone (ic >= 2)");
  const RefTri ref(P);
  auto out = [](double* dst, const std::vector<double>& v) {
    if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(double));
  };
  out(r, ref.r);
  out(s, ref.s);
  out(Dr, ref.Dr);
  out(Ds, ref.Ds);
  out(Mm, ref.M);
  const Ref1D r1(P), rf(Pf);
  out(F, filter_matrix(P, ic, sigma_f));
  out(I, r1.interp_to(rf.r));
  out(Mf, rf.M);
  return SEM_OK;
}

template <class T>
static T* at(sem_mesh* M, const char* name) {
  return reinterpret_cast<T*>(M->ws + M->off.at(name));
}

extern "C" sem_status sem_mesh_bind(sem_mesh* M, void* workspace, size_t bytes, void* stream) {
  if (!M || !workspace) return fail(SEM_E_INVAL, "null argument");
  if (bytes < M->ws_bytes) return fail(SEM_E_NOMEM, "workspace smaller than sem_mesh_query reports");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(SEM_E_INVAL, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  if (!M->prog_host) {
    void* p = nullptr;
    HIPCHK(hipHostMalloc(&p, 256, hipHostMallocMapped | hipHostMallocCoherent));
    M->prog_host = (int32_t*)p;
    void* dp = nullptr;
    HIPCHK(hipHostGetDevicePointer(&dp, p, 0));
    M->prog_dev = (int32_t*)dp;
    *(volatile int32_t*)M->prog_host = 0;
  }
  if (!M->rb_host) HIPCHK(hipHostMalloc(&M->rb_host, 256, hipHostMallocDefault));
  HIPCHK(hipGetDevice(&M->device));
  // the stage solves' timing events, created once per mesh
  for (auto& e : M->solve_ev)
    for (auto& x : e)
      if (!x) HIPCHK(hipEventCreate(&x));
  M->ws = (char*)workspace;
  TankDev& h = M->hd;
  h = TankDev{};
  h.P = M->P;
  h.Np = M->Np;
  h.NpP = M->NpP;
  h.nx = M->nx;
  h.nz = M->nz;
  h.periodic = M->periodic;
  h.nl = M->nl;
  h.nc = M->nc;
  h.n = (int32_t)M->n;
  h.ns = (int32_t)M->ns;
  h.E = (int32_t)M->E;
  h.cb = M->cb;
  h.nb = M->nb;
  h.T = M->T;
  h.EB = M->EB;
  h.m = M->m;
  h.Pf = M->Pf;
  h.L = M->L;
  h.dX = M->L / M->nx;
  h.g = M->g;
  h.nclass_col = M->nclass_col;
  h.pre_kind = M->pre_kind;
  h.use_mfma = M->variant == 0 ? 1 : 0;
  h.Dr = at<double>(M, "Dr");
  h.Ds = at<double>(M, "Ds");
  h.MDr = at<double>(M, "MDr");
  h.MDs = at<double>(M, "MDs");
  h.opf = at<double>(M, "opf");
  h.opf32 = at<float>(M, "opf32");
  h.opf_sz = at<double>(M, "opf_sz");
  h.Mref = at<double>(M, "M");
  h.Dr32 = at<float>(M, "Dr32");
  h.Ds32 = at<float>(M, "Ds32");
  h.MDr32 = at<float>(M, "MDr32");
  h.MDs32 = at<float>(M, "MDs32");
  h.Mref32 = at<float>(M, "M32");
  h.elem_loc = at<int32_t>(M, "elem_loc");
  h.acc_cnt = at<int32_t>(M, "acc_cnt");
  h.acc_ent = at<int32_t>(M, "acc_ent");
  h.acc_pk = at<uint16_t>(M, "acc_pk");
  h.acc_cm = at<uint16_t>(M, "acc_cm");
  h.surf_loc = at<int32_t>(M, "surf_loc");
  h.is_surf_loc = at<int32_t>(M, "is_surf_loc");
  h.lay = at<double>(M, "lay");
  h.nodeq = at<double>(M, "nodeq");
  h.colw = at<double>(M, "colw");
  h.pre_lap = at<double>(M, "pre_lap");
  h.pre_mass = at<double>(M, "pre_mass");
  h.pre_lap32 = at<float>(M, "pre_lap32");
  h.twid = at<double>(M, "twid");
  for (int w = 0; w < 2; ++w) {
    std::string p = w == 0 ? "sd0_" : "sd1_";
    SDData& sd = h.sd[w];
    sd.nI = M->sd_nI[w];
    sd.q = M->sd_q[w];
    sd.zero_surface = w == 0 ? 1 : 0;
    sd.I_idx = at<int32_t>(M, (p + "I_idx").c_str());
    sd.M1 = M->sd_M1[w];
    sd.nMT1 = M->sd_nMT1[w];
    sd.KS1 = M->sd_KS1[w];
    sd.nMT3 = M->sd_nMT3[w];
    sd.KS3 = M->sd_KS3[w];
    sd.A1 = at<double>(M, (p + "A1").c_str());
    sd.C3 = at<double>(M, (p + "C3").c_str());
    sd.Shat = at<double>(M, (p + "Shat").c_str());
    sd.A1_32 = at<float>(M, (p + "A1_32").c_str());
    sd.C3_32 = at<float>(M, (p + "C3_32").c_str());
    sd.Shat32 = at<float>(M, (p + "Shat32").c_str());
    sd.yI = at<double>(M, (p + "yI").c_str());
    sd.TL = at<double>(M, (p + "TL").c_str());
    sd.TR = at<double>(M, (p + "TR").c_str());
    sd.XH = at<double>(M, (p + "XH").c_str());
    sd.wall = M->sd_wall[w];
    sd.Wv = at<double>(M, (p + "Wv").c_str());
    sd.Hm = at<double>(M, (p + "Hm").c_str());
    sd.Qm = at<double>(M, (p + "Qm").c_str());
    sd.vbuf = at<double>(M, (p + "vbuf").c_str());
    sd.WP = at<double>(M, (p + "WP").c_str());
    sd.fft_n1 = M->fft_n1;
    sd.fft_n2 = M->fft_n2;
    sd.FT = at<double>(M, (p + "FT").c_str());
    sd.FG = at<double>(M, (p + "FG").c_str());
    sd.XL = at<double>(M, (p + "XL").c_str());
  }
  h.M1 = at<double>(M, "M1");
  h.S1 = at<double>(M, "S1");
  h.Ifine = at<double>(M, "Ifine");
  h.Mfine = at<double>(M, "Mfine");
  h.Filt = at<double>(M, "Filt");
  h.circ1d = M->circ1d;
  h.circ_band = M->circ_band;
  h.Brow = at<double>(M, "Brow");
  h.Rrow = at<double>(M, "Rrow");
  h.wrows = at<double>(M, "wrows");
  h.wall_nl = M->wall_nl;
  h.wall_nr = M->wall_nr;
  h.wall_wd = M->wall_wd;
  h.h = at<double>(M, "h");
  h.hx = at<double>(M, "hx");
  h.G = at<double>(M, "G");
  h.G32 = at<float>(M, "G32");
  h.G16 = at<uint16_t>(M, "G16");
  h.invd = at<double>(M, "invd");
  h.sigx = at<double>(M, "sigx");
  h.status = at<int32_t>(M, "status");
  h.ks = at<KrylovState>(M, "ks");
  h.H = at<double>(M, "H");
  h.part = at<double>(M, "part");
  h.V = at<double>(M, "V");
  h.Zb = at<double>(M, "Z");
  h.w = at<double>(M, "w");
  h.b = at<double>(M, "b");
  h.tmp = at<double>(M, "tmp");
  h.xs = at<double>(M, "xs");
  h.wmass = at<double>(M, "wmass");
  h.side = at<double>(M, "side");
  h.s1d = at<double>(M, "s1d");
  h.V32 = at<float>(M, "V32");
  h.Z32 = at<float>(M, "Z32");
  h.w32 = at<float>(M, "w32");
  h.x32 = at<float>(M, "x32");
  h.b32 = at<float>(M, "b32");
  M->rk = at<double>(M, "rk");
  M->scal = at<double>(M, "scal");
  h.scal = M->scal;
  h.prog = M->prog_dev;
  h.rk = M->rk;
  h.use_filter = M->sf != 1.0 ? 1 : 0;
  h.hist = at<double>(M, "hist");
  h.pv = at<double>(M, "pv");
  h.hs = at<StageHistory>(M, "hs");
  M->dtank = at<TankDev>(M, "tank");
  // every device array the kernels use must have been laid out
  const void* need[] = {h.Dr, h.Ds, h.MDr, h.MDs, h.opf, h.opf32, h.opf_sz, h.Mref, h.Dr32, h.Ds32, h.MDr32, h.MDs32, h.Mref32, h.elem_loc,
                        h.acc_cnt, h.acc_ent, h.surf_loc, h.is_surf_loc, h.lay, h.nodeq, h.colw, h.pre_lap,
                        h.pre_mass, h.pre_lap32, h.M1, h.S1, h.Ifine, h.Mfine, h.Filt, h.h, h.hx, h.G,
                        h.G32, h.G16, h.invd, h.sigx, h.status, h.ks, h.H, h.part, h.V, h.Zb, h.w, h.b, h.tmp, h.xs,
                        h.wmass, h.side, h.s1d, h.V32, h.Z32, h.w32, h.x32, h.b32, h.twid, h.Brow, h.Rrow,
                        h.sd[0].yI, h.sd[1].yI, h.sd[0].A1, h.sd[1].A1, h.sd[0].C3, h.sd[1].C3, h.sd[0].XH,
                        h.sd[1].XH, M->rk, M->scal, h.hist, h.pv, h.hs};
  for (size_t i = 0; i < sizeof(need) / sizeof(need[0]); ++i)
    if (!need[i]) return fail(SEM_E_INVAL, "internal: workspace layout incomplete (" + std::to_string(i) + ")");
  for (const Upload& u : M->uploads)
    HIPCHK(hipMemcpyAsync(M->ws + u.off, u.data.data(), u.data.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(M->dtank, &h, sizeof(TankDev), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(h.status, 0, 64, st));
  // Krylov state, including the completion counter of the fused reductions
  HIPCHK(hipMemsetAsync(h.ks, 0, sizeof(KrylovState), st));
  HIPCHK(hipMemsetAsync(h.hs, 0, sizeof(StageHistory), st));
  HIPCHK(hipMemsetAsync(h.wmass, 0, M->n * sizeof(double), st));
  HIPCHK(hipMemsetAsync(h.G, 0, M->off.at("G32") - M->off.at("G"), st));
  HIPCHK(hipMemsetAsync(h.G32, 0, M->off.at("G16") - M->off.at("G32"), st));
  HIPCHK(hipMemsetAsync(h.G16, 0, M->off.at("invd") - M->off.at("G16"), st));
  HIPCHK(hipMemsetAsync(h.invd, 0, M->off.at("status") - M->off.at("invd"), st));
  if (M->relax_on)
    HIPCHK(hipMemcpyAsync(M->rk + 9 * (size_t)M->ns, M->relax_w.data(), M->ns * sizeof(double),
                          hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  M->bound = true;
  return SEM_OK;
}

// ------------------------------------------------------------ helpers
sem_status sem::check_bound(sem_mesh* M) {
  if (!M) return fail(SEM_E_INVAL, "null mesh");
  if (!M->bound) return fail(SEM_E_INVAL, "mesh not bound to a workspace");
  return SEM_OK;
}

sem_status sem::status_from_word(int32_t w) {
  if (w & ST_NONFINITE) return SEM_E_NONFINITE;
  if (w & ST_DOMAIN) return SEM_E_DOMAIN;
  if (w & ST_BREAKDOWN) return SEM_E_BREAKDOWN;
  if (w & ST_NOCONV) return SEM_E_NOCONV;
  return SEM_OK;
}

// Small device-to-host reads go through the mesh's pinned readback block.
static sem_status readback(sem_mesh* M, void* out, const void* dev, size_t bytes, hipStream_t st) {
  if (bytes > 256) return fail(SEM_E_INVAL, "readback larger than the pinned block");
  HIPCHK(hipMemcpyAsync(M->rb_host, dev, bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(out, M->rb_host, bytes);
  return SEM_OK;
}

static sem_status read_status(sem_mesh* M, hipStream_t st, int32_t* word) {
  int32_t w = 0;
  if (sem_status e = readback(M, &w, M->hd.status, sizeof(w), st)) return e;
  if (word) *word = w;
  sem_status s = status_from_word(w);
  if (s != SEM_OK) return fail(s, "device reported status " + std::to_string(w));
  return SEM_OK;
}

struct GmresCfg {
  int op, pre;
  bool mask;
  double rtol;
  int max_iter;
  int ahead;   // Krylov steps queued ahead of the device
  int gstore;   // FP32 path: 1 = FP32 factors, 2 = bfloat16 factors
  int ks_ready;   // the Krylov state was reset by the solve's first kernel
  int bnorm_ready;   // ||b||^2 is already in scal[1] (b fixed up), or comes with the first residual
  const double* bside = nullptr;   // FP64: b's shared-line contributions, fixed up by the first residual pass
  // FP64 Laplace solves: the end of the solve (Phi, the stage record) done by
  // the last cycle's update; `done` says whether it was
  struct End {
    const double* phis;
    double* phi;
    int stage;
    bool done;
  }* end = nullptr;
};

struct KrylovBuf {
  double *V, *Z, *w, *side;
};
struct KrylovBufF {
  float *V, *Z, *w, *side;
};

static void gather_t(sem_mesh* M, const GmresCfg& c, int op, const double* u, double* y, double* side, int flags,
                     hipStream_t st) {
  launch_gather(M->hd, M->dtank, op, u, y, side, flags, st);
}
static void gather_t(sem_mesh* M, const GmresCfg& c, int op, const float* u, float* y, float* side, int flags,
                     hipStream_t st) {
  launch_gather(M->hd, M->dtank, op, u, y, side, flags, c.gstore, st);
}

static void stiff_timed_launch(sem_mesh* M, const GmresCfg&, const double* u, double* y, double* side, int flags,
                               hipEvent_t e0, hipEvent_t e1, hipStream_t st, const StiffDots& dots) {
  launch_stiff_mfma_timed(M->hd, M->dtank, u, y, side, flags, e0, e1, st, dots);
}
static void stiff_timed_launch(sem_mesh* M, const GmresCfg& c, const float* u, float* y, float* side, int flags,
                               hipEvent_t e0, hipEvent_t e1, hipStream_t st, const StiffDots& dots) {
  launch_stiff_mfma_timed(M->hd, M->dtank, u, y, side, flags, c.gstore, e0, e1, st, dots);
}

// Stiffness application inside the Krylov loop, bracketed by timing events
// when enabled (the fix-up of shared lines runs after the end event).
// dots (matrix-core stiffness only): the inner products fused into the launch
template <typename T>
static sem_status stiff_timed(sem_mesh* M, const GmresCfg& cfg, const T* u, T* y, T* side, int flags,
                              hipStream_t st, const StiffDots* dots = nullptr) {
  const bool nofix = (flags & F_NOFIX) != 0;   // the caller adds the side buffer itself
  if (!M->kt_on || cfg.op != OP_STIFF) {
    if (dots) {
      stiff_timed_launch(M, cfg, u, y, side, flags, nullptr, nullptr, st, *dots);
      if (!nofix) launch_fixup(M->hd, M->dtank, y, side, flags, st);
    } else {
      gather_t(M, cfg, cfg.op, u, y, side, flags, st);
    }
    return SEM_OK;
  }
  if (M->kt_used == M->kt_ev.size()) {
    std::pair<hipEvent_t, hipEvent_t> e;
    HIPCHK(hipEventCreate(&e.first));
    HIPCHK(hipEventCreate(&e.second));
    M->kt_ev.push_back(e);
  }
  auto& e = M->kt_ev[M->kt_used++];
  if (M->hd.use_mfma) {
    // events stamped by the kernel's own dispatch
    stiff_timed_launch(M, cfg, u, y, side, flags, e.first, e.second, st, dots ? *dots : StiffDots{});
  } else {
    HIPCHK(hipEventRecord(e.first, st));
    gather_t(M, cfg, cfg.op, u, y, side, flags | F_NOFIX, st);
    HIPCHK(hipEventRecord(e.second, st));
  }
  if (!nofix) launch_fixup(M->hd, M->dtank, y, side, flags, st);
  return SEM_OK;
}

// Adds the first `real` recorded launches (the stream has been synchronised)
static sem_status stiff_harvest(sem_mesh* M, size_t real) {
  if (!M->kt_on) return SEM_OK;
  real = std::min(real, M->kt_used);
  for (size_t i = 0; i < real; ++i) {
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, M->kt_ev[i].first, M->kt_ev[i].second));
    M->kt_ms += t;
    M->kt_count += 1;
  }
  M->kt_used = 0;
  return SEM_OK;
}

// Restarted right-preconditioned GMRES (classical Gram-Schmidt, Givens
// rotations) on device vectors of type T: x (in: guess, out: solution), b.
// Inner products, the Hessenberg matrix and the rotations are FP64.
//
// The host queues Arnoldi steps without synchronising: every step's kernels
// return at once when the cycle is done, and the device publishes its
// progress to pinned host memory, so the host stops queueing when it sees
// convergence and never runs more than `ahead` steps in front of the device.
// The stream is synchronised once per cycle.
template <typename T, typename Buf>
static sem_status gmres(sem_mesh* M, const GmresCfg& cfg, const Buf& B, T* x, const T* b, int* iters_out,
                        double* relres_out, hipStream_t st) {
  const TankDev& h = M->hd;
  const TankDev* d = M->dtank;
  const int m = M->m;
  const int64_t n = M->n;
  const int ldp = m + 2;
  double* scal = M->scal;
  const int flags = cfg.mask ? 1 : 0;
  const int gflags = flags | F_GATE;
  const int ahead = std::max(1, cfg.ahead);
  volatile int32_t* prog = M->prog_host;
  M->kt_used = 0;
  if (!cfg.ks_ready) launch_ks_reset(h.ks, cfg.rtol, st);
  int32_t* cnt = &h.ks->pad[0];
  if (!cfg.bnorm_ready) launch_dots(n, 1, b, 0, b, h.part, ldp, scal + 1, cnt, nullptr, st);
  int total = 0;
  KrylovState hks{};
  bool first = true;
  while (true) {
    *prog = 0;
    // r = b - A x (the operator's shared-line fix-up folded into the residual)
    {
      sem_status e = stiff_timed(M, cfg, x, B.w, B.side, flags | F_NOFIX, st);
      if (e) return e;
    }
    if constexpr (std::is_same<T, double>::value) {
      launch_residual_cycle(h, d, n, b, B.w, B.side, B.V, cfg.mask ? 1 : 0, h.part, ldp, scal, cnt, h.ks, h.H, m,
                            first ? 1 : 0, h.status, M->prog_dev, st, first ? cfg.bside : nullptr);
    } else {
      launch_residual_cycle(h, d, n, b, B.w, B.side, B.V, cfg.mask ? 1 : 0, h.part, ldp, scal, cnt, h.ks, h.H, m,
                            first ? 1 : 0, h.status, M->prog_dev, st);
    }
    first = false;
    int32_t seen = 0;   // the progress word that ended the cycle
    // with the exact still-water inverse, V_j = w / h_{j,j-1} is formed while
    // the preconditioner reads w (no separate scaling launch)
    const bool fused = cfg.pre == OP_PRE_LAP && h.pre_kind == 1;
    const double* hnorm = h.H + (size_t)(m + 1) * m + 2 * m + (m + 1);   // norms of V_1.. (scratch of the Givens update)
    for (int j = 0; j < m && total + j < cfg.max_iter; ++j) {
      T* Vj = B.V + (size_t)j * n;
      T* Zj = B.Z + (size_t)j * n;
      if (fused && j > 0) launch_sd(h, d, 0, B.w, Zj, 1, st, hnorm + (j - 1), Vj);
      else gather_t(M, cfg, cfg.pre, Vj, Zj, B.side, gflags, st);
      double* Hcol = h.H + (size_t)j * (m + 1);
      // the matrix-core stiffness launch also forms the products with V_0..V_j
      // (from each block's own contributions); the shared-line fix-up of w is
      // then done as the orthogonalisation reads it, otherwise inside the
      // separate products
      // (not while the stiffness launches are timed: the timing is the plain
      // apply's)
      const bool fdots = h.use_mfma && cfg.op == OP_STIFF && !M->kt_on;
      const StiffDots dots{B.V, n, j + 1, ldp, h.part, Hcol, cnt};
      {
        sem_status e = stiff_timed(M, cfg, Zj, B.w, B.side, gflags | F_NOFIX, st, fdots ? &dots : nullptr);
        if (e) return e;
      }
      if (!fdots) launch_dots(n, j + 1, B.V, n, B.w, h.part, ldp, Hcol, cnt, h.ks, st, d, B.side);
      launch_orth_givens(n, j, B.V, h.H, m, B.w, h.part, ldp, h.ks, cnt, h.status, M->prog_dev, st,
                         fdots ? d : nullptr, fdots ? B.side : nullptr);
      if (!fused) launch_scale_next(n, j, B.w, B.V, h.H, m, h.ks, st);
      // wait while the device is more than `ahead` steps behind: spin on the
      // progress word; ask the runtime whether the queue drained only every
      // 100 us (a drained queue means the word is final)
      bool stop = false;
      auto tq = std::chrono::steady_clock::now();
      while (true) {
        int32_t v = *prog;
        if (v & PROG_DONE) {
          stop = true;
          seen = v;
          break;
        }
        if (j + 1 - (v & PROG_STEPS) <= ahead) break;
        auto now = std::chrono::steady_clock::now();
        if (now - tq > std::chrono::microseconds(100)) {
          tq = now;
          hipError_t q = hipStreamQuery(st);
          if (q == hipSuccess) {
            seen = *prog;
            stop = (seen & PROG_DONE) != 0;
            break;
          }
          if (q != hipErrorNotReady) HIPCHK(q);
        }
        __builtin_ia32_pause();
      }
      if (stop) break;
    }
    const bool last = (seen & PROG_CONV) && !M->kt_on;
    if constexpr (std::is_same<T, double>::value) {
      if (last && cfg.end) {
        launch_solve_update_fused(n, B.Z, h.H, m, h.ks, x, st, d, cfg.end->phis, cfg.end->phi, cfg.end->stage);
        cfg.end->done = true;
      } else {
        launch_solve_update_fused(n, B.Z, h.H, m, h.ks, x, st);
      }
    } else {
      launch_solve_update_fused(n, B.Z, h.H, m, h.ks, x, st);
    }
    if (last) {
      // converged: the progress block carries the final scalars (released
      // with the word), so no readback; the queued update runs in stream
      // order before anything that reads x
      const volatile double* sc = reinterpret_cast<const volatile double*>(M->prog_host) + 1;
      hks = KrylovState{};
      hks.resid = sc[0];
      hks.bnorm = sc[1];
      hks.iters = (int32_t)sc[2];
      hks.j = seen & PROG_STEPS;
      hks.done = hks.converged = 1;
      break;
    }
    if (sem_status e = readback(M, &hks, h.ks, sizeof(hks), st)) return e;
    {
      // the cycle's residual apply plus its executed steps; later ones were gated
      sem_status e = stiff_harvest(M, 1 + (size_t)std::max(0, hks.j));
      if (e) return e;
    }
    total = hks.iters;
    if (hks.status || hks.converged || total >= cfg.max_iter) break;
  }
  *iters_out = hks.iters;
  *relres_out = hks.bnorm > 0 ? hks.resid / hks.bnorm : 0.0;
  if (hks.status) return status_from_word(hks.status);
  if (!hks.converged) return SEM_E_NOCONV;
  return SEM_OK;
}

static sem_status set_status_bits(sem_mesh* M, int32_t bits, hipStream_t st) {
  int32_t w = 0;
  if (sem_status e = readback(M, &w, M->hd.status, sizeof(w), st)) return e;
  w |= bits;
  std::memcpy(M->rb_host, &w, sizeof(w));
  HIPCHK(hipMemcpyAsync(M->hd.status, M->rb_host, sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return SEM_OK;
}

static KrylovBuf buf64(sem_mesh* M) { return KrylovBuf{M->hd.V, M->hd.Zb, M->hd.w, M->hd.side}; }
static KrylovBufF buf32(sem_mesh* M) {
  return KrylovBufF{M->hd.V32, M->hd.Z32, M->hd.w32, reinterpret_cast<float*>(M->hd.side)};
}

void sem::default_opts(sem_solve_opts* o) {
  o->rtol = 1e-12;
  o->max_iter = 5000;
  o->prec = SEM_PREC_FP64;
  o->inner_rtol = 1e-4;
  o->max_refine = 30;
  o->warm_start = 0;
  o->lookahead = 2;
  o->predict = 5;
}

// ------------------------------------------------------------ public calls
extern "C" sem_status sem_set_surface(sem_mesh* M, const double* eta, const double* eta_x, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!eta || !eta_x) return fail(SEM_E_INVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(M->hd.status, 0, sizeof(int32_t), st));
  launch_coef(M->hd, M->dtank, eta, eta_x, 3, st);
  return read_status(M, st, nullptr);
}

extern "C" sem_status sem_kernel_timing(sem_mesh* M, int32_t enable) {
  if (!M) return fail(SEM_E_INVAL, "null mesh");
  M->kt_on = enable != 0;
  M->kt_used = 0;
  if (M->kt_on) {
    M->kt_count = 0;
    M->kt_ms = 0;
  }
  return SEM_OK;
}

extern "C" sem_status sem_kernel_timing_read(const sem_mesh* M, int64_t* launches, double* total_ms) {
  if (!M || !launches || !total_ms) return fail(SEM_E_INVAL, "null argument");
  *launches = M->kt_count;
  *total_ms = M->kt_ms;
  return SEM_OK;
}

extern "C" sem_status sem_apply(sem_mesh* M, sem_operator op, const double* u, double* y, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!u || !y) return fail(SEM_E_INVAL, "null argument");
  int kop;
  switch (op) {
    case SEM_OP_STIFFNESS: kop = 0; break;
    case SEM_OP_MASS2D: kop = 1; break;
    case SEM_OP_PRECOND: kop = 2; break;
    case SEM_OP_SZ: kop = 4; break;
    default: return fail(SEM_E_INVAL, "unknown operator");
  }
  hipStream_t st = (hipStream_t)stream;
  launch_gather(M->hd, M->dtank, kop, u, y, M->hd.side, 0, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return SEM_OK;
}

extern "C" sem_status sem_apply_timed(sem_mesh* M, sem_operator op, int32_t prec, const void* u, void* y,
                                      int32_t reps, float* ms, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!u || !y || !ms || reps < 1) return fail(SEM_E_INVAL, "bad argument");
  if (prec < 0 || prec > 2) return fail(SEM_E_INVAL, "unknown precision");
  if (prec != 0 && op != SEM_OP_STIFFNESS && op != SEM_OP_PRECOND)
    return fail(SEM_E_INVAL, "reduced precision exists for the stiffness and the preconditioner only");
  int kop;
  switch (op) {
    case SEM_OP_STIFFNESS: kop = 0; break;
    case SEM_OP_MASS2D: kop = 1; break;
    case SEM_OP_PRECOND: kop = 2; break;
    case SEM_OP_SZ: kop = 4; break;
    default: return fail(SEM_E_INVAL, "unknown operator");
  }
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  void* side = prec == 0 ? (void*)M->hd.side : (void*)M->hd.w32;
  launch_gather_only(M->hd, M->dtank, kop, prec, u, y, side, st);   // warm-up launch
  HIPCHK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) launch_gather_only(M->hd, M->dtank, kop, prec, u, y, side, st);
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float t = 0;
  HIPCHK(hipEventElapsedTime(&t, e0, e1));
  *ms = t / reps;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return SEM_OK;
}

extern "C" sem_status sem_selftest_mfma(sem_mesh* M, double* max_err, double* raw, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!max_err) return fail(SEM_E_INVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  double* o64 = at<double>(M, "probe");
  float* o32 = reinterpret_cast<float*>(o64 + 256);
  launch_mfma_probe(o64, o32, st);
  std::vector<double> h64(256);
  std::vector<float> h32(256);
  HIPCHK(hipMemcpyAsync(h64.data(), o64, 256 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(h32.data(), o32, 256 * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double err = 0;
  // expected accumulator rows: FP64 4v + lane/16 (interleaved), FP32 4(lane/16) + v
  auto D = [](int i, int j) {
    double ref = 0;
    for (int k = 0; k < 4; ++k) ref += (1.0 + i + 16.0 * k) * (1.0 + 2.0 * k + 3.0 * j);
    return ref;
  };
  for (int lane = 0; lane < 64; ++lane)
    for (int v = 0; v < 4; ++v) {
      int j = lane & 15, g = lane >> 4;
      err = std::max(err, std::fabs(h64[lane * 4 + v] - D(4 * v + g, j)));
      err = std::max(err, std::fabs((double)h32[lane * 4 + v] - D(4 * g + v, j)));
    }
  *max_err = err;
  if (raw)
    for (int i = 0; i < 256; ++i) {
      raw[i] = h64[i];
      raw[256 + i] = h32[i];
    }
  return SEM_OK;
}

// Laplace solve on the device with factors already set; phi in/out [n].
// FP64: GMRES on A_FF x = b.  FP32_IR / BF16_IR: FP64 iterative refinement,
// each correction from an FP32 GMRES solve (FP32 vectors and operators, FP32
// or bfloat16 geometric factors, FP64 inner products) scaled by ||r||.
// RK4 stage solves: the stage index, the extrapolation depth and dt of the
// start-vector predictor (the predictor and the record of the stage's
// change run inside the solve's timed span).
struct StagePredict {
  int stage, depth;
  double dt;
};

// Device time between the two events of a solve (0 if they cannot be read).
static double solve_seconds(hipEvent_t* ev) {
  float ms = 0;
  return (ev[0] && ev[1] && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) ? ms * 1e-3 : 0.0;
}

// A stage solve (pred set) neither waits for the device before it starts nor
// after it ends: its seconds come from the events around its launches, read
// by the RK4 step once the step has synchronised.  A single solve
// synchronises at its end and reports the host clock.
static sem_status laplace_core(sem_mesh* M, const double* phi_s, double* phi, const sem_solve_opts* o,
                               sem_solve_stats* stats, hipStream_t st, const StagePredict* pred = nullptr) {
  const TankDev& h = M->hd;
  const TankDev* d = M->dtank;
  const int64_t n = M->n;
  auto t0 = std::chrono::steady_clock::now();
  hipEvent_t* ev = M->solve_ev[pred ? pred->stage : 0];
  if (pred) HIPCHK(hipEventRecord(ev[0], st));
  const bool fp64 = o->prec == SEM_PREC_FP64;
  // u = [0; phi~], the start vector xs (warm start, stage predictor), the
  // Krylov state; then b = -(A u)_F
  launch_solve_begin(h, d, phi_s, h.tmp, o->warm_start ? phi : nullptr, pred ? pred->stage : -1,
                     pred ? pred->depth : 0, pred ? pred->dt : 0.0, o->rtol, fp64 ? 1 : 0, st);
  // FP64: the lift's shared-line contributions go to a second side buffer
  // (the operator applies of the cycles use the first); the first residual
  // pass fixes b up and forms ||b||^2
  double* bside = h.side + 2 * (size_t)h.nb * h.nl;
  if (fp64) {
    launch_gather(h, d, OP_STIFF, h.tmp, h.b, bside, F_MASK_SURF | F_NEG | F_NOFIX, st);
  } else {
    launch_gather(h, d, OP_STIFF, h.tmp, h.b, h.side, F_MASK_SURF | F_NEG, st);
  }
  int iters = 0, refinements = 0;
  double rel = 0;
  sem_status s = SEM_OK;
  GmresCfg::End end{phi_s, phi, pred ? pred->stage : -1, false};
  if (fp64) {
    GmresCfg cfg{OP_STIFF, OP_PRE_LAP, true, o->rtol, o->max_iter, o->lookahead, 0, 1, 1};
    cfg.bside = bside;
    cfg.end = &end;
    s = gmres(M, cfg, buf64(M), h.xs, h.b, &iters, &rel, st);
  } else {
    const int ldp = M->m + 2;
    double* scal = M->scal;
    double nb2 = 0, rr = 0;
    int32_t* cnt = &h.ks->pad[0];
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t), st));
    launch_dots(n, 1, h.b, 0, h.b, h.part, ldp, scal + 4, cnt, nullptr, st);
    if (sem_status e = readback(M, &nb2, scal + 4, sizeof(nb2), st)) return e;
    double bnorm = std::sqrt(nb2);
    GmresCfg cfg{OP_STIFF, OP_PRE_LAP, true, o->inner_rtol, 0, o->lookahead, o->prec == SEM_PREC_BF16_IR ? 2 : 1};
    s = SEM_E_NOCONV;
    for (int k = 0; k <= o->max_refine; ++k) {
      // FP64 residual r = b - A x
      launch_gather(h, d, OP_STIFF, h.xs, h.w, h.side, F_MASK_SURF, st);
      launch_residual(h, d, n, h.b, h.w, h.tmp, 1, st);
      launch_dots(n, 1, h.tmp, 0, h.tmp, h.part, ldp, scal + 4, cnt, nullptr, st);
      if (sem_status e = readback(M, &rr, scal + 4, sizeof(rr), st)) return e;
      double rn = std::sqrt(rr);
      rel = bnorm > 0 ? rn / bnorm : rn;
      if (!std::isfinite(rn)) {
        s = SEM_E_NONFINITE;
        break;
      }
      if (rn <= o->rtol * bnorm || rn == 0.0) {
        s = SEM_OK;
        break;
      }
      if (k == o->max_refine || iters >= o->max_iter) break;
      launch_to_float(n, h.tmp, 1.0 / rn, h.b32, st);
      launch_fill_f(n, h.x32, st);
      cfg.max_iter = o->max_iter - iters;
      cfg.rtol = inner_tolerance(o->inner_rtol, o->rtol, bnorm, rn);
      int it = 0;
      double rr32 = 0;
      sem_status si = gmres(M, cfg, buf32(M), h.x32, h.b32, &it, &rr32, st);
      iters += it;
      refinements++;
      if (si != SEM_OK && si != SEM_E_NOCONV) {
        s = si;
        break;
      }
      launch_add_float(n, h.x32, rn, h.xs, st);
    }
  }
  if (s == SEM_E_NOCONV) set_status_bits(M, ST_NOCONV, st);
  // Phi = x_F + lift; a stage solve's change into the record
  if (!end.done) launch_solve_end(h, d, phi_s, phi, pred ? pred->stage : -1, st);
  if (pred) {
    HIPCHK(hipEventRecord(ev[1], st));
  } else {
    HIPCHK(hipStreamSynchronize(st));
  }
  if (stats) {
    stats->iters = iters;
    stats->refinements = refinements;
    stats->rel_residual = rel;
    stats->seconds = pred ? 0.0 : std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->status = s;
  }
  return s;
}

extern "C" sem_status sem_laplace_solve(sem_mesh* M, const double* eta, const double* eta_x, const double* phi_s,
                                        double* phi, const sem_solve_opts* opts, sem_solve_stats* stats,
                                        void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!eta || !eta_x || !phi_s || !phi) return fail(SEM_E_INVAL, "null argument");
  sem_solve_opts o;
  if (opts) o = *opts;
  else default_opts(&o);
  if (!(o.rtol > 0) || o.max_iter < 1) return fail(SEM_E_INVAL, "rtol > 0 and max_iter >= 1 required");
  if (o.prec < 0 || o.prec > 2) return fail(SEM_E_INVAL, "unknown precision");
  if (o.prec != SEM_PREC_FP64 && !(o.inner_rtol > 0 && o.inner_rtol < 1))
    return fail(SEM_E_INVAL, "inner_rtol must lie in (0, 1)");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(M->hd.status, 0, sizeof(int32_t), st));
  launch_coef(M->hd, M->dtank, eta, eta_x, 3, st);
  s = read_status(M, st, nullptr);
  if (s) return s;
  return laplace_core(M, phi_s, phi, &o, stats, st);
}

// x = M^-1 rhs for the constant 2D mass matrix: exactly (line condensation
// and DFT) on periodic tanks, preconditioned GMRES to 1e-14 with walls
// (x holds the start vector there)
static sem_status mass_solve(sem_mesh* M, const double* rhs, double* x, hipStream_t st) {
  const TankDev& h = M->hd;
  const TankDev* d = M->dtank;
  if (h.pre_kind == 1) {
    launch_gather(h, d, OP_PRE_MASS, rhs, x, h.side, 0, st);
    return SEM_OK;
  }
  GmresCfg cfg{OP_MASS, OP_PRE_MASS, false, 1e-14, 400, 4, 0};
  int iters;
  double rel;
  sem_status s = gmres(M, cfg, buf64(M), x, rhs, &iters, &rel, st);
  if (s == SEM_E_NOCONV) set_status_bits(M, ST_NOCONV, st);
  return s;
}

sem_status sem::recover_w_core(sem_mesh* M, const double* Phi, double* out, hipStream_t st) {
  const TankDev& h = M->hd;
  const TankDev* d = M->dtank;
  launch_gather(h, d, OP_SZ, Phi, h.b, h.side, 0, st);
  sem_status s = mass_solve(M, h.b, h.wmass, st);
  launch_gather_surface(h, d, h.wmass, out, st);
  return s;
}

extern "C" sem_status sem_recover_kinematics(sem_mesh* M, const double* Phi, const double* eta,
                                             const double* eta_x, double* u, double* w, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!Phi || !eta || !eta_x || (!u && !w)) return fail(SEM_E_INVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const TankDev& h = M->hd;
  const TankDev* d = M->dtank;
  HIPCHK(hipMemsetAsync(h.status, 0, sizeof(int32_t), st));
  // 1/d and d sigma/dx at the element nodes
  launch_coef(h, d, eta, eta_x, 2 | 4, st);
  if ((s = read_status(M, st, nullptr))) return s;
  const int ops[2] = {OP_SZ, OP_SU};
  double* outs[2] = {w, u};
  for (int k = 0; k < 2; ++k) {
    if (!outs[k]) continue;
    launch_gather(h, d, ops[k], Phi, h.b, h.side, 0, st);
    launch_fill(M->n, 0.0, outs[k], st);
    if ((s = mass_solve(M, h.b, outs[k], st))) return s;
  }
  return read_status(M, st, nullptr);
}

extern "C" sem_status sem_gradient_recover(sem_mesh* M, sem_recover_kind kind, const double* in, const double* eta,
                                           double* out, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!in || !out) return fail(SEM_E_INVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(M->hd.status, 0, sizeof(int32_t), st));
  if (kind == SEM_RECOVER_DX) {
    launch_recover_dx(M->hd, M->dtank, in, out, nullptr, nullptr, st);
    return read_status(M, st, nullptr);
  }
  if (kind != SEM_RECOVER_W) return fail(SEM_E_INVAL, "unknown recovery kind");
  if (!eta) return fail(SEM_E_INVAL, "eta required for w recovery");
  launch_coef(M->hd, M->dtank, eta, nullptr, 2, st);
  s = read_status(M, st, nullptr);
  if (s) return s;
  s = recover_w_core(M, in, out, st);
  if (s) return s;
  return read_status(M, st, nullptr);
}

extern "C" sem_status sem_free_surface_rhs(sem_mesh* M, const double* eta, const double* eta_x, const double* phi_x,
                                           const double* w_s, double* deta, double* dphi, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!eta || !eta_x || !phi_x || !w_s || !deta || !dphi) return fail(SEM_E_INVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(M->hd.status, 0, sizeof(int32_t), st));
  launch_fs_rhs(M->hd, M->dtank, eta, eta_x, phi_x, w_s, deta, dphi, st);
  return read_status(M, st, nullptr);
}

extern "C" sem_status sem_rk4_reset_history(sem_mesh* M, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  HIPCHK(hipMemsetAsync(M->hd.hs, 0, sizeof(StageHistory), (hipStream_t)stream));
  return SEM_OK;
}

// One RK4 step; qa (device, [3][2][ns]: eta_a and phi~_a at t, t + dt/2 and
// t + dt) adds the relaxation-zone source of Sec. 2.2 with tau = dt.
static sem_status rk4_step_core(sem_mesh* M, double* eta, double* phi_s, double* phi_ws, double dt, const double* qa,
                                const sem_solve_opts* opts, sem_solve_stats* stats, void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!eta || !phi_s || !phi_ws) return fail(SEM_E_INVAL, "null argument");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(SEM_E_INVAL, "dt must be positive");
  sem_solve_opts o;
  if (opts) o = *opts;
  else default_opts(&o);
  if (o.predict < 0 || o.predict > kHistSteps) return fail(SEM_E_INVAL, "predict must be in 0..6");
  hipStream_t st = (hipStream_t)stream;
  const TankDev& h = M->hd;
  const TankDev* d = M->dtank;
  const int ns = (int)M->ns;
  double* rk = M->rk;
  double* ye = rk + 0 * ns;   // stage state
  double* yp = rk + 1 * ns;
  double* ex = rk + 2 * ns;   // eta_x
  double* px = rk + 3 * ns;   // phi_x
  double* wsf = rk + 4 * ns;  // w~
  double* ke = rk + 5 * ns;   // stage slopes
  double* kp = rk + 6 * ns;
  double* ae = rk + 7 * ns;   // accumulated slopes
  double* ap = rk + 8 * ns;
  HIPCHK(hipMemsetAsync(h.status, 0, sizeof(int32_t), st));
  const double cnode[4] = {0.0, 0.5, 0.5, 1.0};
  const double wts[4] = {1.0 / 6, 2.0 / 6, 2.0 / 6, 1.0 / 6};
  sem_solve_opts lo = o;
  lo.warm_start = 1;
  sem_status first_err = SEM_OK;
  int solved = 0;   // stage solves launched (their events are current)
  for (int sidx = 0; sidx < 4; ++sidx) {
    const double* se = sidx == 0 ? eta : ye;
    const double* sp = sidx == 0 ? phi_s : yp;
    launch_recover_dx(h, d, se, ex, sp, px, st);
    // a non-positive water column found here ends the stage solve at its
    // first cycle (the solve's kernels read the status word), so the step
    // does not wait for the device before the solve
    launch_coef(h, d, se, ex, 3, st);
    sem_solve_stats ls{};
    const StagePredict pred{sidx, o.predict, dt};
    s = laplace_core(M, sp, phi_ws, &lo, &ls, st, &pred);
    ++solved;
    if (stats) stats[sidx] = ls;
    if (s) {
      first_err = s;
      break;
    }
    s = recover_w_core(M, phi_ws, wsf, st);
    if (s) {
      first_err = s;
      break;
    }
    launch_fs_rhs(h, d, se, ex, px, wsf, ke, kp, st);
    if (qa) {
      const int slot = sidx == 0 ? 0 : (sidx == 3 ? 2 : 1);
      launch_relax(ns, 1.0 / dt, M->rk + 9 * (size_t)ns, qa + (size_t)slot * 2 * ns, qa + ((size_t)slot * 2 + 1) * ns,
                   se, sp, ke, kp, st);
    }
    if (sidx < 3)
      launch_rk4_stage(ns, cnode[sidx + 1] * dt, wts[sidx], sidx == 0, eta, phi_s, ke, kp, ye, yp, ae, ap, st);
    else
      launch_rk4_stage(ns, 0.0, wts[sidx], 0, eta, phi_s, ke, kp, ye, yp, ae, ap, st);
  }
  if (first_err) {
    (void)hipStreamSynchronize(st);
    if (stats)
      for (int k = 0; k < solved; ++k) stats[k].seconds = solve_seconds(M->solve_ev[k]);
    return first_err;
  }
  launch_rk4_final(h, d, dt, ae, ap, eta, phi_s, M->sf != 1.0 ? 1 : 0, st);
  s = read_status(M, st, nullptr);
  if (stats)
    for (int k = 0; k < solved; ++k) stats[k].seconds = solve_seconds(M->solve_ev[k]);
  return s;
}

extern "C" sem_status sem_rk4_step(sem_mesh* M, double* eta, double* phi_s, double* phi_ws, double dt,
                                   const sem_solve_opts* opts, sem_solve_stats* stats, void* stream) {
  return rk4_step_core(M, eta, phi_s, phi_ws, dt, nullptr, opts, stats, stream);
}

extern "C" sem_status sem_set_relaxation(sem_mesh* M, const double* weight) {
  if (!M) return fail(SEM_E_INVAL, "null argument");
  if (!weight) {
    M->relax_on = false;
    M->relax_w.clear();
    return SEM_OK;
  }
  for (int64_t i = 0; i < M->ns; ++i)
    if (!(weight[i] >= 0.0 && weight[i] <= 1.0)) return fail(SEM_E_INVAL, "relaxation weights must lie in [0, 1]");
  M->relax_w.assign(weight, weight + M->ns);
  M->relax_on = true;
  if (M->bound) {
    HIPCHK(hipMemcpy(M->rk + 9 * (size_t)M->ns, M->relax_w.data(), M->ns * sizeof(double), hipMemcpyHostToDevice));
  }
  return SEM_OK;
}

extern "C" sem_status sem_rk4_step_forced(sem_mesh* M, double* eta, double* phi_s, double* phi_ws, double dt,
                                          const double* qa, const sem_solve_opts* opts, sem_solve_stats* stats,
                                          void* stream) {
  sem_status s = check_bound(M);
  if (s) return s;
  if (!qa) return fail(SEM_E_INVAL, "null argument");
  if (!M->relax_on) return fail(SEM_E_INVAL, "no relaxation weights set (sem_set_relaxation)");
  return rk4_step_core(M, eta, phi_s, phi_ws, dt, qa, opts, stats, stream);
}

