// Host-side mesh object and helpers shared by the library's driver files.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sem.h"
#include "launch.hpp"
#include "sem_internal.hpp"

namespace sem {
// error text of the last failing call on this thread; returns s
sem_status fail(sem_status s, const std::string& msg);
}  // namespace sem

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) return sem::fail(SEM_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------ mesh object
namespace sem {
struct Upload {
  size_t off;
  std::vector<char> data;
};
}  // namespace sem

struct sem_mesh {
  // description
  int nx = 0, nz = 0, P = 0, periodic = 1, Pf = 0, ic = 2, m = 30;
  double L = 0, g = 9.81, sf = 1.0;
  std::vector<double> h, hx, slev;
  // derived sizes
  int Np = 0, NpP = 0, nl = 0, nc = 0, cb = 1, nb = 1, T = 1, EB = 0, nclass_col = 1;
  int pre_kind = 0, variant = 0;
  int tiles_req = 0;        // requested 16-element tiles per stiffness workgroup (0 = from the size)
  int sd_nI[2] = {0, 0}, sd_q[2] = {0, 0};
  int sd_M1[2] = {0, 0}, sd_nMT1[2] = {0, 0}, sd_KS1[2] = {0, 0}, sd_nMT3[2] = {0, 0}, sd_KS3[2] = {0, 0};
  int sd_wall[2] = {0, 0};
  int fft_n1 = 0, fft_n2 = 0;   // four-step transforms along x (0: direct)
  int circ1d = 0;
  int circ_band = 0;        // elements on each side kept by the periodic 1D applies
  int wall_nl = 0, wall_nr = 0, wall_wd = 0;   // walls: explicit rows near each wall, their window
  int64_t n = 0, ns = 0, E = 0;
  // host tables
  std::vector<int32_t> elem_loc, acc_cnt, acc_ent, surf_loc, is_surf_loc;
  std::vector<uint16_t> acc_pk, acc_cm;   // packed node-sum table of the matrix-core kernels
  std::vector<double> node_x, node_sig;
  std::vector<int64_t> surf_nodes;
  // layout
  size_t ws_bytes = 0;
  std::vector<sem::Upload> uploads;
  sem::TankDev hd{};             // device pointers filled at bind (offsets before)
  char* ws = nullptr;
  sem::TankDev* dtank = nullptr;
  double* scal = nullptr;   // small device scalars
  bool bound = false;
  bool relax_on = false;        // relaxation-zone weights set (sem_set_relaxation)
  std::vector<double> relax_w;  // their host copy, uploaded again at every bind
  // offsets of dynamic arrays
  std::map<std::string, size_t> off;
  // RK4 scratch (surface arrays)
  double *rk = nullptr;
  // progress word of the running Krylov cycle in pinned host memory (written
  // by the device, read by the host while it queues steps)
  int32_t* prog_host = nullptr;
  // pinned host block that every small device-to-host readback lands in
  // (never pageable stack memory: several worker threads may read back at once)
  void* rb_host = nullptr;
  int32_t* prog_dev = nullptr;
  int device = -1;               // the device the workspace was bound on
  // live timing of the stiffness kernel (event pairs of the running cycle)
  bool kt_on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> kt_ev;
  size_t kt_used = 0;
  int64_t kt_count = 0;
  double kt_ms = 0;
  // start and end events of the stage solves of one RK4 step (slot 0 also
  // serves a single solve); created when the mesh is bound
  hipEvent_t solve_ev[4][2] = {};
  ~sem_mesh() {
    if (prog_host) (void)hipHostFree(prog_host);
    if (rb_host) (void)hipHostFree(rb_host);
    for (auto& e : solve_ev)
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    for (auto& e : kt_ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
};

namespace sem {
sem_status check_bound(sem_mesh* M);
sem_status status_from_word(int32_t w);
void default_opts(sem_solve_opts* o);
// w~ from M w = S_z Phi with the factors 1/d current; out [ns]
sem_status recover_w_core(sem_mesh* M, const double* Phi, double* out, hipStream_t st);

// Tolerance of a refinement's inner solve (single tank and batch alike): the
// configured inner tolerance, loosened (up to 1/2) when the residual is
// already near the target, so that the last refinement reduces it only by
// the factor still needed, with a margin of 2.
inline double inner_tolerance(double inner, double rtol, double bnorm, double rn) {
  const double need = rn > 0 ? 0.5 * rtol * bnorm / rn : 0.5;
  return std::max(inner, std::min(0.5, need));
}

}  // namespace sem
