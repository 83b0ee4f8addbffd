// Batches of independent tanks (sem_batch_*).
//
// Lockstep mode (nstreams = 0): the Laplace solves of all tanks run as one
// restarted GMRES in lockstep.  Every launch of an Arnoldi step covers the
// workgroups of all tanks (a work-item table per launch: tank, block), each
// tank keeps its own Krylov scalars and leaves the step launches as soon as
// its own cycle is done, so a tank's arithmetic is exactly the single-tank
// solve's.  Kernels of one tank therefore overlap with those of all others,
// and a step costs one launch per kernel for the whole batch.
//
// Concurrent mode (nstreams >= 1): each tank runs its own single-tank step;
// the tanks are spread over worker threads with one HIP stream each.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "launch.hpp"
#include "mesh.hpp"
#include "sem_internal.hpp"

using namespace sem;

namespace {
// pointer tables handed to the batched kernels, each [count]
enum { PT_PHIS = 0, PT_WS = 1, PT_YP = 2, PT_ETA = 3, PT_ETAX = 4, PT_COUNT = 5 };
// pinned staging copies of small uploads (live flags, per-tank scales): a
// slot is reused only after the stream has drained, so an asynchronous
// upload never reads a later value
constexpr int kStageSlots = 16;
}  // namespace

struct sem_batch {
  std::vector<sem_mesh*> meshes;
  int nstreams = 0;
  // concurrent mode
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  hipEvent_t start = nullptr;
  // lockstep mode: the batch's own stream (graph capture needs one that is
  // not the null stream), ordered after and before the caller's stream
  hipStream_t lstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<TankDev> tanks;   // host copies of the descriptors (progress words redirected)
  char* dmem = nullptr;         // device: descriptors, live flags, work items, pointer tables
  TankDev* dtanks = nullptr;
  int32_t* dlive = nullptr;
  const double** dptr = nullptr;
  char* hpin = nullptr;         // pinned host memory, mapped
  int32_t* prog_host = nullptr;
  int32_t* prog_dev = nullptr;
  KrylovState* ks_host = nullptr;
  KrylovState* ks_dev = nullptr;
  int32_t* st_host = nullptr;
  int32_t* st_dev = nullptr;
  char* stage_host = nullptr;     // kStageSlots staging slots of count doubles
  int stage_slot = 0, stage_pending = 0;
  double* scal_host = nullptr;    // [count] tank scalars read back
  double* scal_dev = nullptr;
  double* dscale = nullptr;       // device [count] per-tank factors of the refinement
  double* drtol = nullptr;        // device [count] per-tank tolerances of the inner solves
  double* ddt = nullptr;          // device [count] time steps of the RK4 call
  const double** ptr_host = nullptr;
  BatchStage vec, dots, dblocks, fixup, per_tank;
  BatchStage stiff[kMaxOrder + 1], stiff32[kMaxOrder + 1];   // FP64, FP32 (LDS sized per word)
  BatchSD sdlap, sdlap32;
  BatchSD sdmass;                 // exact inverse of the 2D mass matrix (w recovery)
  BatchStagePlan stage;           // the RK4 stage work around the solves
  std::vector<int> orders;
  int mmax = 0;
  // Arnoldi steps captured as HIP graphs, per step j and precision (FP64,
  // FP32 factors, bfloat16 factors): one launch per step instead of ~20
  bool use_graphs = true;
  bool graphs_failed = false;
  std::vector<hipGraphExec_t> steps[3];
  ~sem_batch() {
    for (auto& v : steps)
      for (auto g : v)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto s : streams) (void)hipStreamDestroy(s);
    for (auto e : events) (void)hipEventDestroy(e);
    if (start) (void)hipEventDestroy(start);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (lstream) (void)hipStreamDestroy(lstream);
    if (dmem) (void)hipFree(dmem);
    if (hpin) (void)hipHostFree(hpin);
  }
};

// ------------------------------------------------------------ set-up
static sem_status setup_lockstep(sem_batch* B, hipStream_t st) {
  const int count = (int)B->meshes.size();
  for (int t = 0; t < count; ++t) {
    const sem_mesh* M = B->meshes[t];
    if (M->hd.pre_kind != 1 || !M->hd.use_mfma)
      return fail(SEM_E_INVAL, "lockstep batches need tanks with the exact still-water inverse and the matrix-core "
                               "stiffness kernel (variant 0); use nstreams >= 1 for the others");
  }
  // pinned host area: progress words, Krylov states, status words, live flags, pointer tables
  const size_t o_prog = 0;
  const size_t o_ks = (o_prog + count * sizeof(int32_t) + 255) / 256 * 256;
  const size_t o_st = (o_ks + count * sizeof(KrylovState) + 255) / 256 * 256;
  const size_t o_scal = (o_st + count * sizeof(int32_t) + 255) / 256 * 256;
  const size_t o_stage = (o_scal + count * sizeof(double) + 255) / 256 * 256;
  const size_t o_ptr = (o_stage + (size_t)kStageSlots * count * sizeof(double) + 255) / 256 * 256;
  const size_t hbytes = o_ptr + (size_t)PT_COUNT * count * sizeof(double*);
  void* hp = nullptr;
  HIPCHK(hipHostMalloc(&hp, hbytes, hipHostMallocMapped | hipHostMallocCoherent));
  B->hpin = (char*)hp;
  std::memset(hp, 0, hbytes);
  void* dp = nullptr;
  HIPCHK(hipHostGetDevicePointer(&dp, hp, 0));
  char* hd = (char*)dp;
  B->prog_host = (int32_t*)(B->hpin + o_prog);
  B->prog_dev = (int32_t*)(hd + o_prog);
  B->ks_host = (KrylovState*)(B->hpin + o_ks);
  B->ks_dev = (KrylovState*)(hd + o_ks);
  B->st_host = (int32_t*)(B->hpin + o_st);
  B->st_dev = (int32_t*)(hd + o_st);
  B->scal_host = (double*)(B->hpin + o_scal);
  B->scal_dev = (double*)(hd + o_scal);
  B->stage_host = B->hpin + o_stage;
  B->ptr_host = (const double**)(B->hpin + o_ptr);
  // descriptors with the progress words redirected to the batch's array
  B->tanks.resize(count);
  std::vector<int> ids(count);
  for (int t = 0; t < count; ++t) {
    B->tanks[t] = B->meshes[t]->hd;
    B->tanks[t].prog = B->prog_dev + t;
    B->mmax = std::max(B->mmax, B->tanks[t].m);
    ids[t] = t;
  }
  // work-item tables
  for (int t = 0; t < count; ++t) {
    const TankDev& h = B->tanks[t];
    const int nv = (int)((h.n + kBlockThreads - 1) / kBlockThreads);
    for (int x = 0; x < nv; ++x) B->vec.items.push_back(BatchItem{t, x, 0, nv});
    const int nd = dot_nchunk(h.n);
    for (int x = 0; x < nd; ++x) B->dots.items.push_back(BatchItem{t, x, 0, nd});
    // products per stiffness block: about 2 048 nodes per workgroup
    const int kbd = std::max(1, std::min(8, 2048 / (h.cb * h.nc + h.nl)));
    for (int x = 0; x < h.nb; x += kbd) B->dblocks.items.push_back(BatchItem{t, x, kbd, h.nb});
    const int nf = (h.nb * h.nl + kBlockThreads - 1) / kBlockThreads;
    for (int x = 0; x < nf; ++x) B->fixup.items.push_back(BatchItem{t, x, 0, nf});
    B->per_tank.items.push_back(BatchItem{t, 0, 0, 1});
  }
  for (int P = 1; P <= kMaxOrder; ++P) {
    plan_stiff(B->tanks, ids, P, 0, &B->stiff[P]);
    plan_stiff(B->tanks, ids, P, 1, &B->stiff32[P]);
    if (!B->stiff[P].items.empty()) B->orders.push_back(P);
  }
  plan_sd(B->tanks, ids, 0, 0, &B->sdlap);
  plan_sd(B->tanks, ids, 0, 1, &B->sdlap32);
  plan_sd(B->tanks, ids, 1, 0, &B->sdmass);
  plan_stage(B->tanks, ids, &B->stage);
  std::vector<BatchStage*> stages = {&B->vec, &B->dots, &B->dblocks, &B->fixup, &B->per_tank};
  for (int P : B->orders) {
    stages.push_back(&B->stiff[P]);
    stages.push_back(&B->stiff32[P]);
  }
  for (int P = 1; P <= kMaxOrder; ++P)
    for (BatchStage* st2 : {&B->stage.coef[P], &B->stage.final_[P]}) stages.push_back(st2);
  for (BatchStage* st2 : {&B->stage.surf, &B->stage.circ, &B->stage.fsl, &B->stage.fsg}) stages.push_back(st2);
  for (BatchSD* p : {&B->sdlap, &B->sdlap32, &B->sdmass})
    for (BatchStage* s : {&p->cond, &p->modes, &p->fa, &p->fb, &p->fsolve, &p->wlines, &p->wall, &p->wmodes,
                          &p->fc, &p->fd, &p->idft, &p->back})
      stages.push_back(s);
  // one device buffer: descriptors | live flags | scales | pointer tables | item tables
  size_t off = (size_t)count * sizeof(TankDev);
  const size_t o_live_d = (off + 255) / 256 * 256;
  off = o_live_d + count * sizeof(int32_t);
  const size_t o_scale_d = (off + 255) / 256 * 256;
  off = o_scale_d + 3 * count * sizeof(double);
  const size_t o_ptr_d = (off + 255) / 256 * 256;
  off = o_ptr_d + (size_t)PT_COUNT * count * sizeof(double*);
  std::vector<size_t> o_items;
  for (BatchStage* s : stages) {
    off = (off + 255) / 256 * 256;
    o_items.push_back(off);
    off += s->items.size() * sizeof(BatchItem);
  }
  void* dm = nullptr;
  HIPCHK(hipMalloc(&dm, off));
  B->dmem = (char*)dm;
  B->dtanks = (TankDev*)B->dmem;
  B->dlive = (int32_t*)(B->dmem + o_live_d);
  B->dscale = (double*)(B->dmem + o_scale_d);
  B->ddt = B->dscale + count;
  B->drtol = B->ddt + count;
  B->dptr = (const double**)(B->dmem + o_ptr_d);
  HIPCHK(hipMemcpyAsync(B->dtanks, B->tanks.data(), count * sizeof(TankDev), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(B->dlive, 0, count * sizeof(int32_t), st));
  for (size_t i = 0; i < stages.size(); ++i) {
    BatchStage* s = stages[i];
    s->dev = (const BatchItem*)(B->dmem + o_items[i]);
    if (!s->items.empty())
      HIPCHK(hipMemcpyAsync(B->dmem + o_items[i], s->items.data(), s->items.size() * sizeof(BatchItem),
                            hipMemcpyHostToDevice, st));
  }
  // the stage potentials of the RK4 steps (table PT_YP) never move
  for (int t = 0; t < count; ++t) B->ptr_host[PT_YP * count + t] = B->meshes[t]->rk + B->meshes[t]->ns;
  HIPCHK(hipMemcpyAsync(B->dptr + (size_t)PT_YP * count, B->ptr_host + (size_t)PT_YP * count,
                        count * sizeof(double*), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return SEM_OK;
}

static BatchArgs args(const sem_batch* B) {
  BatchArgs a{};
  a.tanks = B->dtanks;
  a.live = B->dlive;
  a.items = nullptr;
  a.ptrs = B->dptr;
  a.count = (int32_t)B->meshes.size();
  return a;
}

static sem_status drain(sem_batch* B, hipStream_t st) {
  HIPCHK(hipStreamSynchronize(st));
  B->stage_pending = 0;
  return SEM_OK;
}

// asynchronous upload of at most count doubles through a staging slot
static sem_status upload(sem_batch* B, void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (B->stage_pending == kStageSlots) {
    sem_status s = drain(B, st);
    if (s) return s;
  }
  char* h = B->stage_host + (size_t)B->stage_slot * B->meshes.size() * sizeof(double);
  B->stage_slot = (B->stage_slot + 1) % kStageSlots;
  B->stage_pending++;
  std::memcpy(h, src, bytes);
  HIPCHK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, st));
  return SEM_OK;
}

// live flags of the tanks that take part in the next launches
static sem_status set_live(sem_batch* B, const std::vector<int>& live, hipStream_t st) {
  std::vector<int32_t> f(B->meshes.size(), 0);
  for (int t : live) f[t] = 1;
  return upload(B, B->dlive, f.data(), f.size() * sizeof(int32_t), st);
}

static sem_status put_pointers(sem_batch* B, int which, const double* const* p, hipStream_t st) {
  const int count = (int)B->meshes.size();
  for (int t = 0; t < count; ++t) B->ptr_host[which * count + t] = p ? p[t] : nullptr;
  HIPCHK(hipMemcpyAsync(B->dptr + (size_t)which * count, B->ptr_host + (size_t)which * count,
                        count * sizeof(double*), hipMemcpyHostToDevice, st));
  return SEM_OK;
}

// ------------------------------------------------------------ lockstep GMRES
// Kernels of Arnoldi step j over all tanks: z_j = M^-1 v_j (for j > 0,
// v_j = w / ||w|| is formed on the way), w = A z_j, the products with
// V_0..V_j per stiffness block and their sums, the orthogonalisation (w's
// shared-line fix-up on the way) and Givens update: the single-tank step's
// arithmetic (there the stiffness launch forms the products itself).  Every launch returns at once for a tank
// whose cycle is done.
static void issue_step(sem_batch* B, int j, int f32, int gstore, hipStream_t st) {
  const BatchArgs a = args(B);
  const BatchStage* stiff = f32 ? B->stiff32 : B->stiff;
  const BatchSD& sdp = f32 ? B->sdlap32 : B->sdlap;
  launch_sd_b(a, sdp, 0, j == 0 ? VSel{BV_V, 0} : VSel{BV_W, 0}, VSel{BV_Z, j}, j, 1, f32, st);
  for (int P : B->orders)
    launch_stiff_b(a, stiff[P], P, VSel{BV_Z, j}, VSel{BV_W, 0}, F_MASK_SURF | F_GATE | F_NOFIX, gstore, st);
  launch_dots_blocks_b(a, B->dblocks, B->per_tank, j + 1, j, f32, st);
  launch_orth_b(a, B->dots, B->per_tank, j, f32, st, 1);
}

// The step as a graph launch: captured from the stream on first use (the
// launches only read device-resident tables and flags, so one capture per
// step and precision serves every later cycle and call).  Falls back to
// direct launches if capture is not possible.
static sem_status arnoldi_step(sem_batch* B, int j, int f32, int gstore, hipStream_t st) {
  if (!B->use_graphs || B->graphs_failed) {
    issue_step(B, j, f32, gstore, st);
    return SEM_OK;
  }
  auto& g = B->steps[f32 ? gstore : 0];
  if ((int)g.size() < B->mmax) g.resize(B->mmax, nullptr);
  if (!g[j]) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      issue_step(B, j, f32, gstore, st);
      ok = hipStreamEndCapture(st, &graph) == hipSuccess && graph;
    }
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    if (!ok) {
      (void)hipGetLastError();
      B->graphs_failed = true;
      issue_step(B, j, f32, gstore, st);
      return SEM_OK;
    }
    g[j] = exec;
  }
  HIPCHK(hipGraphLaunch(g[j], st));
  return SEM_OK;
}

// Restarted right-preconditioned GMRES on every tank in `act`, b and the
// start vector x already in each tank's workspace (FP64 b, xs; or, f32, the
// FP32 copies b32, x32 with FP32 (gstore 1) or bfloat16 (gstore 2) factors).
// iters[t] accumulates.  Tanks whose status word is set leave `act`; with
// mark_noconv, unconverged tanks get the no-convergence bit (and leave too).
// rtol_t (optional, device): a tolerance per tank instead of rtol; x_zero:
// the start vector is zero, so the first cycle's residual is b itself (the
// operator is not applied to it; A 0 = 0 exactly).
static sem_status lockstep_gmres(sem_batch* B, std::vector<int>& act, double rtol, int max_iter, int ahead, int f32,
                                 int gstore, int mark_noconv, std::vector<int32_t>& iters, hipStream_t st,
                                 const double* rtol_t = nullptr, bool x_zero = false) {
  if (act.empty()) return SEM_OK;
  const BatchArgs a = args(B);
  const BatchStage* stiff = f32 ? B->stiff32 : B->stiff;
  const BatchSD& sdp = f32 ? B->sdlap32 : B->sdlap;
  volatile int32_t* prog = B->prog_host;
  ahead = std::max(1, ahead);
  sem_status s = set_live(B, act, st);
  if (s) return s;
  launch_ks_init_b(a, B->per_tank, rtol, rtol_t, st);
  launch_dots_b(a, B->dots, B->per_tank, 1, VSel{BV_B, 0}, VSel{BV_B, 0}, -1, 1, 0, 0, f32, st);
  std::vector<int> live = act;
  bool first = true;
  while (true) {
    for (int t : live) prog[t] = 0;
    // r = b - A x
    if (first && x_zero) {
      launch_residual_b(a, B->vec, VSel{BV_B, 0}, VSel{BV_NONE, 0}, VSel{BV_V, 0}, f32, st);
    } else {
      for (int P : B->orders) launch_stiff_b(a, stiff[P], P, VSel{BV_XS, 0}, VSel{BV_W, 0}, F_MASK_SURF, gstore, st);
      launch_fixup_b(a, B->fixup, VSel{BV_W, 0}, F_MASK_SURF, f32, st);
      launch_residual_b(a, B->vec, VSel{BV_B, 0}, VSel{BV_W, 0}, VSel{BV_V, 0}, f32, st);
    }
    launch_dots_b(a, B->dots, B->per_tank, 1, VSel{BV_V, 0}, VSel{BV_V, 0}, -1, 0, 0, 0, f32, st);
    launch_cycle_start_b(a, B->per_tank, B->vec, first ? 1 : 0, f32, st);
    first = false;
    for (int j = 0; j < B->mmax; ++j) {
      s = arnoldi_step(B, j, f32, gstore, st);
      if (s) return s;
      // queue at most `ahead` steps in front of the slowest running tank
      bool stop = false;
      auto tq = std::chrono::steady_clock::now();
      while (true) {
        bool all_done = true;
        int minsteps = INT_MAX;
        for (int t : live) {
          const int32_t v = prog[t];
          if (!(v & PROG_DONE)) {
            all_done = false;
            minsteps = std::min(minsteps, v & PROG_STEPS);
          }
        }
        if (all_done) {
          stop = true;
          break;
        }
        if (j + 1 - minsteps <= ahead) break;
        auto now = std::chrono::steady_clock::now();
        if (now - tq > std::chrono::microseconds(100)) {
          tq = now;
          hipError_t q = hipStreamQuery(st);
          if (q == hipSuccess) break;   // drained: the words are final, re-read them next step
          if (q != hipErrorNotReady) HIPCHK(q);
        }
        __builtin_ia32_pause();
      }
      if (stop) break;
    }
    launch_solve_update_b(a, B->per_tank, B->vec, VSel{BV_XS, 0}, f32, st);
    launch_state_out_b(a, B->per_tank, B->ks_dev, B->st_dev, 0, st);
    s = drain(B, st);
    if (s) return s;
    std::vector<int> next;
    for (int t : live) {
      const KrylovState& k = B->ks_host[t];
      if (B->st_host[t] || k.status || k.converged || k.iters >= max_iter) continue;
      next.push_back(t);
    }
    if (next.empty()) break;
    live.swap(next);
    s = set_live(B, live, st);
    if (s) return s;
  }
  // final states of every tank of the solve
  s = set_live(B, act, st);
  if (s) return s;
  launch_state_out_b(a, B->per_tank, B->ks_dev, B->st_dev, mark_noconv, st);
  s = drain(B, st);
  if (s) return s;
  std::vector<int> keep;
  for (int t : act) {
    iters[t] += B->ks_host[t].iters;
    if (!B->st_host[t]) keep.push_back(t);
  }
  act.swap(keep);
  return SEM_OK;
}

// FP64 iterative refinement around FP32 lockstep GMRES (the single-tank
// solve's steps, every tank in `act` at once): r = b - A x in FP64, then the
// correction from the inner solve of A d = r / ||r||, x += ||r|| d.  Tanks
// that fail leave `act` with their status bit set.
static sem_status lockstep_ir(sem_batch* B, std::vector<int>& act, const sem_solve_opts& o,
                              std::vector<int32_t>& iters, hipStream_t st) {
  const int count = (int)B->meshes.size();
  const BatchArgs a = args(B);
  const int gstore = o.prec == SEM_PREC_BF16_IR ? 2 : 1;
  sem_status s = set_live(B, act, st);
  if (s) return s;
  launch_dots_b(a, B->dots, B->per_tank, 1, VSel{BV_B, 0}, VSel{BV_B, 0}, -1, 4, 0, 0, 0, st);
  launch_scal_out_b(a, B->per_tank, 4, B->scal_dev, st);
  s = drain(B, st);
  if (s) return s;
  std::vector<double> bnorm(count, 0.0), rn(count, 0.0), scale(count, 0.0), itol(count, 0.0);
  for (int t : act) bnorm[t] = std::sqrt(B->scal_host[t]);
  std::vector<int> cur = act, noconv, nonfinite;
  for (int k = 0; k <= o.max_refine && !cur.empty(); ++k) {
    s = set_live(B, cur, st);
    if (s) return s;
    for (int P : B->orders) launch_stiff_b(a, B->stiff[P], P, VSel{BV_XS, 0}, VSel{BV_W, 0}, F_MASK_SURF, 0, st);
    launch_fixup_b(a, B->fixup, VSel{BV_W, 0}, F_MASK_SURF, 0, st);
    launch_residual_b(a, B->vec, VSel{BV_B, 0}, VSel{BV_W, 0}, VSel{BV_TMP, 0}, 0, st);
    launch_dots_b(a, B->dots, B->per_tank, 1, VSel{BV_TMP, 0}, VSel{BV_TMP, 0}, -1, 4, 0, 0, 0, st);
    launch_scal_out_b(a, B->per_tank, 4, B->scal_dev, st);
    s = drain(B, st);
    if (s) return s;
    std::vector<int> next;
    int min_iters = INT_MAX;
    for (int t : cur) {
      rn[t] = std::sqrt(B->scal_host[t]);
      if (!std::isfinite(rn[t])) {
        nonfinite.push_back(t);
        continue;
      }
      if (rn[t] <= o.rtol * bnorm[t] || rn[t] == 0.0) continue;   // converged
      if (k == o.max_refine || iters[t] >= o.max_iter) {
        noconv.push_back(t);
        continue;
      }
      next.push_back(t);
      min_iters = std::min(min_iters, (int)iters[t]);
    }
    if (next.empty()) break;
    for (int t : next) {
      scale[t] = 1.0 / rn[t];
      itol[t] = inner_tolerance(o.inner_rtol, o.rtol, bnorm[t], rn[t]);
    }
    s = set_live(B, next, st);
    if (!s) s = upload(B, B->dscale, scale.data(), count * sizeof(double), st);
    if (!s) s = upload(B, B->drtol, itol.data(), count * sizeof(double), st);
    if (s) return s;
    launch_to_float_b(a, B->vec, B->dscale, st);
    std::vector<int> inner = next;
    s = lockstep_gmres(B, inner, o.inner_rtol, o.max_iter - min_iters, o.lookahead, 1, gstore, 0, iters, st, B->drtol,
                       true);
    if (s) return s;
    s = set_live(B, inner, st);
    if (!s) s = upload(B, B->dscale, rn.data(), count * sizeof(double), st);
    if (s) return s;
    launch_add_float_b(a, B->vec, B->dscale, st);
    cur.swap(inner);
  }
  if (!noconv.empty()) {
    s = set_live(B, noconv, st);
    if (s) return s;
    launch_status_or_b(a, B->per_tank, ST_NOCONV, st);
  }
  if (!nonfinite.empty()) {
    s = set_live(B, nonfinite, st);
    if (s) return s;
    launch_status_or_b(a, B->per_tank, ST_NONFINITE, st);
  }
  s = set_live(B, act, st);
  if (s) return s;
  launch_state_out_b(a, B->per_tank, B->ks_dev, B->st_dev, 0, st);
  s = drain(B, st);
  if (s) return s;
  std::vector<int> keep;
  for (int t : act)
    if (!B->st_host[t]) keep.push_back(t);
  act.swap(keep);
  return SEM_OK;
}

// Laplace solves of the tanks in `act` with their factors current: lift from
// the surface potentials (pointer table PT_PHIS or PT_YP), the solve, Phi out
// to the PT_WS table's vectors (which hold the start vectors on entry when warm).
static sem_status lockstep_laplace(sem_batch* B, std::vector<int>& act, int phis_table, int warm,
                                   const sem_solve_opts& o, std::vector<int32_t>& iters, hipStream_t st) {
  const int count = (int)B->meshes.size();
  const BatchArgs a = args(B);
  sem_status s = set_live(B, act, st);
  if (s) return s;
  const double* const* phis = B->dptr + (size_t)phis_table * count;
  launch_lift_in_b(a, B->vec, phis, warm ? B->dptr + (size_t)PT_WS * count : nullptr, st);
  for (int P : B->orders)
    launch_stiff_b(a, B->stiff[P], P, VSel{BV_TMP, 0}, VSel{BV_B, 0}, F_MASK_SURF | F_NEG, 0, st);
  launch_fixup_b(a, B->fixup, VSel{BV_B, 0}, F_MASK_SURF | F_NEG, 0, st);
  std::vector<int> solved = act;
  if (o.prec == SEM_PREC_FP64) s = lockstep_gmres(B, act, o.rtol, o.max_iter, o.lookahead, 0, 0, 1, iters, st);
  else s = lockstep_ir(B, act, o, iters, st);
  if (s) return s;
  s = set_live(B, solved, st);
  if (s) return s;
  launch_solution_out_b(a, B->vec, phis, const_cast<double* const*>(B->dptr + (size_t)PT_WS * count), st);
  return SEM_OK;
}

static sem_status check_opts(const sem_solve_opts* opts, sem_solve_opts* o) {
  if (opts) *o = *opts;
  else default_opts(o);
  if (!(o->rtol > 0) || o->max_iter < 1) return fail(SEM_E_INVAL, "rtol > 0 and max_iter >= 1 required");
  if (o->prec < 0 || o->prec > 2) return fail(SEM_E_INVAL, "unknown precision");
  if (o->prec != SEM_PREC_FP64 && !(o->inner_rtol > 0 && o->inner_rtol < 1))
    return fail(SEM_E_INVAL, "inner_rtol must lie in (0, 1)");
  if (o->predict < 0 || o->predict > kHistSteps) return fail(SEM_E_INVAL, "predict must be in 0..6");
  return SEM_OK;
}

static sem_status lockstep_solve(sem_batch* B, const double* const* eta, const double* const* eta_x,
                                 const double* const* phi_s, double* const* phi, const uint8_t* active,
                                 const sem_solve_opts* opts, int32_t* per_status, int32_t* per_iters,
                                 hipStream_t st) {
  const int count = (int)B->meshes.size();
  sem_solve_opts o;
  sem_status s = check_opts(opts, &o);
  if (s) return s;
  std::vector<int> act;
  for (int t = 0; t < count; ++t) {
    if (active && !active[t]) continue;
    if (!eta[t] || !eta_x[t] || !phi_s[t] || !phi[t]) return fail(SEM_E_INVAL, "null per-tank argument");
    act.push_back(t);
  }
  const BatchArgs a = args(B);
  s = put_pointers(B, PT_PHIS, phi_s, st);
  if (!s) s = put_pointers(B, PT_WS, (const double* const*)phi, st);
  if (!s) s = put_pointers(B, PT_ETA, eta, st);
  if (!s) s = put_pointers(B, PT_ETAX, eta_x, st);
  if (s) return s;
  std::vector<int> all = act;
  s = set_live(B, act, st);
  if (s) return s;
  launch_status_clear_b(a, B->per_tank, st);
  launch_coef_b(a, B->stage, SSel{SS_PT, PT_ETA}, SSel{SS_PT, PT_ETAX}, 3, st);
  std::vector<int32_t> iters(count, 0);
  s = lockstep_laplace(B, act, PT_PHIS, o.warm_start, o, iters, st);
  if (s) return s;
  s = set_live(B, all, st);
  if (s) return s;
  launch_state_out_b(a, B->per_tank, B->ks_dev, B->st_dev, 0, st);
  s = drain(B, st);
  if (s) return s;
  sem_status worst = SEM_OK;
  for (int t = 0; t < count; ++t) {
    const bool on = !active || active[t];
    const sem_status ts = on ? status_from_word(B->st_host[t]) : SEM_OK;
    if (per_status) per_status[t] = ts;
    if (per_iters) per_iters[t] = on ? iters[t] : 0;
    if (ts != SEM_OK && worst == SEM_OK) worst = ts;
  }
  if (worst != SEM_OK) return fail(worst, "at least one tank failed; see per_tank_status");
  return SEM_OK;
}

// One RK4 step of every active tank; the same steps as the single-tank call
// (gradient recovery, coefficients, Laplace solve, w recovery, free-surface
// right side, stage update; filter and transactional write-back at the end),
// each as one launch over all tanks.  Tanks with walls take their 1D
// operators from the single-tank kernels.
static sem_status lockstep_rk4(sem_batch* B, double* const* eta, double* const* phi_s, double* const* phi_ws,
                               const double* dt, const uint8_t* active, const sem_solve_opts* opts,
                               int32_t* per_status, int32_t* per_iters, hipStream_t st) {
  const int count = (int)B->meshes.size();
  sem_solve_opts o;
  sem_status s = check_opts(opts, &o);
  if (s) return s;
  std::vector<int> act;
  for (int t = 0; t < count; ++t)
    if (!active || active[t]) act.push_back(t);
  const BatchArgs a = args(B);
  s = put_pointers(B, PT_PHIS, (const double* const*)phi_s, st);
  if (!s) s = put_pointers(B, PT_WS, (const double* const*)phi_ws, st);
  if (!s) s = put_pointers(B, PT_ETA, (const double* const*)eta, st);
  if (!s) s = upload(B, B->ddt, dt, count * sizeof(double), st);
  if (s) return s;
  const std::vector<int> all = act;
  s = set_live(B, act, st);
  if (s) return s;
  launch_status_clear_b(a, B->per_tank, st);
  std::vector<int32_t> iters(count, 0);
  const double cnode[4] = {0.0, 0.5, 0.5, 1.0};
  const double wts[4] = {1.0 / 6, 2.0 / 6, 2.0 / 6, 1.0 / 6};
  const SSel RK[9] = {{SS_RK, 0}, {SS_RK, 1}, {SS_RK, 2}, {SS_RK, 3}, {SS_RK, 4},
                      {SS_RK, 5}, {SS_RK, 6}, {SS_RK, 7}, {SS_RK, 8}};
  for (int sidx = 0; sidx < 4 && !act.empty(); ++sidx) {
    const SSel se = sidx == 0 ? SSel{SS_PT, PT_ETA} : RK[0];
    const SSel sp = sidx == 0 ? SSel{SS_PT, PT_PHIS} : RK[1];
    s = set_live(B, act, st);
    if (s) return s;
    launch_recover_dx_b(a, B->stage, se, RK[2], sp, RK[3], st);
    launch_coef_b(a, B->stage, se, RK[2], 3, st);
    launch_predict_b(a, B->vec, sidx, o.predict, B->ddt, PT_WS, st);
    s = lockstep_laplace(B, act, sidx == 0 ? PT_PHIS : PT_YP, 1, o, iters, st);
    if (s) return s;
    if (act.empty()) break;
    s = set_live(B, act, st);
    if (s) return s;
    launch_history_b(a, B->vec, sidx, PT_WS, st);
    // w~: M w = S_z Phi, w~ = w at the surface
    for (int P = 1; P <= kMaxOrder; ++P) launch_sz_mfma_b(a, B->stiff[P], P, SSel{SS_PT, PT_WS}, st);
    launch_fixup_b(a, B->fixup, VSel{BV_B, 0}, 0, 0, st);
    launch_sd_b(a, B->sdmass, 1, VSel{BV_B, 0}, VSel{BV_WMASS, 0}, 0, 0, 0, st);
    launch_gather_surface_b(a, B->stage, VSel{BV_WMASS, 0}, RK[4], st);
    launch_fs_rhs_b(a, B->stage, se, RK[2], RK[3], RK[4], RK[5], RK[6], st);
    launch_rk4_stage_b(a, B->stage, B->ddt, sidx < 3 ? cnode[sidx + 1] : 0.0, wts[sidx], sidx == 0 ? 1 : 0,
                       SSel{SS_PT, PT_ETA}, SSel{SS_PT, PT_PHIS}, st);
  }
  if (!act.empty()) {
    s = set_live(B, act, st);
    if (s) return s;
    launch_rk4_final_b(a, B->stage, B->ddt, SSel{SS_PT, PT_ETA}, SSel{SS_PT, PT_PHIS}, st);
  }
  s = set_live(B, all, st);
  if (s) return s;
  launch_state_out_b(a, B->per_tank, B->ks_dev, B->st_dev, 0, st);
  s = drain(B, st);
  if (s) return s;
  sem_status worst = SEM_OK;
  for (int t = 0; t < count; ++t) {
    const bool on = !active || active[t];
    const sem_status ts = on ? status_from_word(B->st_host[t]) : SEM_OK;
    if (per_status) per_status[t] = ts;
    if (per_iters) per_iters[t] = on ? iters[t] : 0;
    if (ts != SEM_OK && worst == SEM_OK) worst = ts;
  }
  if (worst != SEM_OK) return fail(worst, "at least one tank failed; see per_tank_status");
  return SEM_OK;
}

// ------------------------------------------------------------ concurrent mode
static sem_status concurrent_rk4(sem_batch* B, double* const* eta, double* const* phi_s, double* const* phi_ws,
                                 const double* dt, const uint8_t* active, const sem_solve_opts* opts,
                                 int32_t* per_status, int32_t* per_iters, hipStream_t cst) {
  const int count = (int)B->meshes.size();
  // inputs written on the caller's stream must be visible to the workers
  HIPCHK(hipEventRecord(B->start, cst));
  const int W = (int)B->streams.size();
  for (int w = 0; w < W; ++w) HIPCHK(hipStreamWaitEvent(B->streams[w], B->start, 0));
  // largest tanks first, dealt to the least-loaded worker
  std::vector<int> order;
  for (int i = 0; i < count; ++i)
    if (!active || active[i]) order.push_back(i);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return B->meshes[a]->n > B->meshes[b]->n; });
  std::vector<std::vector<int>> work(W);
  std::vector<double> load(W, 0.0);
  for (int i : order) {
    int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    work[w].push_back(i);
    load[w] += (double)B->meshes[i]->n;
  }
  std::vector<sem_status> res(count, SEM_OK);
  std::vector<int32_t> its(count, 0);
  auto run = [&](int w) {
    for (int i : work[w]) {
      sem_solve_stats st4[4] = {};
      res[i] = sem_rk4_step(B->meshes[i], eta[i], phi_s[i], phi_ws[i], dt[i], opts, st4, B->streams[w]);
      its[i] = st4[0].iters + st4[1].iters + st4[2].iters + st4[3].iters;
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < W; ++w) th.emplace_back(run, w);
  run(0);
  for (auto& t : th) t.join();
  for (int w = 0; w < W; ++w) {
    HIPCHK(hipEventRecord(B->events[w], B->streams[w]));
    HIPCHK(hipStreamWaitEvent(cst, B->events[w], 0));
  }
  sem_status worst = SEM_OK;
  for (int i = 0; i < count; ++i) {
    if (per_status) per_status[i] = (active && !active[i]) ? SEM_OK : res[i];
    if (per_iters) per_iters[i] = its[i];
    if (res[i] != SEM_OK && worst == SEM_OK) worst = res[i];
  }
  if (worst != SEM_OK) return fail(worst, "at least one tank failed; see per_tank_status");
  return SEM_OK;
}

// work on the batch's stream follows the caller's earlier work, and the
// caller's stream waits for the batch's
static sem_status enter(sem_batch* B, hipStream_t caller) {
  HIPCHK(hipEventRecord(B->ev_in, caller));
  HIPCHK(hipStreamWaitEvent(B->lstream, B->ev_in, 0));
  return SEM_OK;
}
static sem_status leave(sem_batch* B, hipStream_t caller) {
  HIPCHK(hipEventRecord(B->ev_out, B->lstream));
  HIPCHK(hipStreamWaitEvent(caller, B->ev_out, 0));
  return SEM_OK;
}

// ------------------------------------------------------------ public calls
extern "C" sem_status sem_batch_create(sem_mesh* const* meshes, int32_t count, int32_t nstreams, void* stream,
                                       sem_batch** out) {
  if (!meshes || count < 1 || !out) return fail(SEM_E_INVAL, "bad batch arguments");
  if (nstreams < 0 || nstreams > 64) return fail(SEM_E_INVAL, "nstreams must be in 0..64");
  for (int i = 0; i < count; ++i)
    if (!meshes[i] || !meshes[i]->bound) return fail(SEM_E_INVAL, "every mesh must be bound");
  for (int i = 0; i < count; ++i)
    if (meshes[i]->relax_on) return fail(SEM_E_INVAL, "relaxation zones are not supported in batches");
  for (int i = 0; i < count; ++i)
    for (int j = i + 1; j < count; ++j)
      if (meshes[i] == meshes[j]) return fail(SEM_E_INVAL, "a mesh appears twice in the batch");
  std::unique_ptr<sem_batch> B(new (std::nothrow) sem_batch());
  if (!B) return fail(SEM_E_NOMEM, "host allocation failed");
  B->meshes.assign(meshes, meshes + count);
  B->nstreams = nstreams;
  if (nstreams == 0) {
    sem_status s = setup_lockstep(B.get(), (hipStream_t)stream);
    if (s) return s;
    HIPCHK(hipStreamCreateWithFlags(&B->lstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
  } else {
    int ns = std::min<int>(nstreams, count);
    for (int i = 0; i < ns; ++i) {
      hipStream_t st;
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      B->streams.push_back(st);
      hipEvent_t ev;
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      B->events.push_back(ev);
    }
    HIPCHK(hipEventCreateWithFlags(&B->start, hipEventDisableTiming));
  }
  *out = B.release();
  return SEM_OK;
}

extern "C" sem_status sem_batch_rk4_step(sem_batch* B, double* const* eta, double* const* phi_s,
                                         double* const* phi_ws, const double* dt, const uint8_t* active,
                                         const sem_solve_opts* opts, int32_t* per_status, int32_t* per_iters,
                                         void* stream) {
  if (!B || !eta || !phi_s || !phi_ws || !dt) return fail(SEM_E_INVAL, "null argument");
  const int count = (int)B->meshes.size();
  for (int i = 0; i < count; ++i) {
    if (active && !active[i]) continue;
    if (!eta[i] || !phi_s[i] || !phi_ws[i] || !(dt[i] > 0) || !std::isfinite(dt[i]))
      return fail(SEM_E_INVAL, "bad per-tank argument");
  }
  hipStream_t st = (hipStream_t)stream;
  if (B->nstreams == 0) {
    sem_status s = enter(B, st);
    if (s) return s;
    s = lockstep_rk4(B, eta, phi_s, phi_ws, dt, active, opts, per_status, per_iters, B->lstream);
    sem_status s2 = leave(B, st);
    return s ? s : s2;
  }
  return concurrent_rk4(B, eta, phi_s, phi_ws, dt, active, opts, per_status, per_iters, st);
}

extern "C" sem_status sem_batch_laplace_solve(sem_batch* B, const double* const* eta, const double* const* eta_x,
                                              const double* const* phi_s, double* const* phi, const uint8_t* active,
                                              const sem_solve_opts* opts, int32_t* per_status, int32_t* per_iters,
                                              void* stream) {
  if (!B || !eta || !eta_x || !phi_s || !phi) return fail(SEM_E_INVAL, "null argument");
  if (B->nstreams != 0) return fail(SEM_E_INVAL, "batched Laplace solves need a lockstep batch (nstreams = 0)");
  hipStream_t st = (hipStream_t)stream;
  sem_status s = enter(B, st);
  if (s) return s;
  s = lockstep_solve(B, eta, eta_x, phi_s, phi, active, opts, per_status, per_iters, B->lstream);
  sem_status s2 = leave(B, st);
  return s ? s : s2;
}

extern "C" sem_status sem_batch_apply_timed(sem_batch* B, int32_t order, int32_t prec, int32_t reps, float* ms,
                                            void* stream) {
  if (!B || !ms || reps < 1) return fail(SEM_E_INVAL, "bad argument");
  if (prec < 0 || prec > 2) return fail(SEM_E_INVAL, "unknown precision");
  if (B->nstreams != 0) return fail(SEM_E_INVAL, "timing needs a lockstep batch");
  if (order < 1 || order > kMaxOrder || B->stiff[order].items.empty())
    return fail(SEM_E_INVAL, "no tank of this order in the batch");
  hipStream_t cst = (hipStream_t)stream;
  if (sem_status s = enter(B, cst)) return s;
  hipStream_t st = B->lstream;
  std::vector<int> all(B->meshes.size());
  for (size_t t = 0; t < all.size(); ++t) all[t] = (int)t;
  if (sem_status s = set_live(B, all, st)) return s;
  const BatchArgs a = args(B);
  const BatchStage& plan = prec == 0 ? B->stiff[order] : B->stiff32[order];
  // every tank's tmp vector in, w out (FP32 for prec 1 and 2: the
  // refinement's inner vectors), no masking, no gating
  const VSel u = prec == 0 ? VSel{BV_TMP, 0} : VSel{BV_W, 0};
  const VSel y = prec == 0 ? VSel{BV_W, 0} : VSel{BV_B, 0};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  launch_stiff_b(a, plan, order, u, y, 0, prec, st);   // warm-up
  HIPCHK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) launch_stiff_b(a, plan, order, u, y, 0, prec, st);
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float t = 0;
  HIPCHK(hipEventElapsedTime(&t, e0, e1));
  *ms = t / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return leave(B, cst);
}

extern "C" sem_status sem_batch_graphs(sem_batch* B, int32_t enable) {
  if (!B) return fail(SEM_E_INVAL, "null batch");
  B->use_graphs = enable != 0;
  return SEM_OK;
}

extern "C" sem_status sem_batch_graph_count(const sem_batch* B, int32_t* captured) {
  if (!B || !captured) return fail(SEM_E_INVAL, "null argument");
  int32_t c = 0;
  for (const auto& v : B->steps)
    for (auto g : v) c += g != nullptr;
  *captured = c;
  return SEM_OK;
}

extern "C" void sem_batch_destroy(sem_batch* B) { delete B; }
