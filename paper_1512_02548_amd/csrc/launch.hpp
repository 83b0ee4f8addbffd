// Host-side declarations of the kernel launchers (kernels.hip).  Overloads
// select the working precision from the pointer types.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "sem_internal.hpp"

namespace sem {

enum { OP_STIFF = 0, OP_MASS = 1, OP_PRE_LAP = 2, OP_PRE_MASS = 3, OP_SZ = 4, OP_SU = 5 };
// gather flags: mask the surface rows, negate, skip the launch once the
// tank's Krylov cycle is done (kernels queued ahead of a convergence test)
enum { F_MASK_SURF = 1, F_NEG = 2, F_GATE = 4, F_NOFIX = 8 };   // F_NOFIX: element kernel only
// progress word mirrored to host memory by the Krylov kernels
enum { PROG_STEPS = 0xffff, PROG_DONE = 1 << 16, PROG_CONV = 1 << 17 };

// Inner products of a stiffness output y with Krylov vectors, done by the
// stiffness launch itself: each block's part of <y, V_i> (i < nvec) from its
// own contributions (at a shared line, the value it stores or puts in the
// side buffer, so no fix-up has to come first), then the blocks' parts added
// in a fixed order by the last workgroup into out.
struct StiffDots {
  const void* V = nullptr;     // V_0 .. V_{nvec-1} (working type), stride n
  int64_t n = 0;
  int nvec = 0;                // 0: no products
  int ldp = 0;
  double* part = nullptr;      // [blocks][ldp]
  double* out = nullptr;       // nvec results
  int32_t* counter = nullptr;  // completion count (zero between launches)
};

size_t gather_lds_bytes(const TankDev& h, size_t word);
void launch_coef(const TankDev& h, const TankDev* d, const double* eta, const double* etax, int what, hipStream_t st);
void launch_gather(const TankDev& h, const TankDev* d, int op, const double* u, double* y, double* side, int flags,
                   hipStream_t st);
void launch_gather(const TankDev& h, const TankDev* d, int op, const float* u, float* y, float* side, int flags,
                   int gstore, hipStream_t st);
void launch_gather_only(const TankDev& h, const TankDev* d, int op, int prec, const void* u, void* y, void* side,
                        hipStream_t st);
void launch_stiff_mfma(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, int flags,
                       hipStream_t st);
void launch_stiff_mfma(const TankDev& h, const TankDev* d, const float* u, float* y, float* side, int flags,
                       int gstore, hipStream_t st);
// e0, e1 (optional): events stamped by the dispatch; dots: fused inner products
void launch_stiff_mfma_timed(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, int flags,
                             hipEvent_t e0, hipEvent_t e1, hipStream_t st, const StiffDots& dots = StiffDots{});
void launch_stiff_mfma_timed(const TankDev& h, const TankDev* d, const float* u, float* y, float* side, int flags,
                             int gstore, hipEvent_t e0, hipEvent_t e1, hipStream_t st,
                             const StiffDots& dots = StiffDots{});
void launch_mfma_probe(double* out64, float* out32, hipStream_t st);
void launch_fixup(const TankDev& h, const TankDev* d, double* y, double* side, int flags, hipStream_t st);
void launch_fixup(const TankDev& h, const TankDev* d, float* y, float* side, int flags, hipStream_t st);
// Exact still-water inverse (which 0) or 2D mass inverse (which 1): y = A^{-1} u.
// With nscale, the input is u / *nscale (0 when *nscale <= 0) and, with vout,
// that scaled input is also stored to vout (the normalised Krylov vector).
void launch_sd(const TankDev& h, const TankDev* d, int which, const double* u, double* y, int gate, hipStream_t st,
               const double* nscale = nullptr, double* vout = nullptr);
void launch_sd(const TankDev& h, const TankDev* d, int which, const float* u, float* y, int gate, hipStream_t st,
               const double* nscale = nullptr, float* vout = nullptr);
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st);
void launch_fill(int64_t n, double v, double* y, hipStream_t st);
void launch_ks_reset(KrylovState* ks, double rtol, hipStream_t st);
void launch_relax(int ns, double inv_tau, const double* w, const double* qae, const double* qap, const double* se,
                  const double* sp, double* ke, double* kp, hipStream_t st);
void launch_fill_f(int64_t n, float* y, hipStream_t st);
void launch_mask_surface(const TankDev& h, const TankDev* d, double* y, hipStream_t st);
void launch_scatter_surface(const TankDev& h, const TankDev* d, const double* phis, double* u, int zero_rest,
                            hipStream_t st);
void launch_gather_surface(const TankDev& h, const TankDev* d, const double* u, double* out, hipStream_t st);
void dot_layout(int64_t n, int* nchunk, int64_t* chunk);
// With fixd (the tank) and side: w is an operator output whose shared-line
// contributions are still in `side`; the kernel adds them (and stores w)
// before the products.
void launch_dots(int64_t n, int nvec, const double* X, int64_t ldx, const double* w, double* part, int ldp,
                 double* out, int32_t* counter, const KrylovState* gate, hipStream_t st,
                 const TankDev* fixd = nullptr, const double* side = nullptr);
void launch_dots(int64_t n, int nvec, const float* X, int64_t ldx, const float* w, double* part, int ldp,
                 double* out, int32_t* counter, const KrylovState* gate, hipStream_t st,
                 const TankDev* fixd = nullptr, const float* side = nullptr);
// With fixd (the tank) and side: w's shared-line contributions are still in
// `side`; they are added as w is read.
void launch_orth_givens(int64_t n, int j, const double* V, double* H, int m, double* w, double* part, int ldp,
                        KrylovState* ks, int32_t* counter, int32_t* status, int32_t* mirror, hipStream_t st,
                        const TankDev* fixd = nullptr, const double* side = nullptr);
void launch_orth_givens(int64_t n, int j, const float* V, double* H, int m, float* w, double* part, int ldp,
                        KrylovState* ks, int32_t* counter, int32_t* status, int32_t* mirror, hipStream_t st,
                        const TankDev* fixd = nullptr, const float* side = nullptr);
void launch_scale_next(int64_t n, int j, const double* w, double* V, const double* H, int m, const KrylovState* ks,
                       hipStream_t st);
void launch_scale_next(int64_t n, int j, const float* w, float* V, const double* H, int m, const KrylovState* ks,
                       hipStream_t st);
void launch_residual(const TankDev& h, const TankDev* d, int64_t n, const double* b, const double* y, double* r,
                     int mask, hipStream_t st);
void launch_residual(const TankDev& h, const TankDev* d, int64_t n, const float* b, const float* y, float* r,
                     int mask, hipStream_t st);
void launch_to_float(int64_t n, const double* r, double scale, float* r32, hipStream_t st);
void launch_add_float(int64_t n, const float* x32, double scale, double* x, hipStream_t st);
void launch_recover_dx(const TankDev& h, const TankDev* d, const double* in0, double* out0, const double* in1,
                       double* out1, hipStream_t st);
void launch_fs_rhs(const TankDev& h, const TankDev* d, const double* eta, const double* etax, const double* phix,
                   const double* ws, double* et, double* pt, hipStream_t st);
// the same with caller-chosen scratch: loc [2 nx (P+1)], re and rp [ns]
void launch_fs_rhs_into(const TankDev& h, const TankDev* d, const double* eta, const double* etax,
                        const double* phix, const double* ws, double* et, double* pt, double* loc, double* re,
                        double* rp, hipStream_t st);
void launch_rk4_stage(int ns, double adt, double wgt, int first, const double* y0e, const double* y0p,
                      const double* ke, const double* kp, double* ye, double* yp, double* acce, double* accp,
                      hipStream_t st);
void launch_solve_begin(const TankDev& h, const TankDev* d, const double* phis, double* u, const double* ws,
                        int stage, int maxdepth, double dt, double rtol, int init_ks, hipStream_t st);
void launch_solve_end(const TankDev& h, const TankDev* d, const double* phis, double* phi, int stage, hipStream_t st);
// r = b - y (fix-up folded in) into V_0, ||r||^2 into rr[0], the cycle start; then V_0 /= beta
// bside (FP64 Laplace solves, first cycle): b's shared-line contributions;
// b is fixed up in place and ||b||^2 goes to rr[1]
void launch_residual_cycle(const TankDev& h, const TankDev* d, int64_t n, const double* b, const double* y,
                           const double* side, double* r, int mask, double* part, int ldp, double* rr,
                           int32_t* counter, KrylovState* ks, double* H, int m, int first, int32_t* status,
                           int32_t* mirror, hipStream_t st, const double* bside = nullptr);
void launch_residual_cycle(const TankDev& h, const TankDev* d, int64_t n, const float* b, const float* y,
                           const float* side, float* r, int mask, double* part, int ldp, double* rr,
                           int32_t* counter, KrylovState* ks, double* H, int m, int first, int32_t* status,
                           int32_t* mirror, hipStream_t st);
// y from the small triangular system and x += Z y, one launch
void launch_solve_update_fused(int64_t n, const double* Z, double* H, int m, KrylovState* ks, double* x,
                               hipStream_t st, const TankDev* d = nullptr, const double* phis = nullptr,
                               double* phi = nullptr, int stage = -1);
void launch_solve_update_fused(int64_t n, const float* Z, double* H, int m, KrylovState* ks, float* x,
                               hipStream_t st);
void launch_rk4_final(const TankDev& h, const TankDev* d, double dt, const double* acce, const double* accp,
                      double* eta, double* phi, int use_filter, hipStream_t st);

// ------------------------------------------------------------ batched launches
// One launch over many tanks: its work items (one per workgroup; the device
// copy is placed by the batch) and the dynamic LDS it needs (the most any of
// its tanks needs).  A stage without items is not launched.
struct BatchStage {
  std::vector<BatchItem> items;
  size_t lds = 0;
  const BatchItem* dev = nullptr;
};
// the exact-inverse chain of one operator (which) and precision
struct BatchSD {
  BatchStage cond, modes, fa, fb, fsolve, wlines, wall, wmodes, fc, fd, idft, back;
};
void plan_sd(const std::vector<TankDev>& tanks, const std::vector<int>& ids, int which, int f32, BatchSD* out);
void plan_stiff(const std::vector<TankDev>& tanks, const std::vector<int>& ids, int P, int f32, BatchStage* out);
// input rin -> output zout; jn > 0: the input is w / ||w|| and V_jn is stored
void launch_sd_b(const BatchArgs& a, const BatchSD& p, int which, VSel rin, VSel zout, int jn, int gate, int f32,
                 hipStream_t st);
// gstore as for the single-tank kernel (0 FP64, 1 FP32, 2 bfloat16 factors)
void launch_stiff_b(const BatchArgs& a, const BatchStage& p, int P, VSel u, VSel y, int flags, int gstore,
                    hipStream_t st);
// products of the stiffness output w (before its fix-up) with V_0 ..
// V_{nvec-1} as the single-tank stiffness launch forms them (per stiffness
// block, over p's items {tank, first block, blocks}), then their sums into
// H column hcol
void launch_dots_blocks_b(const BatchArgs& a, const BatchStage& p, const BatchStage& per_tank, int nvec, int hcol,
                          int f32, hipStream_t st);
// partial products over p's work items, then their sums in one workgroup per tank
void launch_dots_b(const BatchArgs& a, const BatchStage& p, const BatchStage& per_tank, int nvec, VSel X, VSel w,
                   int hcol, int sidx, int fix, int gate, int f32, hipStream_t st);
// fix: w's shared-line contributions are still in the side buffer
void launch_orth_b(const BatchArgs& a, const BatchStage& p, const BatchStage& per_tank, int j, int f32,
                   hipStream_t st, int fix = 0);
void launch_fixup_b(const BatchArgs& a, const BatchStage& p, VSel y, int flags, int f32, hipStream_t st);
void launch_residual_b(const BatchArgs& a, const BatchStage& p, VSel b, VSel y, VSel r, int f32, hipStream_t st);
void launch_cycle_start_b(const BatchArgs& a, const BatchStage& per_tank, const BatchStage& vec, int first, int f32,
                          hipStream_t st);
void launch_solve_update_b(const BatchArgs& a, const BatchStage& per_tank, const BatchStage& vec, VSel x, int f32,
                           hipStream_t st);
void launch_ks_init_b(const BatchArgs& a, const BatchStage& per_tank, double rtol, const double* rtol_t,
                      hipStream_t st);
void launch_status_clear_b(const BatchArgs& a, const BatchStage& per_tank, hipStream_t st);
// ks_out / st_out: host-visible arrays indexed by tank
void launch_state_out_b(const BatchArgs& a, const BatchStage& per_tank, KrylovState* ks_out, int32_t* st_out,
                        int mark_noconv, hipStream_t st);
// scalar idx of every tank to out[tank] (host-visible)
void launch_scal_out_b(const BatchArgs& a, const BatchStage& per_tank, int idx, double* out, hipStream_t st);
// iterative refinement: b32 = tmp * scale[t], x32 = 0; then xs += scale[t] * x32
void launch_predict_b(const BatchArgs& a, const BatchStage& vec, int stage, int maxdepth, const double* dt, int table,
                      hipStream_t st);
void launch_history_b(const BatchArgs& a, const BatchStage& vec, int stage, int table, hipStream_t st);
void launch_to_float_b(const BatchArgs& a, const BatchStage& vec, const double* scale, hipStream_t st);
void launch_add_float_b(const BatchArgs& a, const BatchStage& vec, const double* scale, hipStream_t st);
void launch_status_or_b(const BatchArgs& a, const BatchStage& per_tank, int bits, hipStream_t st);
// the RK4 stage work around the Laplace solve, per launch over many tanks
struct BatchStagePlan {
  BatchStage coef[kMaxOrder + 1], final_[kMaxOrder + 1];   // per order
  BatchStage surf;            // elementwise over the surface nodes
  BatchStage circ, fsl, fsg;  // periodic 1D operators (tanks with walls use the single-tank kernels)
};
void plan_stage(const std::vector<TankDev>& tanks, const std::vector<int>& ids, BatchStagePlan* out);
void launch_recover_dx_b(const BatchArgs& a, const BatchStagePlan& p, SSel in0, SSel out0, SSel in1, SSel out1,
                         hipStream_t st);
void launch_coef_b(const BatchArgs& a, const BatchStagePlan& p, SSel eta, SSel etax, int what, hipStream_t st);
// S_z u into each tank's b (element kernel; the line fix-up follows separately)
// S_z of the w~ recovery on the matrix cores (FP64): b = S_z u (side buffer for the fix-up)
void launch_sz_mfma(const TankDev& h, const TankDev* d, const double* u, double* y, double* side, hipStream_t st);
// batched, over the tanks of order P (the FP64 stiffness plan of that order): d.b = S_z u
void launch_sz_mfma_b(const BatchArgs& a, const BatchStage& p, int P, SSel u, hipStream_t st);
void launch_gather_surface_b(const BatchArgs& a, const BatchStagePlan& p, VSel u, SSel out, hipStream_t st);
void launch_fs_rhs_b(const BatchArgs& a, const BatchStagePlan& p, SSel eta, SSel etax, SSel phix, SSel ws,
                     SSel et, SSel pt, hipStream_t st);
// dt: device [count]; ye, yp = stage arrays 0, 1 of each tank
void launch_rk4_stage_b(const BatchArgs& a, const BatchStagePlan& p, const double* dt, double c, double wgt,
                        int first, SSel y0e, SSel y0p, hipStream_t st);
void launch_rk4_final_b(const BatchArgs& a, const BatchStagePlan& p, const double* dt, SSel eta, SSel phi,
                        hipStream_t st);
void launch_lift_in_b(const BatchArgs& a, const BatchStage& vec, const double* const* phis,
                      const double* const* guess, hipStream_t st);
void launch_solution_out_b(const BatchArgs& a, const BatchStage& vec, const double* const* phis, double* const* phi,
                           hipStream_t st);
}  // namespace sem
