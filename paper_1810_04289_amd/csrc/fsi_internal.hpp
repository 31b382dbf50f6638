// Internal state of the HIP FSI library: host-side setup products and the device-resident
// data layout.  Every device array lives in HBM for the solver's lifetime; nothing is
// re-uploaded per Newton step except the step data of fsi_set_step.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fsi.h"

namespace fsi {

enum : int8_t { VK_FLUID = 0, VK_IFACE = 1, VK_SOLID = 2 };
enum : uint8_t { RK_ELEM = 0, RK_DIR = 1, RK_KIN = 2, RK_DUMMY = 3 };

constexpr int kMaxRestart = 200;
constexpr int kRedBlocks = 1024;  // fixed reduction grid: deterministic sums
constexpr int kSweepWaves = 8;    // wavefronts per subdomain in the triangular sweeps
// device flags: [0] inverted element, [1] zero pivot, [2] factorization wait bound, [3] sweep
// wait bound, [4] 1 + the last local row with a singular pivot block, [5] INT32_MAX - the
// first such row, [6] how many there are
constexpr int kFlags = 8;
constexpr int kFacHalf = 9;      // factorization group: 2 * kFacHalf U blocks, lane q < 63 takes two

// Host-side setup products (independent of any device state).
struct HostSetup {
  int V = 0, E = 0, B = 0;
  std::vector<double> X;
  std::vector<int32_t> tets;
  std::vector<int8_t> dom;
  std::vector<int32_t> bfaces;
  std::vector<int8_t> btag;

  std::vector<int8_t> vkind;
  std::vector<uint8_t> rowkind_base, forced_zero;
  std::vector<int32_t> iface;  // [n_iface][3]

  std::vector<int32_t> rowptr, colind;          // block pattern
  // fluid and wall elements in ascending order (residual), and each kind grouped by colour
  // (Jacobian): no two elements of one colour share a vertex; colour c of the fluid is
  // fluid_celems[fluid_col[c] .. fluid_col[c+1])
  std::vector<int32_t> fluid_elems, solid_elems, fluid_celems, solid_celems, fluid_col, solid_col;
  std::vector<int32_t> vinc_ptr, vinc;          // vertex -> (e*4 + local) ascending e
  std::vector<int32_t> elem_blk;                // [E][16]: block of J of (local a, local b)

  // Schwarz subdomains (concatenated; a "local row" is one vertex of one subdomain)
  int ns = 0;
  std::vector<int32_t> part;
  std::vector<int32_t> sub_row_off;   // [ns+1]
  std::vector<int32_t> sub_nowned;    // [ns]
  std::vector<int32_t> lglob;         // [R] global vertex (RCM order inside each subdomain)
  std::vector<uint8_t> lowned;        // [R]
  std::vector<int32_t> lrowptr;       // [R+1] into the concatenated local blocks
  std::vector<int32_t> lcol;          // [NB] column as a concatenated local row index
  std::vector<int32_t> lsrc;          // [NB] block of J, or -1 for a fill block
  std::vector<int32_t> ldiag;         // [R]
  // level schedules: rows of level l of subdomain s are
  // rows[lvl_ptr[sub_lvl[s] + l] .. lvl_ptr[sub_lvl[s] + l + 1])
  std::vector<int32_t> fwd_sub_lvl, fwd_lvl_ptr, fwd_rows;
  std::vector<int32_t> bwd_sub_lvl, bwd_lvl_ptr, bwd_rows;
  // factorization work lists: row i's pivots are piv[4*kent_ptr[i] .. 4*kent_ptr[i+1]),
  // each {position of A_ik in row i, D_k block, length n of U_k, offset o into row i's
  // part of umap}; umap[umap_row[i] + o + t] = 1 + position in row i of the block matching
  // U_k's t-th block, or 0.  (The whole map can exceed 2^31 entries; a row's part cannot.)
  std::vector<int32_t> kent_ptr;  // [R+1]
  std::vector<int32_t> piv;       // [4K]
  std::vector<int32_t> umap;      // [sum of the pivots' U lengths]
  std::vector<int64_t> umap_row;  // [R+1] start of each row's part of umap
  // LDS slots of the sweeps: a row's result occupies a slot from its level to the level
  // of its last reader (interval colouring per subdomain and direction).
  std::vector<int32_t> fwd_qslot, bwd_qslot;  // per schedule slot: own LDS slot or -1 (no reader)
  std::vector<int32_t> lslot;                 // per block: LDS slot of the column row (L: fwd, U: bwd)
  int nslots = 0;                             // max slots over subdomains and directions
};

std::string build_topology(HostSetup& h);
std::string build_subdomains(HostSetup& h, const fsi_opts& o);

// Task lists of one triangular sweep.  Each subdomain's levels are phases, walked by its
// kSweepWaves wavefronts with a workgroup barrier between phases; the rows go to the
// wavefronts round-robin in schedule order.  Wavefront w of subdomain s runs tasks
// [wtask[s*kSweepWaves + w], wtask[s*kSweepWaves + w + 1]).  A task covers at most mb
// blocks: task = {row, global vertex (bit 31 = owned), first, last}, its blocks
// [first, last) (forward: L; backward: U; when a backward row takes several tasks, the one
// next to D_i comes last); aux = {own LDS slot or -1, phase, flags, 0}.
// nphase[s] = phases of subdomain s.
enum : int { kTaskCont = 1, kTaskMore = 2 };
struct SweepTasks {
  std::vector<int32_t> wtask, nphase;
  std::vector<int4> task, aux;
};
SweepTasks build_sweep_tasks(const HostSetup& h, bool bwd, const std::vector<int32_t>& sub_lvl,
                             const std::vector<int32_t>& lvl_ptr, const std::vector<int32_t>& rows,
                             const std::vector<int32_t>& qslot, int mb);

// One sweep schedule: task lists of both sweeps with tasks of at most mb blocks (the kernel
// for mb fixes the prefetch depth).  kSweepPlanMB lists the candidates.
constexpr int kSweepPlans = 4;
// default bound of the factorization's and the sweeps' waits, in polls (about a second);
// a correct schedule never comes near it
constexpr int kWaitLimit = 1 << 23;
constexpr int kSweepPlanMB[kSweepPlans] = {8, 16, 24, 32};
struct SweepPlan {
  int mb = 0;
  int32_t *fwd_wtask = nullptr, *bwd_wtask = nullptr, *fwd_nphase = nullptr, *bwd_nphase = nullptr;
  int4 *fwd_task = nullptr, *bwd_task = nullptr, *fwd_task_aux = nullptr, *bwd_task_aux = nullptr;
};

struct ProfEntry {
  std::string name;
  hipEvent_t a, b;
};

}  // namespace fsi

struct fsi_solver {
  fsi::HostSetup h;
  fsi_physics ph{};
  fsi_opts opts{};
  hipStream_t stream = nullptr;
  std::string err;
  int64_t n = 0, nnzb = 0, R = 0, NB = 0;
  int max_lblk = 0, max_ublk = 0, max_rowblk = 0;  // longest L part, U part, whole local row

  // mesh and maps
  double* X = nullptr;
  int32_t *tets = nullptr, *fluid_elems = nullptr, *solid_elems = nullptr;
  int32_t *fluid_celems = nullptr, *solid_celems = nullptr;
  int32_t *vinc_ptr = nullptr, *vinc = nullptr, *elem_blk = nullptr;
  int32_t *rowptr = nullptr, *colind = nullptr, *blkrow = nullptr;
  double* vals = nullptr;
  double* elemR = nullptr;
  // step data
  uint8_t* rowkind = nullptr;
  double *gval = nullptr, *yold = nullptr, *bforce = nullptr;
  bool has_bforce = false, has_step = false, jac_ready = false, pc_ready = false;
  double t = 0.0, dt = 0.0;
  std::vector<uint8_t> rowkind_host;
  // Schwarz / ILU
  int32_t *lglob = nullptr, *lrowptr = nullptr, *lcol = nullptr, *lsrc = nullptr, *ldiag = nullptr;
  uint8_t* lowned = nullptr;
  int32_t *fwd_sub_lvl = nullptr, *fwd_lvl_ptr = nullptr, *fwd_rows = nullptr;
  int32_t *bwd_sub_lvl = nullptr, *bwd_lvl_ptr = nullptr, *bwd_rows = nullptr;
  // sweep task lists (see SweepTasks) of the selected schedule; sweep_mb: blocks per task.
  // Every candidate schedule's lists are kept (plans), so that the tuner can switch.
  int sweep_mb = 0;
  fsi::SweepPlan plans[fsi::kSweepPlans];
  int32_t *fwd_wtask = nullptr, *bwd_wtask = nullptr, *fwd_nphase = nullptr, *bwd_nphase = nullptr;
  int4 *fwd_task = nullptr, *bwd_task = nullptr;
  int4 *fwd_task_aux = nullptr, *bwd_task_aux = nullptr;
  int32_t* lslot = nullptr;  // per block: LDS byte offset (56 * slot) of its column row's slot
  // factorization groups: row i's are fgrp[fgrp_ptr[i] .. fgrp_ptr[i+1]), for each pivot k
  // (ascending) the blocks of U_k with a match in row i, in runs of up to 2*kFacHalf (one run
  // if there are none): {first block of U_k, D_k block, offset of the run's codes within row
  // i's, (position of A_ik << 6) | (blocks << 1) | first run}.  Row i's codes start at
  // umap[umap_row[i]]; a block's code is (index in U_k << 16) | (position in row i + 1).
  int32_t *fgrp_ptr = nullptr, *umap = nullptr;
  int64_t* umap_row = nullptr;
  int4* fgrp = nullptr;
  // fgrp_lvl[g]: forward level of group g's pivot row.  The factorization's rows go to its
  // fac_nw wavefronts round-robin in level order: wavefront w of subdomain s factors rows
  // fw_row[fw_ptr[s*fac_nw + w] ..] (levels fw_lvl[..])
  int32_t* fgrp_lvl = nullptr;
  int fac_nw = 0;
  // polls a factorization or sweep wait makes before it gives up and flags an error
  int wait_limit = fsi::kWaitLimit;
  int32_t *fw_ptr = nullptr, *fw_row = nullptr, *fw_lvl = nullptr;
  int32_t* sub_row_off = nullptr;
  double *fac = nullptr, *udiag = nullptr, *ylocal = nullptr;
  void* facs = nullptr;  // FP32 or BF16 factors for the sweeps (precision 1 or 2), in fac's buffer
  // precision 3: the factorization itself in FP32, into these (fac and udiag stay null)
  float* fac32 = nullptr;
  float* udiag32 = nullptr;
  // Krylov / Newton work vectors
  double *Vb = nullptr, *w = nullptr, *z = nullptr, *r = nullptr, *tmp = nullptr;
  double *partial = nullptr, *hdev = nullptr, *yvdev = nullptr;
  double *F = nullptr, *Ft = nullptr, *yt = nullptr, *dy = nullptr, *rhs = nullptr;
  int32_t* flags = nullptr;      // [0] inverted, [1] zero pivot
  double* pinned = nullptr;      // host-pinned readback buffer (256 doubles)
  // this solver's device's copy of the allocation-free entry point's scratch (capi.hip),
  // or null with scratch_err set if its address could not be taken
  char* scratch = nullptr;
  hipError_t scratch_err = hipSuccess;
  std::vector<void*> allocs;

  bool prof = false;
  // GMRES Arnoldi steps captured as graphs, one per basis index j (null until first use;
  // dropped when the sweep schedule changes)
  bool graphs = false;
  hipGraphExec_t arnoldi[fsi::kMaxRestart] = {};
  hipStream_t cap_stream = nullptr;  // where the graphs are captured
  std::vector<fsi::ProfEntry> prof_events;
  std::vector<hipEvent_t> event_pool;
};

namespace fsi {
// launchers (assembly.hip, linalg.hip, ilu.hip); all enqueue on s->stream
hipError_t launch_residual(fsi_solver* s, const double* y, double* F);
hipError_t launch_jacobian(fsi_solver* s, const double* y);
hipError_t launch_impose(fsi_solver* s, double* y);
hipError_t launch_spmv(fsi_solver* s, const double* x, double* y);
hipError_t launch_pc_setup(fsi_solver* s);
hipError_t launch_pc_apply(fsi_solver* s, const double* v, double* z);
// the same with the sweeps' work values (pc_apply_ws_bytes of them) and error flags (four
// int32) in caller-given device memory
hipError_t launch_pc_apply_ws(fsi_solver* s, const double* v, double* z, void* yl_ws, int32_t* flags_ws);
size_t pc_apply_ws_bytes(const fsi_solver* s);
hipError_t launch_fac_round(fsi_solver* s);
int sweep_task_blocks(int longest_part);
bool select_plan(fsi_solver* s, int mb);
// wavefronts of the factorization (each stages one row of up to max_rowblk blocks in LDS)
struct FacLayout {  // the factorization's wavefronts per subdomain and LDS slice (blocks)
  int waves, slice;
};
FacLayout fac_layout(int max_rowblk, int elem_bytes);
void drop_graphs(fsi_solver* s);
hipError_t launch_dot_partial(fsi_solver* s, const double* a, const double* b, int64_t n, double* out);
hipError_t launch_mdot(fsi_solver* s, const double* Vb, int nv, const double* w, int64_t n, double* h);
hipError_t launch_vupdate(fsi_solver* s, const double* Vb, int nv, const double* h, double* w, int64_t n);
// the second Gram-Schmidt pass's coefficients into hout, fused with the first pass's update
hipError_t launch_vupdate_mdot(fsi_solver* s, const double* Vb, int nv, const double* h, double* w, int64_t n,
                               double* hout);
// the second pass's update fused with |w|^2 into out
hipError_t launch_vupdate_sqnorm(fsi_solver* s, const double* Vb, int nv, const double* h, double* w, int64_t n,
                                 double* out);
hipError_t launch_vcombine(fsi_solver* s, const double* Vb, int nv, const double* y, double* out, int64_t n);
hipError_t launch_axpby(fsi_solver* s, double a, const double* x, double b, const double* y, double* out, int64_t n);
hipError_t launch_scale(fsi_solver* s, double a, const double* x, double* out, int64_t n);

// profiling helpers (capi.hip)
void prof_begin(fsi_solver* s, const char* name, hipEvent_t* ev_begin);
void prof_end(fsi_solver* s, const char* name, hipEvent_t ev_begin);
}  // namespace fsi

#define FSI_PROF_LAUNCH(s, name, ...)                   \
  do {                                                  \
    hipEvent_t _pe = nullptr;                           \
    if ((s)->prof) fsi::prof_begin((s), (name), &_pe);  \
    __VA_ARGS__;                                        \
    if ((s)->prof) fsi::prof_end((s), (name), _pe);     \
  } while (0)
