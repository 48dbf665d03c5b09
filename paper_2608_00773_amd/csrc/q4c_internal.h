// Internal declarations shared by the host plan builder and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "q4c.h"

namespace q4c {

// Contraction tile edge (functions) and points per staged K chunk.
constexpr int kTile = 64;
constexpr int kChunk = 16;
constexpr int kTicketStride = 16;                  // one 64-byte line per ticket queue
constexpr int kTicketsPerLaunch = 8 * kTicketStride; // 8 XCD queues

// Work item of the contraction / adjoint kernels: one (batch, row tile, column tile)
// with ti <= tj over the batch's local function list.
struct WorkItem {
  int32_t batch;
  int16_t ti, tj;
};

// Everything a kernel needs about the plan, as raw device pointers.
struct DevPlan {
  // basis
  const double *R;             // [3 n_atoms]
  const int32_t *fn_atom;      // [n_fn]
  const int32_t *fn_shlm;      // [n_fn] shell * 32 + (l*l + l + m), l <= 4
  const double *shell_rcut;    // [n_shells]
  const int32_t *shell_nint;   // [n_shells]
  const double *shell_knot;    // [2 n_shells]: nint^2 / rcut, rcut / nint^2
  const int64_t *shell_coef_off;   // into coef (scaled table, see q4c_plan::coef_scaled)
  const double *coef;
  const int64_t *shell_u_off;  // into ucoef (ket potential, scaled like coef); null until set
  const double *ucoef;
  // grid, batch order
  const double *px, *py, *pz, *pw;  // [n_active]
  const int32_t *perm;              // [n_active] user index
  const int32_t *batch_pt_off;      // [n_batches + 1]
  const int32_t *batch_fn_off;      // [n_batches + 1]
  const int32_t *loc_fn;            // [fn_entries] global function
  const int32_t *loc_slot;          // [fn_entries] slot (relevant atom) within the batch
  const int64_t *loc_info;          // [fn_entries] slot | slot's first local function << 20 | its function count << 40
  const int64_t *loc_rowoff;        // [fn_entries] staging offset of the function's slot block row (pass relative)
  const int32_t *batch_slot_off;    // [n_batches + 1]
  const int32_t *slot_fnoff;        // [n_slots] local function offset of the slot
  const int32_t *slot_nfn;          // [n_slots]
  const int64_t *slot_row_off;      // [n_slots] staging offset of the slot's block row (pass relative)
  const int64_t *work_part_off;     // [n_work] adjoint partial offset (pass relative)
  const int64_t *pair_off;          // [n_pairs + 1]
  const int32_t *pair_na, *pair_nb; // [n_pairs]
  const int32_t *pair_a, *pair_b;   // [n_pairs]
  const int64_t *batch_work_off;    // [n_batches + 1] first work item of each batch
  // per batch, for slot pairs si <= sj (upper triangle, row-major): the stored
  // pair of the two atoms, or -1; batch b's table starts at batch_sp_off[b]
  const int32_t *sp_pair;
  const int64_t *sp_poff;           // the same table holding the pair's store offset (pair_off), or -1
  const int64_t *batch_sp_off;      // [n_batches + 1]
  const int64_t *tab_off;           // [n_batches + 1] prefix of P_b n_b (nao_tabulate layout)
  const int64_t *panel_off;         // [n_batches] pass-relative offset of the batch's operand panel
  int64_t store_len;
  int64_t n_active;
  int64_t n_points;
  double cprime;  // 1 / (4 c^2)
};

// How the two contraction kernels are launched: work order (0: batch order,
// 1: largest items first) and persistent workgroup count (0: one workgroup
// per work item).
struct LaunchCfg {
  int32_t order = 0;
  int32_t persistent = 0;
};

// One adjoint position: a column half (32 columns from tj * 64 + 32 half) of
// work item (batch, ti, tj) whose columns start inside the batch, with the
// batch data its kernel needs (64 bytes, one load).
struct AdjPos {
  int32_t batch;
  int16_t ti, tj;
  int32_t half, f0;
  int32_t n, g0, P, sbase;
  int32_t ns, pad_;
  int64_t panel_off;  // pass relative
  int64_t spb;        // batch_sp_off of the batch
  int64_t part;       // pass-relative offset of the half's P partials
};
static_assert(sizeof(AdjPos) == 64, "AdjPos is 64 bytes");

struct Pass {
  int64_t b0, b1;        // batch range
  int64_t w0, w1;        // work range
  int64_t r0, r1;        // reduction-entry range
  int64_t t0, t1;        // panel-tile range
  int64_t staging_len;   // doubles
  int64_t partial_len;   // doubles (adjoint partials, stored after the staging)
  int64_t panel_len;     // doubles (operand panels, stored after the partials)
  int64_t ap0, ap1;      // adjoint positions (d_adjpos, d_adjpos_cost)
};

// Scalar -> spinor transformation (Eq. 33): coefficients of one spinor type
// (l, kappa, m_j) on the scalar functions of its large shell (component 0)
// and of its small partner shell (component 1), per spin (0: up, 1: down).
struct SpinorType {
  int32_t n[2][2];        // [component][spin]: number of entries (0..2)
  int32_t m[2][2][2];     // function offset within the shell (m' + l)
  double re[2][2][2], im[2][2][2];
};
// One scalar function of one component in the reverse transformation: the
// spinor functions (atom-local) it enters, per spin, with their coefficients.
struct ScalarRel {
  int32_t n[2];
  int32_t mu[2][4];
  double re[2][4], im[2][4];
};
// One spinor function: atom-local offsets of its large and small shells, type.
struct SpinorFn {
  int32_t offL, offS, type;
};

// Padded panel sizes: points to a multiple of kChunk, functions to a multiple of 16.
__host__ __device__ inline int64_t pad16(int64_t x) { return (x + 15) / 16 * 16; }

}  // namespace q4c

struct q4c_plan {
  // ---- host copies of the inputs
  int32_t n_atoms = 0, n_shells = 0, n_fn = 0;
  std::vector<double> R;
  std::vector<int32_t> atom_shell_off, shell_l, shell_nint;
  std::vector<double> shell_rcut;
  std::vector<int64_t> shell_coef_off;
  std::vector<double> coef;
  // Radial tables re-expressed in d = s - r_j: (c0, c1/h, c2/h^2, c3/h^3) per
  // interval, so the kernels evaluate Rt and Rt' without dividing by h.
  std::vector<double> coef_scaled;
  std::vector<int64_t> shell_cs_off;
  std::vector<double> shell_knot;
  // Ket potential u_s = eps_s - V_s per shell (H/S integrand), in the same
  // scaled form; empty until q4c_plan_set_ket_potential.
  std::vector<double> ucoef_scaled;
  std::vector<int64_t> shell_us_off;
  std::vector<int32_t> atom_fn_off;  // [n_atoms + 1]
  std::vector<double> atom_rcut;     // [n_atoms]
  std::vector<int32_t> fn_atom, fn_shlm;
  double c_light = 137.035999084;
  int32_t p_max = 300;
  int32_t flags = 0;
  int64_t staging_budget = 0;

  // ---- independent systems (one unless built by q4c_plan_create_batched)
  int32_t n_systems = 1;
  std::vector<int32_t> atom_sys;  // [n_atoms]
  std::vector<int64_t> sys_atom_off, sys_point_off, sys_batch_off, sys_pair_off;  // [n_systems + 1]

  // ---- grid / batches
  int64_t n_points = 0, n_active = 0, n_batches = 0;
  std::vector<int32_t> perm;  // batch-ordered active point -> user index
  std::vector<double> px, py, pz, pw;
  std::vector<int32_t> batch_pt_off, batch_fn_off, loc_fn, loc_slot;
  std::vector<int32_t> batch_slot_off, slot_atom, slot_fnoff, slot_nfn;
  std::vector<int64_t> slot_row_off;

  // ---- pairs
  int64_t n_pairs = 0, store_len = 0;
  int64_t max_pair_block = 1;  // largest n_A n_B of a stored pair (the reduction's grid)
  std::vector<int32_t> pair_a, pair_b, pair_na, pair_nb;
  std::vector<int64_t> pair_off;
  std::vector<int64_t> atom_pair_start;  // [n_atoms + 1] pairs with first atom A

  // ---- work, passes, reductions
  std::vector<q4c::WorkItem> work;
  std::vector<int64_t> work_part_off;
  std::vector<q4c::Pass> passes;
  std::vector<int32_t> red_pair;
  std::vector<uint8_t> red_first;
  std::vector<int64_t> red_inc_off;  // [n_red + 1]
  std::vector<int64_t> inc_src;      // staging offsets (pass relative)
  std::vector<int32_t> untouched_pairs;
  std::vector<int64_t> batch_work_off, tab_off, panel_off;
  std::vector<q4c::WorkItem> ptile;  // (batch, function tile) list of the panel kernel
  std::vector<int64_t> batch_tile_off;  // [n_batches + 1] first ptile item of each batch
  std::vector<int32_t> work_order;   // per pass, pass-relative work indices by decreasing cost
  std::vector<int32_t> sp_pair;      // see DevPlan::sp_pair
  std::vector<int64_t> batch_sp_off;
  int64_t max_scratch = 0;
  int64_t max_batch_points = 0, max_batch_fn = 0, fn_entries = 0;
  double flops_alg = 0.0;
  double flops_alg_hs = 0.0;  // sum_B 3 P_B n_B^2: the three contractions of q4c_integrate_HS

  // ---- device
  bool on_device = false;
  int device = -1;
  int64_t device_bytes = 0;
  std::vector<void *> allocations;
  q4c::DevPlan dp{};
  q4c::WorkItem *d_work = nullptr;
  int32_t *d_red_pair = nullptr;
  uint8_t *d_red_first = nullptr;
  int64_t *d_red_inc_off = nullptr;
  int64_t *d_inc_src = nullptr;
  int32_t *d_untouched = nullptr;
  q4c::WorkItem *d_ptile = nullptr;
  double *d_om = nullptr;  // [n_active + 16] point weights w_g v_g of the current call
  q4c::AdjPos *d_adjpos = nullptr;       // adjoint positions per pass, batch order
  q4c::AdjPos *d_adjpos_cost = nullptr;  // the same, work items by decreasing cost
  double *d_coef_fold = nullptr;  // [5][store_len + 16] the adjoint's coefficients of the current call (k_coef_fold)
  double *d_ucoef = nullptr;         // ket-potential tables (q4c_plan_set_ket_potential)
  int64_t *d_shell_us_off = nullptr;
  double *d_staging = nullptr;
  int32_t *d_flag = nullptr;
  int32_t *d_order = nullptr;      // per pass: work items sorted by cost (pass-relative indices)
  unsigned *d_tickets = nullptr;   // [2][n_passes][kTicketsPerLaunch] persistent-launch queues
  int n_cu = 256;                  // compute units of the plan's device

  // ---- scalar -> spinor transformation tables, built for one small-component
  // plan on first use (q4c_spinor_transform); mutable: calls take a const plan
  mutable const q4c_plan *sp_small = nullptr;
  mutable int64_t sp_small_fn = -1, sp_small_len = -1;
  mutable q4c::SpinorType *d_sp_types = nullptr;
  mutable q4c::SpinorFn *d_sp_fns = nullptr;
  mutable int32_t *d_sp_off = nullptr;  // [n_atoms + 1] first spinor function of each atom
  mutable int32_t *d_sp_nL = nullptr;   // [n_atoms] large-component functions per atom
  mutable int32_t *d_sp_nS = nullptr;   // [n_atoms] small-component functions per atom
  mutable int64_t *d_sp_poffS = nullptr;  // [n_pairs + 1] block offsets in the small plan's store
  mutable q4c::ScalarRel *d_sp_relL = nullptr, *d_sp_relS = nullptr;  // reverse transformation, per scalar function
  mutable int32_t *d_sp_fL = nullptr, *d_sp_fS = nullptr;  // [n_atoms] first scalar function of each atom
  mutable int64_t sp_store_len_S = 0;

  // ---- periodic cells (q4c_plan_set_cells): cell pairs a <= b of the
  // reference cell's atoms and the stored pairs contributing to each
  int32_t n_cell_atoms = 0;
  std::vector<int32_t> cell_atom;       // [n_atoms]
  std::vector<int32_t> cp_a, cp_b;      // [n_cell_pairs]
  std::vector<int64_t> cp_off;          // [n_cell_pairs + 1] block offsets (n_a n_b each)
  int32_t *d_cp_a = nullptr, *d_cp_b = nullptr;
  int64_t *d_cp_off = nullptr, *d_ct_off = nullptr;  // contributions of cell pair c: [ct_off[c], ct_off[c+1])
  int32_t *d_ct_pair = nullptr, *d_ct_flag = nullptr;  // stored pair; 1: transposed orientation
  double *d_ct_T = nullptr;             // [3 per contribution] translation of the phase exp(i k.T)
  int64_t n_contrib = 0;                // contributions over all cell pairs
  int32_t *d_pc_cp = nullptr, *d_pc_flag = nullptr;  // per stored pair: cell pair; 1: reached transposed (a > b)
  double *d_pc_T = nullptr;             // [3 per stored pair] T_B' - T_A'
  int32_t *d_pc_order = nullptr;        // stored pairs sorted by cell pair
  mutable double *d_kpts = nullptr;     // k-points (3 n_k) and weights (n_k) of the last call (grown on demand)
  mutable int64_t kpts_cap = 0;
  mutable double *d_bloch_ph = nullptr; // phases of one k chunk: kBlochKChunk max(n_contrib, n_pairs) complex
  mutable int64_t bloch_ph_cap = 0;     // doubles

  // ---- density_gradient_on_grid tables, built on first use: per pass the
  // items (batch, 64-point tile, 64-function tile) of the product and
  // (batch, 64 x 64 tile rt <= ct) of the dense M, per batch the pass-relative offsets
  // of its M (np x np) and partials (function tiles x 4 x Pp), and buffers
  // for the largest pass
  mutable std::vector<int64_t> gr_item_off, gr_cd_item_off;  // [n_passes + 1]
  mutable int32_t *d_gr_items = nullptr, *d_gr_cditems = nullptr;
  mutable int64_t *d_gr_cd_off = nullptr, *d_gr_part_off = nullptr;
  mutable int64_t *d_gr_fninfo = nullptr;  // [fn_entries] slot | slot's first function << 20 | its count << 40
  mutable double *d_gr_cd = nullptr, *d_gr_part = nullptr;

  // ---- what the panel region holds after the calls enqueued so far: the
  // W-path panels (phi, grad phi) of pass panel_pass, or -1 (nothing usable:
  // H/S panels, or unknown).  Calls on one plan are stream-ordered, so the
  // host can track it.
  mutable int64_t panel_pass = -1;

  // ---- launch configuration (chosen by q4c_plan_autotune or set directly)
  q4c::LaunchCfg cfg_contract{}, cfg_density{}, cfg_hs{};
  bool use_graphs = false;
  mutable hipStream_t capture_stream = nullptr;
  struct GraphEntry {
    int kind;  // 0 integrate, 1 density
    const void *in;
    void *out0, *out1, *out2;
    int64_t a, b, c;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  mutable std::vector<GraphEntry> graphs;

  // ---- profiling (mutable: calls take a const plan)
  mutable bool profiling = false;
  mutable std::vector<hipEvent_t> ev_pool;                // free events
  mutable std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_live;  // (timer, start/stop)
};

namespace q4c {
void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);
int fail_status(int code, const char *msg);  // set_error(msg) and return code

// kernel launchers (q4c_kernels.hip)
int launch_tabulate(const q4c_plan *p, int64_t b0, int64_t b1, int deriv, int dtype, void *out, hipStream_t s);
int launch_integrate(const q4c_plan *p, const double *v, int precision, uint32_t parts, uint32_t flags,
                     double *store, double *spin_w, double *spin_v, hipStream_t s);
// resident_pass >= 0: the plan's panel region already holds the W-path
// panels of that pass (left by the previous call), which is then not tabulated
int launch_density(const q4c_plan *p, const double *coef, uint32_t terms, int precision, int weight_mode,
                   double *out, int64_t resident_pass, hipStream_t s);
int launch_integrate_hs(const q4c_plan *p, const double *v, uint32_t flags, double *hs, hipStream_t s);
int launch_density_grad(const q4c_plan *p, const double *coef, double *out, hipStream_t s);
// dense M, product and point sums of one pass of density_gradient_on_grid
// (q4c_grad_kernels.hip), on the pass's panel
int launch_grad_pass(const q4c_plan *p, size_t ip, const double *coef, const double *panel, double *out,
                     hipStream_t s);
// Bloch sums of a store over the plan's cell pairs (q4c_bloch_kernels.hip),
// k-points in chunks of kBlochKChunk; phase: 2 kBlochKChunk n_contrib doubles
constexpr int kBlochKChunk = 64;
int launch_bloch_sum(const q4c_plan *p, int n_parts, const double *store, int n_k, const double *kpts_dev,
                     double *phase, double *out, hipStream_t s);
// q4c_bloch_sum_noalloc: the phase table in the library's fixed device
// scratch (kNoAllocScratchDoubles per device, address looked up once per
// device), k-points already on the device
constexpr int64_t kNoAllocScratchDoubles = (int64_t)1 << 19;  // 4 MiB
constexpr int kMaxDevices = 64;
int noalloc_scratch(int device, double **ptr);
int launch_bloch_sum_noalloc(const q4c_plan *p, int n_parts, const double *store, int n_k, const double *kpts_dev,
                             double *out, hipStream_t s);
int launch_bloch_density(const q4c_plan *p, int n_parts, const double *rho, int n_k, const double *kpts_dev,
                         const double *kw_dev, double *phase, double *coef, hipStream_t s);
// spinor density -> scalar density matrices of both components (q4c_spinor_kernels.hip)
int launch_spinor_to_scalar(const q4c_plan *pl, const double *d_spin, double *c_large, double *c_small,
                            hipStream_t s);
// scalar -> spinor transformation of two H/S stores (q4c_spinor_kernels.hip)
int launch_spinor_transform(const q4c_plan *pl, const double *hs_large, const double *hs_small, double *h_out,
                            double *s_out, hipStream_t s);
// k_contract_hs over work items [w0, w0 + nw) of a pass (q4c_hs_kernels.hip)
int launch_contract_hs(const q4c_plan *p, int64_t w0, int64_t nw, const int32_t *order, const double *panel,
                       unsigned *tickets, unsigned grid, hipStream_t s);
int launch_coef_from_spinor(const q4c_plan *p, const double *spin_d, double *coef_out, hipStream_t s);
int launch_check_finite(const q4c_plan *p, const double *v, hipStream_t s, bool *finite);

// Brackets one launch with events when the plan is profiling.
struct TimedLaunch {
  const q4c_plan *p;
  int timer;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TimedLaunch(const q4c_plan *p_, int timer_, hipStream_t s_);
  ~TimedLaunch();
};
}  // namespace q4c
