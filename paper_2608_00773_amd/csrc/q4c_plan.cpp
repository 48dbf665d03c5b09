// Host side of libq4c: argument validation, the integration plan (batching,
// basis-relevance lists, atom-pair store layout, staging passes), device
// upload and the C ABI entry points.
//
// Paper Sec. III A: the grid is split into batches B_v of nearby points
// (Eq. 31) and only the functions non-zero on a batch, nnz(B_v), enter its
// partial integrals.  Here the batches come from recursive median bisection
// of the active points (points inside at least one basis support), the
// relevant set is taken per atom (all functions of an atom with a point of
// the batch inside its cutoff; with equal shell cutoffs this is the exact
// set), and the per-batch dense partial matrices are summed into a sparse
// atom-pair block store instead of per-task dense matrices.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <stdexcept>
#include <numeric>
#include <string>
#include <vector>

#include "q4c_internal.h"

namespace {
thread_local std::string g_last_error;

struct CellList {
  double lo[3]{}, h = 1.0;
  int n[3]{1, 1, 1};
  std::vector<int32_t> head, next;
  void build(int na, const double *R, double cell) {
    h = cell > 1e-6 ? cell : 1.0;
    double hi[3] = {-1e300, -1e300, -1e300};
    for (int d = 0; d < 3; ++d) lo[d] = 1e300;
    for (int a = 0; a < na; ++a)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], R[3 * a + d]);
        hi[d] = std::max(hi[d], R[3 * a + d]);
      }
    if (na == 0)
      for (int d = 0; d < 3; ++d) lo[d] = hi[d] = 0.0;
    for (int d = 0; d < 3; ++d) n[d] = std::max(1, (int)std::floor((hi[d] - lo[d]) / h) + 1);
    head.assign((size_t)n[0] * n[1] * n[2], -1);
    next.assign(std::max(na, 1), -1);
    for (int a = na - 1; a >= 0; --a) {
      int ix[3];
      for (int d = 0; d < 3; ++d) ix[d] = std::min(n[d] - 1, std::max(0, (int)((R[3 * a + d] - lo[d]) / h)));
      size_t id = ((size_t)ix[2] * n[1] + ix[1]) * n[0] + ix[0];
      next[a] = head[id];
      head[id] = a;
    }
  }
  // visit atoms in cells overlapping the box [bl, bh]
  template <class F>
  void visit_box(const double *bl, const double *bh, F &&f) const {
    int a0[3], a1[3];
    for (int d = 0; d < 3; ++d) {
      a0[d] = std::max(0, (int)std::floor((bl[d] - lo[d]) / h));
      a1[d] = std::min(n[d] - 1, (int)std::floor((bh[d] - lo[d]) / h));
      if (a0[d] > a1[d]) return;
    }
    for (int iz = a0[2]; iz <= a1[2]; ++iz)
      for (int iy = a0[1]; iy <= a1[1]; ++iy)
        for (int ix = a0[0]; ix <= a1[0]; ++ix)
          for (int a = head[((size_t)iz * n[1] + iy) * n[0] + ix]; a >= 0; a = next[a]) f(a);
  }
};

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Recursive median bisection along the axis of largest extent until a batch
// holds at most pmax points.  The cut goes at the multiple of 16 points
// nearest the median (once a half holds 16 points or more), so every batch
// but the last of each system fills whole 16-point chunks of the MFMA
// contractions.  Ties are broken by index, so the result does not depend on
// the nth_element implementation.
void bisect(std::vector<int32_t> &idx, int64_t lo, int64_t hi, int pmax, const double *const xyz[3],
            std::vector<int64_t> &ends) {
  struct Seg {
    int64_t lo, hi;
  };
  std::vector<Seg> stack{{lo, hi}};
  std::vector<Seg> leaves;
  // depth-first, left before right: push right first
  while (!stack.empty()) {
    Seg s = stack.back();
    stack.pop_back();
    int64_t n = s.hi - s.lo;
    if (n <= pmax) {
      leaves.push_back(s);
      continue;
    }
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = s.lo; i < s.hi; ++i)
      for (int d = 0; d < 3; ++d) {
        double c = xyz[d][idx[i]];
        mn[d] = std::min(mn[d], c);
        mx[d] = std::max(mx[d], c);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (mx[d] - mn[d] > mx[ax] - mn[ax]) ax = d;
    const double *c = xyz[ax];
    const int64_t half = n / 2;
    const int64_t left = half >= 16 ? std::min<int64_t>((half + 8) / 16 * 16, n - 1) : half;
    int64_t mid = s.lo + left;
    std::nth_element(idx.begin() + s.lo, idx.begin() + mid, idx.begin() + s.hi,
                     [c](int32_t a, int32_t b) { return c[a] < c[b] || (c[a] == c[b] && a < b); });
    stack.push_back({mid, s.hi});
    stack.push_back({s.lo, mid});
  }
  for (auto &s : leaves) ends.push_back(s.hi);
}

template <class T>
int upload(q4c_plan *p, const std::vector<T> &h, T **d) {
  size_t bytes = std::max<size_t>(h.size() * sizeof(T), 16);
  void *ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) return q4c::hip_fail(e, "hipMalloc");
  p->allocations.push_back(ptr);
  p->device_bytes += (int64_t)bytes;
  if (!h.empty()) {
    e = hipMemcpy(ptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return q4c::hip_fail(e, "hipMemcpy");
  }
  *d = (T *)ptr;
  return Q4C_OK;
}

int device_alloc(q4c_plan *p, size_t bytes, void **d) {
  void *ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, std::max<size_t>(bytes, 16));
  if (e != hipSuccess) return q4c::hip_fail(e, "hipMalloc");
  p->allocations.push_back(ptr);
  p->device_bytes += (int64_t)bytes;
  *d = ptr;
  return Q4C_OK;
}

void free_device(q4c_plan *p) {
  if (!p->graphs.empty() || p->capture_stream) {
    if (p->device >= 0) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (auto &g : p->graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    p->graphs.clear();
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    p->capture_stream = nullptr;
  }
  if (p->device >= 0 && (!p->ev_pool.empty() || !p->ev_live.empty())) {
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    for (auto &x : p->ev_live) {
      (void)hipEventDestroy(x.second.first);
      (void)hipEventDestroy(x.second.second);
    }
    p->ev_pool.clear();
    p->ev_live.clear();
  }
  if (!p->allocations.empty()) {
    if (p->device >= 0) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (void *ptr : p->allocations) (void)hipFree(ptr);
    p->allocations.clear();
  }
}

int validate(const q4c_basis *b, const q4c_grid *g) {
  if (!b || !g) return fail(Q4C_EINVAL, "basis and grid descriptors are required");
  if (b->n_atoms < 0 || b->n_shells < 0 || b->n_coef < 0 || g->n_points < 0)
    return fail(Q4C_EINVAL, "negative size");
  if (g->n_points >= (int64_t)INT32_MAX) return fail(Q4C_EINVAL, "more than 2^31-1 grid points");
  if (b->n_atoms > 0 && (!b->R || !b->atom_shell_off)) return fail(Q4C_EINVAL, "NULL atom arrays");
  if (b->n_shells > 0 && (!b->shell_l || !b->shell_rcut || !b->shell_nint || !b->shell_coef_off || !b->coef))
    return fail(Q4C_EINVAL, "NULL shell arrays");
  if (g->n_points > 0 && (!g->x || !g->y || !g->z || !g->w)) return fail(Q4C_EINVAL, "NULL grid arrays");
  if (b->n_atoms > 0) {
    if (b->atom_shell_off[0] != 0 || b->atom_shell_off[b->n_atoms] != b->n_shells)
      return fail(Q4C_EINVAL, "atom_shell_off must run from 0 to n_shells");
    for (int a = 0; a < b->n_atoms; ++a)
      if (b->atom_shell_off[a + 1] < b->atom_shell_off[a]) return fail(Q4C_EINVAL, "atom_shell_off decreasing");
    if (!finite_all(b->R, 3 * (int64_t)b->n_atoms)) return fail(Q4C_EINVAL, "non-finite atom position");
  } else if (b->n_shells != 0) {
    return fail(Q4C_EINVAL, "shells without atoms");
  }
  for (int s = 0; s < b->n_shells; ++s) {
    if (b->shell_l[s] < 0) return fail(Q4C_EINVAL, "negative angular momentum");
    if (b->shell_l[s] > 4) return fail(Q4C_EUNSUPPORTED, "angular momentum above 4 (g) is not supported");
    if (!(b->shell_rcut[s] > 0.0) || !std::isfinite(b->shell_rcut[s])) return fail(Q4C_EINVAL, "bad shell cutoff");
    if (b->shell_nint[s] < 1) return fail(Q4C_EINVAL, "shell_nint must be >= 1");
    if (b->shell_coef_off[s] < 0 || b->shell_coef_off[s] + 4 * (int64_t)b->shell_nint[s] > b->n_coef)
      return fail(Q4C_EINVAL, "radial table outside coef");
    if (b->shell_coef_off[s] % 4 != 0) return fail(Q4C_EINVAL, "shell_coef_off must be a multiple of 4");
  }
  if (b->n_coef > 0 && !finite_all(b->coef, b->n_coef)) return fail(Q4C_EINVAL, "non-finite radial coefficient");
  if (g->n_points > 0) {
    if (!finite_all(g->x, g->n_points) || !finite_all(g->y, g->n_points) || !finite_all(g->z, g->n_points) ||
        !finite_all(g->w, g->n_points))
      return fail(Q4C_EINVAL, "non-finite grid coordinate or weight");
  }
  return Q4C_OK;
}

// sys_atom_off: [n_sys + 1] atom ranges of the independent systems (system-major);
// pt_sys: system of every grid point (NULL: one system).  Points, batches,
// relevant atoms and pairs never mix systems.
int build_host(q4c_plan *p, const q4c_basis *b, const q4c_grid *g, const std::vector<int64_t> &sys_atom_off,
               const int32_t *pt_sys) {
  const int na = b->n_atoms;
  const int nsys = (int)sys_atom_off.size() - 1;
  p->n_systems = nsys;
  p->atom_sys.assign(na, 0);
  for (int sy = 0; sy < nsys; ++sy)
    for (int64_t a = sys_atom_off[sy]; a < sys_atom_off[sy + 1]; ++a) p->atom_sys[a] = sy;
  p->sys_atom_off = sys_atom_off;
  auto psys = [&](int64_t i) -> int32_t { return pt_sys ? pt_sys[i] : 0; };
  p->n_atoms = na;
  p->n_shells = b->n_shells;
  p->R.assign(b->R, b->R + 3 * (size_t)na);
  p->atom_shell_off.assign(b->atom_shell_off, b->atom_shell_off + na + 1);
  if (na == 0) p->atom_shell_off.assign(1, 0);
  p->shell_l.assign(b->shell_l, b->shell_l + b->n_shells);
  p->shell_rcut.assign(b->shell_rcut, b->shell_rcut + b->n_shells);
  p->shell_nint.assign(b->shell_nint, b->shell_nint + b->n_shells);
  p->shell_coef_off.assign(b->shell_coef_off, b->shell_coef_off + b->n_shells);
  p->coef.assign(b->coef, b->coef + b->n_coef);

  // radial tables in d = s - r_j (one scaled copy per distinct (offset, rcut, nint))
  {
    std::vector<std::pair<std::pair<int64_t, int32_t>, std::pair<double, int64_t>>> seen;
    p->shell_cs_off.assign(b->n_shells, 0);
    for (int s = 0; s < b->n_shells; ++s) {
      int64_t found = -1;
      for (auto &e : seen)
        if (e.first.first == p->shell_coef_off[s] && e.first.second == p->shell_nint[s] &&
            e.second.first == p->shell_rcut[s]) {
          found = e.second.second;
          break;
        }
      if (found < 0) {
        found = (int64_t)p->coef_scaled.size();
        const int n = p->shell_nint[s];
        const double rc = p->shell_rcut[s];
        for (int j = 0; j < n; ++j) {
          const double h = rc * (2.0 * j + 1.0) / ((double)n * (double)n);
          const double *c = &p->coef[p->shell_coef_off[s] + 4 * (int64_t)j];
          p->coef_scaled.push_back(c[0]);
          p->coef_scaled.push_back(c[1] / h);
          p->coef_scaled.push_back(c[2] / (h * h));
          p->coef_scaled.push_back(c[3] / (h * h * h));
        }
        seen.push_back({{p->shell_coef_off[s], p->shell_nint[s]}, {p->shell_rcut[s], found}});
      }
      p->shell_cs_off[s] = found;
      const double n2 = (double)p->shell_nint[s] * (double)p->shell_nint[s];
      p->shell_knot.push_back(n2 / p->shell_rcut[s]);
      p->shell_knot.push_back(p->shell_rcut[s] / n2);
    }
  }

  // functions and per-atom data
  p->atom_fn_off.assign(na + 1, 0);
  p->atom_rcut.assign(na, 0.0);
  for (int a = 0; a < na; ++a) {
    int nf = 0;
    for (int s = p->atom_shell_off[a]; s < p->atom_shell_off[a + 1]; ++s) {
      nf += 2 * p->shell_l[s] + 1;
      p->atom_rcut[a] = std::max(p->atom_rcut[a], p->shell_rcut[s]);
      for (int m = -p->shell_l[s]; m <= p->shell_l[s]; ++m) {
        p->fn_atom.push_back(a);
        p->fn_shlm.push_back(s * 32 + p->shell_l[s] * p->shell_l[s] + p->shell_l[s] + m);
      }
    }
    p->atom_fn_off[a + 1] = p->atom_fn_off[a] + nf;
  }
  p->n_fn = p->atom_fn_off[na];
  double rmax = 0.0;
  for (double r : p->atom_rcut) rmax = std::max(rmax, r);

  // active points
  CellList cl;
  cl.build(na, p->R.data(), rmax);
  p->n_points = g->n_points;
  std::vector<int32_t> active;
  active.reserve(g->n_points);
  for (int64_t i = 0; i < g->n_points; ++i) {
    double q[3] = {g->x[i], g->y[i], g->z[i]};
    double bl[3] = {q[0] - rmax, q[1] - rmax, q[2] - rmax}, bh[3] = {q[0] + rmax, q[1] + rmax, q[2] + rmax};
    bool hit = false;
    const int32_t sy = psys(i);
    cl.visit_box(bl, bh, [&](int a) {
      if (hit || p->atom_sys[a] != sy) return;
      double dx = q[0] - p->R[3 * a], dy = q[1] - p->R[3 * a + 1], dz = q[2] - p->R[3 * a + 2];
      if (dx * dx + dy * dy + dz * dz < p->atom_rcut[a] * p->atom_rcut[a]) hit = true;
    });
    if (hit) active.push_back((int32_t)i);
  }
  p->n_active = (int64_t)active.size();

  // batching
  const double *xyz[3] = {g->x, g->y, g->z};
  std::vector<int64_t> ends;
  // points arrive system-major (user order), so each system's active points
  // are one contiguous range; each range is bisected on its own
  p->sys_point_off.assign(nsys + 1, 0);
  p->sys_batch_off.assign(nsys + 1, 0);
  {
    int64_t lo = 0;
    for (int sy = 0; sy < nsys; ++sy) {
      int64_t hi = lo;
      while (hi < (int64_t)active.size() && psys(active[hi]) == sy) ++hi;
      if (hi > lo) bisect(active, lo, hi, p->p_max, xyz, ends);
      p->sys_batch_off[sy + 1] = (int64_t)ends.size();
      lo = hi;
    }
    if (lo != (int64_t)active.size()) throw std::invalid_argument("grid points are not ordered by system");
  }
  if (pt_sys) {
    for (int64_t i = 0; i < g->n_points; ++i) p->sys_point_off[pt_sys[i] + 1]++;
    for (int sy = 0; sy < nsys; ++sy) p->sys_point_off[sy + 1] += p->sys_point_off[sy];
  } else {
    p->sys_point_off[1] = g->n_points;
  }
  p->n_batches = (int64_t)ends.size();
  p->perm = active;
  p->px.resize(p->n_active);
  p->py.resize(p->n_active);
  p->pz.resize(p->n_active);
  p->pw.resize(p->n_active);
  for (int64_t i = 0; i < p->n_active; ++i) {
    p->px[i] = g->x[active[i]];
    p->py[i] = g->y[active[i]];
    p->pz[i] = g->z[active[i]];
    p->pw[i] = g->w[active[i]];
  }
  p->batch_pt_off.assign(1, 0);
  for (int64_t e : ends) p->batch_pt_off.push_back((int32_t)e);

  // pairs A <= B within rcut_A + rcut_B
  CellList cl2;
  cl2.build(na, p->R.data(), 2.0 * rmax);
  p->atom_pair_start.assign(na + 1, 0);
  for (int a = 0; a < na; ++a) {
    std::vector<int32_t> nb;
    double q[3] = {p->R[3 * a], p->R[3 * a + 1], p->R[3 * a + 2]};
    double r2 = p->atom_rcut[a] + rmax;
    double bl[3] = {q[0] - r2, q[1] - r2, q[2] - r2}, bh[3] = {q[0] + r2, q[1] + r2, q[2] + r2};
    cl2.visit_box(bl, bh, [&](int c) {
      if (c < a || p->atom_sys[c] != p->atom_sys[a]) return;
      double dx = q[0] - p->R[3 * c], dy = q[1] - p->R[3 * c + 1], dz = q[2] - p->R[3 * c + 2];
      double rc = p->atom_rcut[a] + p->atom_rcut[c];
      if (dx * dx + dy * dy + dz * dz < rc * rc) nb.push_back(c);
    });
    std::sort(nb.begin(), nb.end());
    for (int c : nb) {
      p->pair_a.push_back(a);
      p->pair_b.push_back(c);
    }
    p->atom_pair_start[a + 1] = (int64_t)p->pair_a.size();
  }
  p->n_pairs = (int64_t)p->pair_a.size();
  p->pair_off.assign(p->n_pairs + 1, 0);
  p->pair_na.resize(p->n_pairs);
  p->pair_nb.resize(p->n_pairs);
  for (int64_t q = 0; q < p->n_pairs; ++q) {
    int a = p->pair_a[q], c = p->pair_b[q];
    p->pair_na[q] = p->atom_fn_off[a + 1] - p->atom_fn_off[a];
    p->pair_nb[q] = p->atom_fn_off[c + 1] - p->atom_fn_off[c];
    p->pair_off[q + 1] = p->pair_off[q] + (int64_t)p->pair_na[q] * p->pair_nb[q];
    p->max_pair_block = std::max<int64_t>(p->max_pair_block, (int64_t)p->pair_na[q] * p->pair_nb[q]);
  }
  p->store_len = p->pair_off[p->n_pairs];
  // the batch-to-global sum spreads a pair's five blocks over 256-element
  // workgroups along the grid's second dimension (at most 65535)
  if ((5 * p->max_pair_block + 255) / 256 > 65535)
    return fail(Q4C_EUNSUPPORTED, "an atom pair block has more than 3.3M elements");
  p->sys_pair_off.assign(nsys + 1, 0);
  for (int sy = 0; sy < nsys; ++sy) p->sys_pair_off[sy + 1] = p->atom_pair_start[sys_atom_off[sy + 1]];
  auto pair_index = [&](int a, int c) -> int64_t {
    auto beg = p->pair_b.begin() + p->atom_pair_start[a], end = p->pair_b.begin() + p->atom_pair_start[a + 1];
    auto it = std::lower_bound(beg, end, c);
    if (it == end || *it != c) return -1;
    return it - p->pair_b.begin();
  };

  // per-batch relevant atoms (slots), local functions, staging layout, work, passes
  p->batch_fn_off.assign(1, 0);
  p->batch_slot_off.assign(1, 0);
  p->batch_sp_off.assign(1, 0);
  const int T = q4c::kTile;
  int64_t staging = 0, partial = 0, panel = 0;
  q4c::Pass cur{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<std::pair<int32_t, int64_t>> pass_inc;  // (pair, staging offset) for the current pass
  std::vector<uint8_t> pair_seen(p->n_pairs, 0);
  const int64_t budget_doubles = std::max<int64_t>(p->staging_budget / 8, 1);
  auto close_pass = [&](int64_t b_end) {
    cur.b1 = b_end;
    cur.w1 = (int64_t)p->work.size();
    // region lengths rounded to 64 doubles: the panel region after them stays 512-byte aligned
    staging = (staging + 63) / 64 * 64;
    partial = (partial + 63) / 64 * 64;
    cur.staging_len = staging;
    cur.partial_len = partial;
    cur.panel_len = panel;
    std::stable_sort(pass_inc.begin(), pass_inc.end(),
                     [](const std::pair<int32_t, int64_t> &x, const std::pair<int32_t, int64_t> &y) {
                       return x.first < y.first;
                     });
    cur.r0 = (int64_t)p->red_pair.size();
    for (size_t i = 0; i < pass_inc.size(); ++i) {
      if (i == 0 || pass_inc[i].first != pass_inc[i - 1].first) {
        p->red_pair.push_back(pass_inc[i].first);
        p->red_first.push_back(pair_seen[pass_inc[i].first] ? 0 : 1);
        pair_seen[pass_inc[i].first] = 1;
        p->red_inc_off.push_back((int64_t)p->inc_src.size());
      }
      p->inc_src.push_back(pass_inc[i].second);
    }
    cur.r1 = (int64_t)p->red_pair.size();
    cur.t1 = (int64_t)p->ptile.size();
    p->passes.push_back(cur);
    p->max_scratch = std::max(p->max_scratch, staging + partial + panel);
    pass_inc.clear();
    staging = 0;
    partial = 0;
    panel = 0;
    int64_t nt_ = (int64_t)p->ptile.size();
    cur = q4c::Pass{b_end, b_end, (int64_t)p->work.size(), (int64_t)p->work.size(), 0, 0, nt_, nt_, 0, 0, 0};
  };

  std::vector<int32_t> rel;
  for (int64_t bt = 0; bt < p->n_batches; ++bt) {
    int64_t g0 = p->batch_pt_off[bt], g1 = p->batch_pt_off[bt + 1];
    double bl[3] = {1e300, 1e300, 1e300}, bh[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = g0; i < g1; ++i) {
      double q[3] = {p->px[i], p->py[i], p->pz[i]};
      for (int d = 0; d < 3; ++d) {
        bl[d] = std::min(bl[d], q[d]);
        bh[d] = std::max(bh[d], q[d]);
      }
    }
    double el[3] = {bl[0] - rmax, bl[1] - rmax, bl[2] - rmax}, eh[3] = {bh[0] + rmax, bh[1] + rmax, bh[2] + rmax};
    rel.clear();
    const int32_t bsys = g1 > g0 ? psys(p->perm[g0]) : 0;
    cl.visit_box(el, eh, [&](int a) {
      if (p->atom_sys[a] != bsys) return;
      double rc = p->atom_rcut[a], rc2 = rc * rc;
      // distance from the atom to the batch box
      double dmin2 = 0.0, dmax2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        double c = p->R[3 * a + d];
        double lo = bl[d] - c, hi = bh[d] - c;
        double dn = (lo > 0) ? lo : ((hi < 0) ? -hi : 0.0);
        double df = std::max(std::fabs(lo), std::fabs(hi));
        dmin2 += dn * dn;
        dmax2 += df * df;
      }
      if (!(dmin2 < rc2)) return;
      bool hit = dmax2 < rc2;
      for (int64_t i = g0; i < g1 && !hit; ++i) {
        double dx = p->px[i] - p->R[3 * a], dy = p->py[i] - p->R[3 * a + 1], dz = p->pz[i] - p->R[3 * a + 2];
        if (dx * dx + dy * dy + dz * dz < rc2) hit = true;
      }
      if (hit) rel.push_back(a);
    });
    std::sort(rel.begin(), rel.end());
    int nb_fn = 0;
    for (int a : rel) nb_fn += p->atom_fn_off[a + 1] - p->atom_fn_off[a];
    // staging size of this batch: upper atom-block triangle, five parts
    int64_t bstage = 0;
    {
      int off = 0;
      for (int a : rel) {
        int nf = p->atom_fn_off[a + 1] - p->atom_fn_off[a];
        bstage += 5 * (int64_t)nf * (nb_fn - off);
        off += nf;
      }
    }
    int nt = (nb_fn + T - 1) / T;
    int64_t bpart = 2 * (int64_t)(nt * (nt + 1) / 2) * (g1 - g0);  // two column halves per work item
    // panel: 4 FP64 components (or phi in FP64 and up to 6 FP32 gradient planes: as much)
    // panel: 4 FP64 planes (the largest kind)
    int64_t bpanel = 4 * q4c::pad16(g1 - g0) * q4c::pad16(nb_fn);
    if (bt > cur.b0 && (staging + partial + panel + bstage + bpart + bpanel > budget_doubles)) close_pass(bt);
    p->panel_off.push_back(panel);
    panel += bpanel;
    p->batch_tile_off.push_back((int64_t)p->ptile.size());
    for (int t = 0; t < nt; ++t) p->ptile.push_back(q4c::WorkItem{(int32_t)bt, (int16_t)t, (int16_t)t});
    // slot-pair -> stored pair table (upper triangle)
    {
      const int ns = (int)rel.size();
      for (int si = 0; si < ns; ++si)
        for (int sj = si; sj < ns; ++sj) p->sp_pair.push_back((int32_t)pair_index(rel[si], rel[sj]));
      p->batch_sp_off.push_back((int64_t)p->sp_pair.size());
    }
    // slots
    int off = 0;
    int32_t slot0 = (int32_t)p->slot_atom.size();
    for (size_t si = 0; si < rel.size(); ++si) {
      int a = rel[si];
      int nf = p->atom_fn_off[a + 1] - p->atom_fn_off[a];
      p->slot_atom.push_back(a);
      p->slot_fnoff.push_back(off);
      p->slot_nfn.push_back(nf);
      p->slot_row_off.push_back(staging);
      for (int f = 0; f < nf; ++f) {
        p->loc_fn.push_back(p->atom_fn_off[a] + f);
        p->loc_slot.push_back((int32_t)si);
      }
      // incidences of this row: (a, c) for slots c >= a that form a stored pair
      int64_t col_off = 0;
      for (size_t sj = si; sj < rel.size(); ++sj) {
        int c = rel[sj];
        int nfc = p->atom_fn_off[c + 1] - p->atom_fn_off[c];
        int64_t q = pair_index(a, c);
        if (q >= 0) pass_inc.push_back({(int32_t)q, staging + 5 * (int64_t)nf * col_off});
        col_off += nfc;
      }
      staging += 5 * (int64_t)nf * (nb_fn - off);
      off += nf;
    }
    (void)slot0;
    p->batch_slot_off.push_back((int32_t)p->slot_atom.size());
    p->batch_fn_off.push_back((int32_t)p->loc_fn.size());
    for (int ti = 0; ti < nt; ++ti)
      for (int tj = ti; tj < nt; ++tj) {
        p->work.push_back(q4c::WorkItem{(int32_t)bt, (int16_t)ti, (int16_t)tj});
        // adjoint partials of this work item: two column halves of P doubles at 2 * work_part_off
        p->work_part_off.push_back(partial / 2);
        partial += 2 * (g1 - g0);
      }
    p->max_batch_points = std::max<int64_t>(p->max_batch_points, g1 - g0);
    p->max_batch_fn = std::max<int64_t>(p->max_batch_fn, nb_fn);
    p->flops_alg += 10.0 * (double)(g1 - g0) * (double)nb_fn * (double)nb_fn;
    p->flops_alg_hs += 3.0 * (double)(g1 - g0) * (double)nb_fn * (double)nb_fn;
  }
  close_pass(p->n_batches);
  p->batch_tile_off.push_back((int64_t)p->ptile.size());
  p->red_inc_off.push_back((int64_t)p->inc_src.size());
  p->batch_work_off.assign(p->n_batches + 1, 0);
  for (auto &w : p->work) p->batch_work_off[w.batch + 1]++;
  for (int64_t b = 0; b < p->n_batches; ++b) p->batch_work_off[b + 1] += p->batch_work_off[b];
  p->tab_off.assign(p->n_batches + 1, 0);
  for (int64_t b = 0; b < p->n_batches; ++b)
    p->tab_off[b + 1] = p->tab_off[b] + (int64_t)(p->batch_pt_off[b + 1] - p->batch_pt_off[b]) *
                                            (p->batch_fn_off[b + 1] - p->batch_fn_off[b]);
  p->fn_entries = (int64_t)p->loc_fn.size();
  // per pass: work items by decreasing estimated cost (padded points x active
  // rows x active columns; a diagonal tile computes about half its blocks)
  p->work_order.resize(p->work.size());
  for (const q4c::Pass &ps : p->passes) {
    std::vector<std::pair<double, int32_t>> c;
    c.reserve(ps.w1 - ps.w0);
    for (int64_t w = ps.w0; w < ps.w1; ++w) {
      const q4c::WorkItem &it = p->work[w];
      const int64_t P = p->batch_pt_off[it.batch + 1] - p->batch_pt_off[it.batch];
      const int n = p->batch_fn_off[it.batch + 1] - p->batch_fn_off[it.batch];
      const double rows = std::min(T, n - T * it.ti), cols = std::min(T, n - T * it.tj);
      c.push_back({-(double)q4c::pad16(P) * rows * cols * (it.ti == it.tj ? 0.55 : 1.0), (int32_t)(w - ps.w0)});
    }
    std::stable_sort(c.begin(), c.end(),
                     [](const std::pair<double, int32_t> &x, const std::pair<double, int32_t> &y) {
                       return x.first < y.first;
                     });
    for (size_t i = 0; i < c.size(); ++i) p->work_order[ps.w0 + i] = c[i].second;
  }
  for (int64_t q = 0; q < p->n_pairs; ++q)
    if (!pair_seen[q]) p->untouched_pairs.push_back((int32_t)q);
  if (p->fn_entries >= (int64_t)INT32_MAX) return fail(Q4C_EINVAL, "too many batch-function entries");
  return Q4C_OK;
}

int build_device(q4c_plan *p) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return q4c::hip_fail(e, "hipGetDevice");
  p->device = dev;
  q4c::DevPlan &d = p->dp;
  int rc = Q4C_OK;
#define UP(vec, ptr)                                           \
  do {                                                         \
    rc = upload(p, vec, &ptr);                                 \
    if (rc != Q4C_OK) return rc;                               \
  } while (0)
  double *R, *rcut, *coef, *px, *py, *pz, *pw;
  int32_t *fn_atom, *fn_shlm, *nint, *perm, *bpo, *bfo, *lfn, *lsl, *bso, *sfo, *snf, *pna, *pnb, *pa, *pb;
  int64_t *coff, *sro, *wpo, *poff, *bwo, *toff, *pnoff;
  double *sknot;
  UP(p->R, R);
  UP(p->fn_atom, fn_atom);
  UP(p->fn_shlm, fn_shlm);
  UP(p->shell_rcut, rcut);
  UP(p->shell_nint, nint);
  UP(p->shell_cs_off, coff);
  UP(p->shell_knot, sknot);
  UP(p->coef_scaled, coef);
  UP(p->px, px);
  UP(p->py, py);
  UP(p->pz, pz);
  UP(p->pw, pw);
  UP(p->perm, perm);
  UP(p->batch_pt_off, bpo);
  UP(p->batch_fn_off, bfo);
  UP(p->loc_fn, lfn);
  UP(p->loc_slot, lsl);
  UP(p->batch_slot_off, bso);
  UP(p->slot_fnoff, sfo);
  UP(p->slot_nfn, snf);
  UP(p->slot_row_off, sro);
  UP(p->work_part_off, wpo);
  UP(p->pair_off, poff);
  UP(p->pair_na, pna);
  UP(p->pair_nb, pnb);
  UP(p->pair_a, pa);
  UP(p->pair_b, pb);
  UP(p->batch_work_off, bwo);
  UP(p->tab_off, toff);
  UP(p->panel_off, pnoff);
  UP(p->ptile, p->d_ptile);
  UP(p->work, p->d_work);
  UP(p->red_pair, p->d_red_pair);
  UP(p->red_first, p->d_red_first);
  UP(p->red_inc_off, p->d_red_inc_off);
  UP(p->inc_src, p->d_inc_src);
  UP(p->untouched_pairs, p->d_untouched);
  UP(p->work_order, p->d_order);
  {
    int32_t *spp;
    int64_t *spo;
    UP(p->sp_pair, spp);
    UP(p->batch_sp_off, spo);
    p->dp.sp_pair = spp;
    p->dp.batch_sp_off = spo;
  }
  {
    // packed slot data and the slot's staging row per batch function, and
    // store offsets per slot pair: the contraction epilogue and the adjoint
    // read them in one round trip each instead of two
    int64_t n_b = (int64_t)p->batch_fn_off.size() - 1;
    std::vector<int64_t> linfo(std::max<size_t>(p->loc_slot.size(), 1), 0);
    std::vector<int64_t> lrow(std::max<size_t>(p->loc_slot.size(), 1), 0);
    for (int64_t b = 0; b < n_b; ++b) {
      if (p->batch_fn_off[b + 1] - p->batch_fn_off[b] >= (1 << 20))
        return fail(Q4C_EUNSUPPORTED, "a batch has 2^20 or more relevant functions");
      for (int32_t e = p->batch_fn_off[b]; e < p->batch_fn_off[b + 1]; ++e) {
        const int64_t sl = p->loc_slot[e], so = p->batch_slot_off[b] + sl;
        linfo[e] = sl | ((int64_t)p->slot_fnoff[so] << 20) | ((int64_t)p->slot_nfn[so] << 40);
        lrow[e] = p->slot_row_off[so];
      }
    }
    std::vector<int64_t> sppo(std::max<size_t>(p->sp_pair.size(), 1), -1);
    for (size_t t = 0; t < p->sp_pair.size(); ++t) sppo[t] = p->sp_pair[t] >= 0 ? p->pair_off[p->sp_pair[t]] : -1;
    int64_t *li, *sp;
    int64_t *lr;
    UP(linfo, li);
    UP(lrow, lr);
    UP(sppo, sp);
    d.loc_info = li;
    d.loc_rowoff = lr;
    d.sp_poff = sp;
  }
#undef UP
  rc = device_alloc(p, (size_t)p->max_scratch * sizeof(double), (void **)&p->d_staging);
  if (rc != Q4C_OK) return rc;
  rc = device_alloc(p, 64, (void **)&p->d_flag);
  if (rc != Q4C_OK) return rc;
  rc = device_alloc(p, (size_t)(p->n_active + 16) * sizeof(double), (void **)&p->d_om);
  if (rc != Q4C_OK) return rc;
  rc = device_alloc(p, (size_t)5 * (p->store_len + 16) * sizeof(double), (void **)&p->d_coef_fold);
  if (rc != Q4C_OK) return rc;
  {
    // adjoint positions: the column halves of the work items that start
    // inside their batch, per pass, in batch order and in the work items'
    // cost order
    std::vector<q4c::AdjPos> ab, ac;
    auto add = [&](std::vector<q4c::AdjPos> &v, int64_t w) {
      const q4c::WorkItem &it = p->work[w];
      const int b = it.batch;
      const int f0 = p->batch_fn_off[b], n = p->batch_fn_off[b + 1] - f0;
      const int g0 = p->batch_pt_off[b], P = p->batch_pt_off[b + 1] - g0;
      for (int h = 0; h < 2; ++h) {
        if (it.tj * q4c::kTile + 32 * h >= n) continue;
        q4c::AdjPos a{};
        a.batch = b;
        a.ti = it.ti;
        a.tj = it.tj;
        a.half = h;
        a.f0 = f0;
        a.n = n;
        a.g0 = g0;
        a.P = P;
        a.sbase = p->batch_slot_off[b];
        a.ns = p->batch_slot_off[b + 1] - p->batch_slot_off[b];
        a.panel_off = p->panel_off[b];
        a.spb = p->batch_sp_off[b];
        a.part = 2 * p->work_part_off[w] + (int64_t)h * P;
        v.push_back(a);
      }
    };
    for (q4c::Pass &ps : p->passes) {
      ps.ap0 = (int64_t)ab.size();
      for (int64_t w = ps.w0; w < ps.w1; ++w) add(ab, w);
      for (int64_t i = 0; i < ps.w1 - ps.w0; ++i) add(ac, ps.w0 + p->work_order[ps.w0 + i]);
      ps.ap1 = (int64_t)ab.size();
    }
    if ((rc = upload(p, ab, &p->d_adjpos)) != Q4C_OK) return rc;
    if ((rc = upload(p, ac, &p->d_adjpos_cost)) != Q4C_OK) return rc;
  }
  {
    const size_t nt = 2 * std::max<size_t>(p->passes.size(), 1) * q4c::kTicketsPerLaunch;
    rc = device_alloc(p, nt * sizeof(unsigned), (void **)&p->d_tickets);
    if (rc != Q4C_OK) return rc;
    if (hipMemset(p->d_tickets, 0, nt * sizeof(unsigned)) != hipSuccess) return fail(Q4C_EHIP, "hipMemset");
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) p->n_cu = ncu;
  }
  d.R = R;
  d.fn_atom = fn_atom;
  d.fn_shlm = fn_shlm;
  d.shell_rcut = rcut;
  d.shell_nint = nint;
  d.shell_knot = sknot;
  d.shell_coef_off = coff;
  d.coef = coef;
  d.px = px;
  d.py = py;
  d.pz = pz;
  d.pw = pw;
  d.perm = perm;
  d.batch_pt_off = bpo;
  d.batch_fn_off = bfo;
  d.loc_fn = lfn;
  d.loc_slot = lsl;
  d.batch_slot_off = bso;
  d.slot_fnoff = sfo;
  d.slot_nfn = snf;
  d.slot_row_off = sro;
  d.work_part_off = wpo;
  d.pair_off = poff;
  d.pair_na = pna;
  d.pair_nb = pnb;
  d.pair_a = pa;
  d.pair_b = pb;
  d.batch_work_off = bwo;
  d.tab_off = toff;
  d.panel_off = pnoff;
  d.store_len = p->store_len;
  d.n_active = p->n_active;
  d.n_points = p->n_points;
  d.cprime = 1.0 / (4.0 * p->c_light * p->c_light);
  p->on_device = true;
  return Q4C_OK;
}

int check_plan_dev(const q4c_plan *p) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (!p->on_device) return fail(Q4C_ENODEV, "plan has no device data");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return q4c::hip_fail(e, "hipSetDevice");
  return Q4C_OK;
}

}  // namespace

namespace q4c {
static hipEvent_t take_event(const q4c_plan *p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

TimedLaunch::TimedLaunch(const q4c_plan *p_, int timer_, hipStream_t s_) : p(p_), timer(timer_), s(s_) {
  if (!p->profiling) return;
  e0 = take_event(p);
  e1 = take_event(p);
  if (e0 && e1) (void)hipEventRecord(e0, s);
}

TimedLaunch::~TimedLaunch() {
  if (!e0 || !e1) return;
  (void)hipEventRecord(e1, s);
  p->ev_live.push_back({timer, {e0, e1}});
}

void set_error(const std::string &msg) { g_last_error = msg; }
int fail_status(int code, const char *msg) {
  g_last_error = msg;
  return code;
}
int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return Q4C_EHIP;
}
}  // namespace q4c

extern "C" {

namespace {
int create_plan(const q4c_basis *basis, const q4c_grid *grid, const q4c_opts *opts,
                const std::vector<int64_t> &sys_atom_off, const int32_t *pt_sys, q4c_plan **out) {
  q4c_plan *p = nullptr;
  int rc = Q4C_OK;
  try {
    p = new q4c_plan();
    if (opts) {
      if (opts->c_light > 0.0) p->c_light = opts->c_light;
      if (opts->p_max > 0) p->p_max = opts->p_max;
      p->flags = opts->flags;
      p->staging_budget = opts->staging_bytes;
    }
    if (p->p_max < 1) p->p_max = 300;
    if (p->staging_budget <= 0) p->staging_budget = (int64_t)32 << 30;
    rc = build_host(p, basis, grid, sys_atom_off, pt_sys);
    if (rc == Q4C_OK && !(p->flags & Q4C_PLAN_HOST_ONLY)) rc = build_device(p);
  } catch (const std::bad_alloc &) {
    rc = fail(Q4C_ENOMEM, "host allocation failed");
  } catch (const std::exception &ex) {
    rc = fail(Q4C_EINVAL, ex.what());
  }
  if (rc != Q4C_OK) {
    if (p) {
      free_device(p);
      delete p;
    }
    return rc;
  }
  *out = p;
  return Q4C_OK;
}
}  // namespace

int q4c_plan_create(const q4c_basis *basis, const q4c_grid *grid, const q4c_opts *opts, q4c_plan **out) {
  if (!out) return fail(Q4C_EINVAL, "NULL output handle");
  *out = nullptr;
  int rc = validate(basis, grid);
  if (rc != Q4C_OK) return rc;
  return create_plan(basis, grid, opts, std::vector<int64_t>{0, (int64_t)basis->n_atoms}, nullptr, out);
}

int q4c_plan_create_batched(int32_t n_systems, const q4c_basis *bases, const q4c_grid *grids, const q4c_opts *opts,
                            q4c_plan **out) {
  if (!out) return fail(Q4C_EINVAL, "NULL output handle");
  *out = nullptr;
  if (n_systems < 1 || !bases || !grids) return fail(Q4C_EINVAL, "need n_systems >= 1 basis and grid descriptors");
  for (int sy = 0; sy < n_systems; ++sy) {
    int rc = validate(&bases[sy], &grids[sy]);
    if (rc != Q4C_OK) return rc;
  }
  try {
    // union descriptors: atoms, shells and points system-major; radial tables
    // shared between systems that pass the same coefficient array
    std::vector<double> R, coef, rcut, x, y, z, w;
    std::vector<int32_t> aso{0}, sl, sn, pt_sys;
    std::vector<int64_t> sco, sys_atom_off{0};
    std::vector<std::pair<std::pair<const double *, int64_t>, int64_t>> coef_seen;
    int64_t np = 0;
    for (int sy = 0; sy < n_systems; ++sy) np += grids[sy].n_points;
    if (np >= (int64_t)INT32_MAX) return fail(Q4C_EINVAL, "more than 2^31-1 grid points in total");
    for (int sy = 0; sy < n_systems; ++sy) {
      const q4c_basis &b = bases[sy];
      const q4c_grid &g = grids[sy];
      int64_t cbase = -1;
      for (auto &e : coef_seen)
        if (e.first.first == b.coef && e.first.second == b.n_coef) cbase = e.second;
      if (cbase < 0) {
        cbase = (int64_t)coef.size();
        if (b.n_coef > 0) coef.insert(coef.end(), b.coef, b.coef + b.n_coef);
        coef_seen.push_back({{b.coef, b.n_coef}, cbase});
      }
      const int32_t s0 = (int32_t)sl.size();
      R.insert(R.end(), b.R, b.R + 3 * (size_t)b.n_atoms);
      for (int a = 0; a < b.n_atoms; ++a) aso.push_back(s0 + b.atom_shell_off[a + 1]);
      for (int s = 0; s < b.n_shells; ++s) {
        sl.push_back(b.shell_l[s]);
        rcut.push_back(b.shell_rcut[s]);
        sn.push_back(b.shell_nint[s]);
        sco.push_back(cbase + b.shell_coef_off[s]);
      }
      sys_atom_off.push_back(sys_atom_off.back() + b.n_atoms);
      if (g.n_points > 0) {
        x.insert(x.end(), g.x, g.x + g.n_points);
        y.insert(y.end(), g.y, g.y + g.n_points);
        z.insert(z.end(), g.z, g.z + g.n_points);
        w.insert(w.end(), g.w, g.w + g.n_points);
        pt_sys.insert(pt_sys.end(), (size_t)g.n_points, sy);
      }
    }
    q4c_basis ub{};
    ub.n_atoms = (int32_t)(R.size() / 3);
    ub.R = R.data();
    ub.atom_shell_off = aso.data();
    ub.n_shells = (int32_t)sl.size();
    ub.shell_l = sl.data();
    ub.shell_rcut = rcut.data();
    ub.shell_nint = sn.data();
    ub.shell_coef_off = sco.data();
    ub.n_coef = (int64_t)coef.size();
    ub.coef = coef.data();
    q4c_grid ug{};
    ug.n_points = np;
    ug.x = x.data();
    ug.y = y.data();
    ug.z = z.data();
    ug.w = w.data();
    return create_plan(&ub, &ug, opts, sys_atom_off, pt_sys.data(), out);
  } catch (const std::bad_alloc &) {
    return fail(Q4C_ENOMEM, "host allocation failed");
  }
}

int q4c_plan_systems(const q4c_plan *p, int64_t *atom_off, int64_t *point_off, int64_t *batch_off,
                     int64_t *pair_off, int64_t *store_off) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  for (int sy = 0; sy <= p->n_systems; ++sy) {
    if (atom_off) atom_off[sy] = p->sys_atom_off[sy];
    if (point_off) point_off[sy] = p->sys_point_off[sy];
    if (batch_off) batch_off[sy] = p->sys_batch_off[sy];
    if (pair_off) pair_off[sy] = p->sys_pair_off[sy];
    if (store_off) store_off[sy] = p->pair_off[p->sys_pair_off[sy]];
  }
  return Q4C_OK;
}

void q4c_plan_destroy(q4c_plan *plan) {
  if (!plan) return;
  free_device(plan);
  delete plan;
}

int q4c_plan_info(const q4c_plan *p, q4c_info *info) {
  if (!p || !info) return fail(Q4C_EINVAL, "NULL argument");
  info->n_atoms = p->n_atoms;
  info->n_systems = p->n_systems;
  info->scratch_bytes = p->max_scratch * (int64_t)sizeof(double);
  info->n_fn = p->n_fn;
  info->n_points = p->n_points;
  info->n_active = p->n_active;
  info->n_batches = p->n_batches;
  info->n_pairs = p->n_pairs;
  info->store_len = p->store_len;
  info->fn_entries = p->fn_entries;
  info->max_batch_points = p->max_batch_points;
  info->max_batch_fn = p->max_batch_fn;
  info->n_work = (int64_t)p->work.size();
  info->n_passes = (int64_t)p->passes.size();
  info->device_bytes = p->device_bytes;
  info->flops_alg = p->flops_alg;
  info->flops_alg_hs = p->flops_alg_hs;
  info->staging_bytes = 0;
  for (const q4c::Pass &ps : p->passes) info->staging_bytes += ps.staging_len * (int64_t)sizeof(double);
  info->tab_elems = p->n_batches > 0 ? p->tab_off[p->n_batches] : 0;
  return Q4C_OK;
}

int q4c_plan_pairs(const q4c_plan *p, int32_t *pair_atoms, int64_t *pair_off) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (pair_atoms)
    for (int64_t q = 0; q < p->n_pairs; ++q) {
      pair_atoms[2 * q] = p->pair_a[q];
      pair_atoms[2 * q + 1] = p->pair_b[q];
    }
  if (pair_off) std::copy(p->pair_off.begin(), p->pair_off.end(), pair_off);
  return Q4C_OK;
}

int q4c_plan_batches(const q4c_plan *p, int64_t *pt_off, int64_t *point_index, int64_t *fn_off, int32_t *fn_index) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (pt_off)
    for (int64_t b = 0; b <= p->n_batches; ++b) pt_off[b] = p->batch_pt_off[b];
  if (point_index)
    for (int64_t i = 0; i < p->n_active; ++i) point_index[i] = p->perm[i];
  if (fn_off)
    for (int64_t b = 0; b <= p->n_batches; ++b) fn_off[b] = p->batch_fn_off[b];
  if (fn_index) std::copy(p->loc_fn.begin(), p->loc_fn.end(), fn_index);
  return Q4C_OK;
}

int q4c_store_layout(const q4c_plan *p, q4c_layout *layout, int32_t *pair_atoms, int64_t *pair_off,
                     int32_t *pair_nfn) {
  if (!p || !layout) return fail(Q4C_EINVAL, "NULL argument");
  layout->n_pairs = p->n_pairs;
  layout->store_len = p->store_len;
  layout->part_bytes = 8 * p->store_len;
  layout->store_bytes = 40 * p->store_len;
  layout->hs_bytes = 16 * p->store_len;
  layout->spinor_bytes = 64 * p->store_len;
  for (int64_t q = 0; q < p->n_pairs; ++q) {
    if (pair_atoms) {
      pair_atoms[2 * q] = p->pair_a[q];
      pair_atoms[2 * q + 1] = p->pair_b[q];
    }
    if (pair_nfn) {
      pair_nfn[2 * q] = p->pair_na[q];
      pair_nfn[2 * q + 1] = p->pair_nb[q];
    }
  }
  if (pair_off)
    for (int64_t q = 0; q <= p->n_pairs; ++q) pair_off[q] = p->pair_off[q];
  return Q4C_OK;
}

int q4c_tabulate_size(const q4c_plan *p, int64_t b0, int64_t b1, int32_t deriv, int64_t *n) {
  if (!p || !n) return fail(Q4C_EINVAL, "NULL argument");
  if (b0 < 0 || b1 < b0 || b1 > p->n_batches) return fail(Q4C_EINVAL, "batch range outside the plan");
  if (deriv != 0 && deriv != 1) return fail(Q4C_EINVAL, "deriv must be 0 or 1");
  int64_t tot = 0;
  for (int64_t b = b0; b < b1; ++b)
    tot += (int64_t)(p->batch_pt_off[b + 1] - p->batch_pt_off[b]) * (p->batch_fn_off[b + 1] - p->batch_fn_off[b]);
  *n = tot * (deriv ? 4 : 1);
  return Q4C_OK;
}

int nao_tabulate(const q4c_plan *p, int64_t b0, int64_t b1, int32_t deriv, int32_t dtype, void *out_dev,
                 int64_t out_bytes, void *stream) {
  int64_t need = 0;
  int rc = q4c_tabulate_size(p, b0, b1, deriv, &need);
  if (rc != Q4C_OK) return rc;
  if (dtype != Q4C_DTYPE_F64 && dtype != Q4C_DTYPE_F32_HILO) return fail(Q4C_EINVAL, "unknown dtype");
  if (out_bytes < 8 * need) return fail(Q4C_ESIZE, "output buffer too small for nao_tabulate");
  if (need > 0 && !out_dev) return fail(Q4C_EINVAL, "NULL output");
  rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  if (need == 0) return Q4C_OK;
  return q4c::launch_tabulate(p, b0, b1, deriv, dtype, out_dev, (hipStream_t)stream);
}

namespace {
// Replays one captured HIP graph per distinct call (kind, buffers, options);
// the first call of each captures the launch sequence on the plan's capture
// stream.  Graphs never contain memset nodes: all clearing is done by kernels.
int run_graph(const q4c_plan *p, int kind, const void *in, void *o0, void *o1, void *o2, int64_t a, int64_t b,
              int64_t c, hipStream_t user, const std::function<int(hipStream_t)> &body) {
  using GE = q4c_plan::GraphEntry;
  const GE *hit = nullptr;
  for (const GE &g : p->graphs)
    if (g.kind == kind && g.in == in && g.out0 == o0 && g.out1 == o1 && g.out2 == o2 && g.a == a && g.b == b &&
        g.c == c)
      hit = &g;
  if (!hit) {
    hipError_t e;
    if (!p->capture_stream) {
      e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return q4c::hip_fail(e, "hipStreamCreateWithFlags");
    }
    e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return q4c::hip_fail(e, "hipStreamBeginCapture");
    const int rc = body(p->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->capture_stream, &graph);
    if (rc != Q4C_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return q4c::hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return q4c::hip_fail(e, "hipGraphInstantiate");
    }
    if (p->graphs.size() >= 16) {  // bounded cache: drop the oldest once nothing runs
      (void)hipDeviceSynchronize();
      (void)hipGraphExecDestroy(p->graphs.front().exec);
      (void)hipGraphDestroy(p->graphs.front().graph);
      p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back(GE{kind, in, o0, o1, o2, a, b, c, graph, exec});
    hit = &p->graphs.back();
  }
  hipError_t e = hipGraphLaunch(hit->exec, user);
  if (e != hipSuccess) return q4c::hip_fail(e, "hipGraphLaunch");
  return Q4C_OK;
}

void drop_graphs(q4c_plan *p) {
  if (p->graphs.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto &g : p->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  p->graphs.clear();
}
}  // namespace

int q4c_integrate_H(const q4c_plan *p, const double *v_dev, int32_t precision, uint32_t parts, uint32_t flags,
                    double *store_dev, double *spin_w_dev, double *spin_v_dev, void *stream) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (precision != Q4C_PREC_F64 && precision != Q4C_PREC_SPLIT_F32 && precision != Q4C_PREC_F32 &&
      precision != Q4C_PREC_BF16X3 && precision != Q4C_PREC_F64_VALU)
    return fail(Q4C_EINVAL, "unknown precision");
  if (parts == 0 || (parts & ~(uint32_t)Q4C_PART_ALL)) return fail(Q4C_EINVAL, "bad part selection");
  if (flags & ~(uint32_t)(Q4C_ACCUMULATE | Q4C_ASSEMBLE_W | Q4C_ASSEMBLE_V | Q4C_CHECK_FINITE))
    return fail(Q4C_EINVAL, "unknown flag");
  if ((flags & Q4C_ASSEMBLE_W) && (parts & (Q4C_PART_WS | Q4C_PART_WSO)) != (Q4C_PART_WS | Q4C_PART_WSO))
    return fail(Q4C_EINVAL, "the W spinor blocks need the Ws and Wso parts");
  if ((flags & Q4C_ASSEMBLE_V) && !(parts & Q4C_PART_V)) return fail(Q4C_EINVAL, "the V spinor blocks need V");
  if (p->n_points > 0 && !v_dev) return fail(Q4C_EINVAL, "NULL potential");
  if (p->store_len > 0 && !store_dev) return fail(Q4C_EINVAL, "NULL store");
  if ((flags & Q4C_ASSEMBLE_W) && p->store_len > 0 && !spin_w_dev) return fail(Q4C_EINVAL, "NULL W spinor output");
  if ((flags & Q4C_ASSEMBLE_V) && p->store_len > 0 && !spin_v_dev) return fail(Q4C_EINVAL, "NULL V spinor output");
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  if (flags & Q4C_CHECK_FINITE) {
    bool ok = true;
    rc = q4c::launch_check_finite(p, v_dev, (hipStream_t)stream, &ok);
    if (rc != Q4C_OK) return rc;
    if (!ok) return fail(Q4C_ENONFINITE, "potential contains NaN or Inf");
  }
  p->panel_pass = -1;
  if (p->use_graphs && !p->profiling) {
    const uint32_t f = flags & ~(uint32_t)Q4C_CHECK_FINITE;
    rc = run_graph(p, 0, v_dev, store_dev, spin_w_dev, spin_v_dev, precision, f, parts, (hipStream_t)stream,
                   [&](hipStream_t cs) {
                     return q4c::launch_integrate(p, v_dev, precision, parts, f, store_dev, spin_w_dev, spin_v_dev,
                                                  cs);
                   });
  } else {
    rc = q4c::launch_integrate(p, v_dev, precision, parts, flags, store_dev, spin_w_dev, spin_v_dev,
                               (hipStream_t)stream);
  }
  // an FP64 call with W parts tabulates FP64 panels of phi and its gradient
  // (the adjoint's operands) in every pass; the last pass's stay resident
  if (rc == Q4C_OK && precision == Q4C_PREC_F64 && (parts & (Q4C_PART_WS | Q4C_PART_WSO)))
    p->panel_pass = (int64_t)p->passes.size() - 1;
  return rc;
}

int q4c_plan_set_ket_potential(q4c_plan *p, const int64_t *shell_u_off, int64_t n_u, const double *u_coef) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  int rc = Q4C_OK;
  if (n_u < 0) return fail(Q4C_EINVAL, "negative table length");
  if (p->n_shells > 0 && (!shell_u_off || !u_coef)) return fail(Q4C_EINVAL, "NULL ket-potential table");
  for (int s = 0; s < p->n_shells; ++s) {
    if (shell_u_off[s] < 0 || shell_u_off[s] % 4 != 0 || shell_u_off[s] + 4 * (int64_t)p->shell_nint[s] > n_u)
      return fail(Q4C_EINVAL, "ket-potential table outside u_coef (or offset not a multiple of 4)");
  }
  if (n_u > 0 && !finite_all(u_coef, n_u)) return fail(Q4C_EINVAL, "non-finite ket-potential coefficient");
  // the same scaling as the radial tables: (c0, c1/h, c2/h^2, c3/h^3) per interval
  std::vector<double> scaled;
  std::vector<int64_t> off(p->n_shells, 0);
  std::vector<std::pair<std::pair<int64_t, int32_t>, std::pair<double, int64_t>>> seen;
  for (int s = 0; s < p->n_shells; ++s) {
    int64_t found = -1;
    for (auto &e : seen)
      if (e.first.first == shell_u_off[s] && e.first.second == p->shell_nint[s] && e.second.first == p->shell_rcut[s]) {
        found = e.second.second;
        break;
      }
    if (found < 0) {
      found = (int64_t)scaled.size();
      const int n = p->shell_nint[s];
      const double rc = p->shell_rcut[s];
      for (int j = 0; j < n; ++j) {
        const double h = rc * (2.0 * j + 1.0) / ((double)n * (double)n);
        const double *c = u_coef + shell_u_off[s] + 4 * (int64_t)j;
        scaled.push_back(c[0]);
        scaled.push_back(c[1] / h);
        scaled.push_back(c[2] / (h * h));
        scaled.push_back(c[3] / (h * h * h));
      }
      seen.push_back({{shell_u_off[s], p->shell_nint[s]}, {p->shell_rcut[s], found}});
    }
    off[s] = found;
  }
  p->ucoef_scaled.swap(scaled);
  p->shell_us_off.swap(off);
  if (!p->on_device) return Q4C_OK;  // host-only plan: validated and kept
  // new device copies; earlier ones stay allocated until the plan is destroyed
  // (captured graphs may still hold their addresses)
  if ((rc = check_plan_dev(p)) != Q4C_OK) return rc;
  double *d_u = nullptr;
  int64_t *d_off = nullptr;
  if ((rc = upload(p, p->ucoef_scaled, &d_u)) != Q4C_OK) return rc;
  if ((rc = upload(p, p->shell_us_off, &d_off)) != Q4C_OK) return rc;
  p->d_ucoef = d_u;
  p->d_shell_us_off = d_off;
  p->dp.ucoef = d_u;
  p->dp.shell_u_off = d_off;
  drop_graphs(p);
  return Q4C_OK;
}

namespace {

// C_alpha (spin 0, m_s = +1/2) or C_beta (spin 1) of Eq. 10 for j = j2/2,
// m_j = mj2/2: a = 2(j - l); C_alpha = a sqrt((l + a m_j + 1/2)/(2l+1)),
// C_beta = sqrt((l - a m_j + 1/2)/(2l+1)).
double spinor_cg(int l, int j2, int mj2, int spin) {
  const int a = j2 - 2 * l;
  const double mj = 0.5 * mj2;
  const double r = spin == 0 ? l + a * mj + 0.5 : l - a * mj + 0.5;
  const double v = std::sqrt(std::max(r, 0.0) / (2.0 * l + 1.0));
  return spin == 0 ? a * v : v;
}

// The Condon-Shortley complex harmonic Y~_l^m in terms of the real harmonics
// of App. B (which carry (-1)^m themselves): m > 0: (Y_m + i Y_-m)/sqrt2;
// m < 0: (-1)^m (Y_|m| - i Y_-|m|)/sqrt2; m = 0: Y_0.  Writes up to two
// (m', re, im); returns their number.
int complex_harmonic(int m, int *mp, double *re, double *im) {
  const double h = 0.70710678118654752440;
  if (m == 0) {
    mp[0] = 0;
    re[0] = 1.0;
    im[0] = 0.0;
    return 1;
  }
  if (m > 0) {
    mp[0] = m, re[0] = h, im[0] = 0.0;
    mp[1] = -m, re[1] = 0.0, im[1] = h;
    return 2;
  }
  const double sg = (-m) & 1 ? -1.0 : 1.0;
  mp[0] = -m, re[0] = sg * h, im[0] = 0.0;
  mp[1] = m, re[1] = 0.0, im[1] = -sg * h;
  return 2;
}

// The relation table of the scalar -> spinor transformation (the global form
// of Algorithm 1: here every plan holds the whole system): spinor functions
// per atom (large shells in order; kappa = -(l+1), then kappa = l for l >= 1;
// m_j ascending), each tied to its large shell and to the small shell of the
// same (shell, kappa), which the small plan must list right after one another
// (l + 1, then l - 1).  Coefficient types are shared by all spinors of one
// (l, kappa, m_j).
int build_spinor_tables(const q4c_plan *pl, const q4c_plan *ps) {
  if (ps->n_atoms != pl->n_atoms || ps->R != pl->R)
    return fail(Q4C_EINVAL, "spinor transform: the two plans have different atoms");
  if (ps->n_pairs != pl->n_pairs || ps->pair_a != pl->pair_a || ps->pair_b != pl->pair_b)
    return fail(Q4C_EINVAL, "spinor transform: the two plans have different atom pairs");
  std::vector<q4c::SpinorType> types;
  std::vector<std::array<int, 3>> type_key;
  std::vector<q4c::SpinorFn> fns;
  std::vector<int32_t> sp_off(pl->n_atoms + 1, 0), nL(pl->n_atoms), nS(pl->n_atoms);
  for (int a = 0; a < pl->n_atoms; ++a) {
    sp_off[a] = (int32_t)fns.size();
    int offL = 0, offS = 0, ks = ps->atom_shell_off[a];
    for (int sh = pl->atom_shell_off[a]; sh < pl->atom_shell_off[a + 1]; ++sh) {
      const int l = pl->shell_l[sh];
      for (int kk = 0; kk < (l >= 1 ? 2 : 1); ++kk) {
        const int kappa = kk == 0 ? -(l + 1) : l;
        const int lt = kappa < 0 ? l + 1 : l - 1;
        if (ks >= ps->atom_shell_off[a + 1] || ps->shell_l[ks] != lt)
          return fail(Q4C_EINVAL, "spinor transform: the small plan's shells do not pair with the large plan's "
                                  "(expected l+1, then l-1 after every large shell of l)");
        const int j2 = 2 * (kappa < 0 ? -kappa : kappa) - 1;
        for (int mj2 = -j2; mj2 <= j2; mj2 += 2) {
          int t = -1;
          for (size_t u = 0; u < type_key.size(); ++u)
            if (type_key[u][0] == l && type_key[u][1] == kappa && type_key[u][2] == mj2) t = (int)u;
          if (t < 0) {
            q4c::SpinorType T{};
            for (int c = 0; c < 2; ++c) {
              const int lc = c == 0 ? l : lt;
              for (int spin = 0; spin < 2; ++spin) {
                const int ml2 = mj2 - (spin == 0 ? 1 : -1);
                const int ml = ml2 / 2;
                T.n[c][spin] = 0;
                if (ml < -lc || ml > lc) continue;
                const double cg = spinor_cg(lc, j2, mj2, spin);
                int mp[2];
                double re[2], im[2];
                const int k = complex_harmonic(ml, mp, re, im);
                for (int e = 0; e < k; ++e) {
                  T.m[c][spin][e] = mp[e] + lc;
                  T.re[c][spin][e] = cg * re[e];
                  T.im[c][spin][e] = cg * im[e];
                }
                T.n[c][spin] = k;
              }
            }
            t = (int)types.size();
            types.push_back(T);
            type_key.push_back({l, kappa, mj2});
          }
          fns.push_back(q4c::SpinorFn{offL, offS, t});
        }
        offS += 2 * lt + 1;
        ++ks;
      }
      offL += 2 * l + 1;
    }
    if (ks != ps->atom_shell_off[a + 1])
      return fail(Q4C_EINVAL, "spinor transform: the small plan has extra shells on an atom");
    nL[a] = offL;
    nS[a] = offS;
  }
  sp_off[pl->n_atoms] = (int32_t)fns.size();
  // reverse relations: for every scalar function of each component, the
  // spinor functions of its atom it enters, per spin (at most 4 for the large
  // component: two m_l of the complex harmonic x two kappa; 2 for the small)
  std::vector<int32_t> fL(pl->n_atoms, 0), fS(pl->n_atoms, 0);
  for (int a = 1; a < pl->n_atoms; ++a) {
    fL[a] = fL[a - 1] + nL[a - 1];
    fS[a] = fS[a - 1] + nS[a - 1];
  }
  std::vector<q4c::ScalarRel> relL(pl->n_atoms ? fL.back() + nL.back() : 0),
      relS(pl->n_atoms ? fS.back() + nS.back() : 0);
  for (auto &r : relL) r = q4c::ScalarRel{};
  for (auto &r : relS) r = q4c::ScalarRel{};
  for (int a = 0; a < pl->n_atoms; ++a)
    for (int mu = 0; mu < sp_off[a + 1] - sp_off[a]; ++mu) {
      const q4c::SpinorFn &f = fns[sp_off[a] + mu];
      const q4c::SpinorType &T = types[f.type];
      for (int c = 0; c < 2; ++c)
        for (int spin = 0; spin < 2; ++spin)
          for (int k = 0; k < T.n[c][spin]; ++k) {
            q4c::ScalarRel &r = c == 0 ? relL[fL[a] + f.offL + T.m[c][spin][k]] : relS[fS[a] + f.offS + T.m[c][spin][k]];
            const int e = r.n[spin]++;
            if (e >= 4) return fail(Q4C_EUNSUPPORTED, "spinor transform: more than 4 spinors per scalar function");
            r.mu[spin][e] = mu;
            r.re[spin][e] = T.re[c][spin][k];
            r.im[spin][e] = T.im[c][spin][k];
          }
    }
  q4c_plan *mp = const_cast<q4c_plan *>(pl);  // device tables cached on the plan
  int rc;
  if ((rc = upload(mp, types, &mp->d_sp_types)) != Q4C_OK) return rc;
  if ((rc = upload(mp, fns, &mp->d_sp_fns)) != Q4C_OK) return rc;
  if ((rc = upload(mp, sp_off, &mp->d_sp_off)) != Q4C_OK) return rc;
  if ((rc = upload(mp, nL, &mp->d_sp_nL)) != Q4C_OK) return rc;
  if ((rc = upload(mp, nS, &mp->d_sp_nS)) != Q4C_OK) return rc;
  std::vector<int64_t> poffS(ps->pair_off.begin(), ps->pair_off.begin() + ps->n_pairs + 1);
  if ((rc = upload(mp, poffS, &mp->d_sp_poffS)) != Q4C_OK) return rc;
  if ((rc = upload(mp, relL, &mp->d_sp_relL)) != Q4C_OK) return rc;
  if ((rc = upload(mp, relS, &mp->d_sp_relS)) != Q4C_OK) return rc;
  if ((rc = upload(mp, fL, &mp->d_sp_fL)) != Q4C_OK) return rc;
  if ((rc = upload(mp, fS, &mp->d_sp_fS)) != Q4C_OK) return rc;
  pl->sp_small = ps;
  pl->sp_small_fn = ps->n_fn;
  pl->sp_small_len = ps->store_len;
  pl->sp_store_len_S = ps->store_len;
  return Q4C_OK;
}

}  // namespace

int q4c_spinor_transform(const q4c_plan *pl, const q4c_plan *ps, const double *hs_large_dev,
                         const double *hs_small_dev, double *h_dev, double *s_dev, void *stream) {
  if (!pl || !ps) return fail(Q4C_EINVAL, "NULL plan");
  int rc = check_plan_dev(ps);
  if (rc != Q4C_OK) return rc;
  if ((rc = check_plan_dev(pl)) != Q4C_OK) return rc;
  if (ps->device != pl->device) return fail(Q4C_EINVAL, "spinor transform: plans on different devices");
  if (pl->store_len > 0 && (!hs_large_dev || !h_dev || !s_dev)) return fail(Q4C_EINVAL, "NULL H/S or output");
  if (ps->store_len > 0 && !hs_small_dev) return fail(Q4C_EINVAL, "NULL small-component H/S");
  if (pl->sp_small != ps || pl->sp_small_fn != ps->n_fn || pl->sp_small_len != ps->store_len) {
    // tables for this small plan (validated; earlier copies stay allocated until destroy)
    if ((rc = build_spinor_tables(pl, ps)) != Q4C_OK) {
      pl->sp_small = nullptr;
      return rc;
    }
  }
  return q4c::launch_spinor_transform(pl, hs_large_dev, hs_small_dev, h_dev, s_dev, (hipStream_t)stream);
}

int q4c_spinor_density_to_scalar(const q4c_plan *pl, const q4c_plan *ps, const double *d_dev, double *cl_dev,
                                 double *cs_dev, void *stream) {
  if (!pl || !ps) return fail(Q4C_EINVAL, "NULL plan");
  int rc = check_plan_dev(ps);
  if (rc != Q4C_OK) return rc;
  if ((rc = check_plan_dev(pl)) != Q4C_OK) return rc;
  if (ps->device != pl->device) return fail(Q4C_EINVAL, "spinor transform: plans on different devices");
  if (pl->store_len > 0 && (!d_dev || !cl_dev)) return fail(Q4C_EINVAL, "NULL density or output");
  if (ps->store_len > 0 && !cs_dev) return fail(Q4C_EINVAL, "NULL small-component output");
  if (pl->sp_small != ps || pl->sp_small_fn != ps->n_fn || pl->sp_small_len != ps->store_len) {
    if ((rc = build_spinor_tables(pl, ps)) != Q4C_OK) {
      pl->sp_small = nullptr;
      return rc;
    }
  }
  return q4c::launch_spinor_to_scalar(pl, d_dev, cl_dev, cs_dev, (hipStream_t)stream);
}

// The work items and buffers of density_gradient_on_grid (built on its first
// call): per pass the product's items (batch, 64-point tile, 64-function
// tile) and the dense-M items (batch, 64 x 64 tile rt <= ct), per batch the
// pass-relative offsets of its dense M (np x np doubles) and of its partials
// (function tiles x 4 x Pp doubles), per batch function its packed slot data
// (slot | slot's first function << 20 | its count << 40), and the M and
// partial buffers of the largest pass.
static int build_grad_tables(const q4c_plan *p) {
  const int64_t nb = (int64_t)p->batch_pt_off.size() - 1;
  std::vector<int32_t> items, cditems;
  std::vector<int64_t> cd_off(std::max<int64_t>(nb, 1), 0), part_off(std::max<int64_t>(nb, 1), 0);
  std::vector<int64_t> item_off(1, 0), cd_item_off(1, 0);
  int64_t max_cd = 0, max_part = 0;
  for (const auto &ps : p->passes) {
    int64_t cd = 0, part = 0;
    for (int64_t b = ps.b0; b < ps.b1; ++b) {
      const int64_t Pp = q4c::pad16(p->batch_pt_off[b + 1] - p->batch_pt_off[b]);
      const int64_t np = q4c::pad16(p->batch_fn_off[b + 1] - p->batch_fn_off[b]);
      const int64_t ntp = (Pp + 63) / 64, nti = (np + 63) / 64;
      cd_off[b] = cd;
      part_off[b] = part;
      cd += np * np;
      part += nti * 4 * Pp;
      for (int64_t tp = 0; tp < ntp; ++tp)
        for (int64_t ti = 0; ti < nti; ++ti) {
          items.push_back((int32_t)b);
          items.push_back((int32_t)tp);
          items.push_back((int32_t)ti);
        }
      for (int64_t rt = 0; rt < nti; ++rt)
        for (int64_t ct = rt; ct < nti; ++ct) {
          cditems.push_back((int32_t)b);
          cditems.push_back((int32_t)rt);
          cditems.push_back((int32_t)ct);
        }
    }
    max_cd = std::max(max_cd, cd);
    max_part = std::max(max_part, part);
    item_off.push_back((int64_t)items.size() / 3);
    cd_item_off.push_back((int64_t)cditems.size() / 3);
  }
  if (items.empty()) items.assign(3, 0);
  if (cditems.empty()) cditems.assign(3, 0);
  // per relevant function: batch-local slot (20 bits), the slot's first
  // batch-local function (20 bits) and its function count
  std::vector<int64_t> fninfo(std::max<size_t>(p->loc_slot.size(), 1), 0);
  for (int64_t b = 0; b < nb; ++b)
    if (p->batch_fn_off[b + 1] - p->batch_fn_off[b] >= (1 << 20))
      return fail(Q4C_EUNSUPPORTED, "a batch has 2^20 or more relevant functions");
  for (int64_t b = 0; b < nb; ++b)
    for (int32_t e = p->batch_fn_off[b]; e < p->batch_fn_off[b + 1]; ++e) {
      const int64_t sl = p->loc_slot[e], so = p->batch_slot_off[b] + sl;
      fninfo[e] = sl | ((int64_t)p->slot_fnoff[so] << 20) | ((int64_t)p->slot_nfn[so] << 40);
    }
  q4c_plan *w = const_cast<q4c_plan *>(p);
  int rc;
  if ((rc = upload(w, fninfo, &w->d_gr_fninfo)) != Q4C_OK) return rc;
  if ((rc = upload(w, items, &w->d_gr_items)) != Q4C_OK) return rc;
  if ((rc = upload(w, cditems, &w->d_gr_cditems)) != Q4C_OK) return rc;
  if ((rc = upload(w, cd_off, &w->d_gr_cd_off)) != Q4C_OK) return rc;
  if ((rc = upload(w, part_off, &w->d_gr_part_off)) != Q4C_OK) return rc;
  void *ptr = nullptr;
  if ((rc = device_alloc(w, (size_t)(max_cd + 64) * sizeof(double), &ptr)) != Q4C_OK) return rc;
  w->d_gr_cd = (double *)ptr;
  if ((rc = device_alloc(w, (size_t)(max_part + 64) * sizeof(double), &ptr)) != Q4C_OK) return rc;
  w->d_gr_part = (double *)ptr;
  w->gr_item_off = item_off;
  w->gr_cd_item_off = cd_item_off;
  return Q4C_OK;
}

int density_gradient_on_grid(const q4c_plan *p, const double *coef_dev, double *out_dev, void *stream) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (p->store_len > 0 && !coef_dev) return fail(Q4C_EINVAL, "NULL coefficients");
  if (p->n_points > 0 && !out_dev) return fail(Q4C_EINVAL, "NULL output");
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  if (p->gr_item_off.empty() && (rc = build_grad_tables(p)) != Q4C_OK) return rc;
  p->panel_pass = -1;
  rc = q4c::launch_density_grad(p, coef_dev, out_dev, (hipStream_t)stream);
  // every pass tabulates its W-path panels; the last pass's stay resident
  if (rc == Q4C_OK) p->panel_pass = (int64_t)p->passes.size() - 1;
  return rc;
}

int q4c_plan_set_cells(q4c_plan *p, int32_t n_cell_atoms, const int32_t *cell_atom, const double *shift) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (n_cell_atoms <= 0 || n_cell_atoms > p->n_atoms) return fail(Q4C_EINVAL, "n_cell_atoms out of range");
  if (p->n_atoms > 0 && (!cell_atom || !shift)) return fail(Q4C_EINVAL, "NULL cell map");
  if (p->n_systems != 1) return fail(Q4C_EUNSUPPORTED, "periodic cells need a single-system plan");
  std::vector<int32_t> nf(n_cell_atoms, -1);
  for (int a = 0; a < p->n_atoms; ++a) {
    const int c = cell_atom[a];
    if (c < 0 || c >= n_cell_atoms) return fail(Q4C_EINVAL, "cell_atom out of range");
    if (!finite_all(shift + 3 * a, 3)) return fail(Q4C_EINVAL, "non-finite shift");
    const int n = p->atom_fn_off[a + 1] - p->atom_fn_off[a];
    if (nf[c] < 0) nf[c] = n;
    if (nf[c] != n) return fail(Q4C_EINVAL, "an image has a different basis than its cell atom");
  }
  for (int c = 0; c < n_cell_atoms; ++c)
    if (nf[c] < 0) return fail(Q4C_EINVAL, "a cell atom has no copy in the plan");
  // contributions per cell pair (a <= b): every stored pair (A', B') in the
  // orientation whose cell atoms ascend (both orientations when A' != B' and
  // both map to one cell atom)
  std::map<std::pair<int, int>, std::vector<std::pair<int64_t, int>>> contrib;  // -> (pair, flag)
  for (int64_t q = 0; q < p->n_pairs; ++q) {
    const int A = p->pair_a[q], B = p->pair_b[q];
    const int a = cell_atom[A], b = cell_atom[B];
    if (a <= b) contrib[{a, b}].push_back({q, 0});
    if (A != B && b <= a) contrib[{b, a}].push_back({q, 1});
  }
  std::vector<int32_t> ca, cb, ct_pair, ct_flag;
  std::vector<int64_t> coff(1, 0), ctoff(1, 0);
  std::vector<double> ct_T;
  for (auto &kv : contrib) {
    const int a = kv.first.first, b = kv.first.second;
    ca.push_back(a);
    cb.push_back(b);
    coff.push_back(coff.back() + (int64_t)nf[a] * nf[b]);
    for (auto &e : kv.second) {
      const int A = p->pair_a[e.first], B = p->pair_b[e.first];
      // phase exp(i k.(T_col - T_row)): rows of the target block are the row atom's images
      const int rowat = e.second ? B : A, colat = e.second ? A : B;
      ct_pair.push_back((int32_t)e.first);
      ct_flag.push_back(e.second);
      for (int d = 0; d < 3; ++d) ct_T.push_back(shift[3 * colat + d] - shift[3 * rowat + d]);
    }
    ctoff.push_back((int64_t)ct_pair.size());
  }
  p->n_cell_atoms = n_cell_atoms;
  p->cell_atom.assign(cell_atom, cell_atom + p->n_atoms);
  p->cp_a = ca;
  p->cp_b = cb;
  p->cp_off = coff;
  p->n_contrib = (int64_t)ct_pair.size();
  // per stored pair: its cell pair (a <= b), whether it is reached transposed
  // (cell atoms a > b), and T_B' - T_A' (the reverse sum)
  std::map<std::pair<int, int>, int32_t> cp_index;
  for (size_t c = 0; c < ca.size(); ++c) cp_index[{ca[c], cb[c]}] = (int32_t)c;
  std::vector<int32_t> pc_cp(p->n_pairs), pc_flag(p->n_pairs);
  std::vector<double> pc_T(3 * p->n_pairs);
  for (int64_t q = 0; q < p->n_pairs; ++q) {
    const int A = p->pair_a[q], B = p->pair_b[q];
    const int a = cell_atom[A], b = cell_atom[B];
    pc_cp[q] = cp_index.at({std::min(a, b), std::max(a, b)});
    pc_flag[q] = a > b ? 1 : 0;
    for (int d = 0; d < 3; ++d) pc_T[3 * q + d] = shift[3 * B + d] - shift[3 * A + d];
  }
  // stored pairs grouped by cell pair (the reverse sum reads a cell pair's
  // rho for all of its image pairs; consecutive ones share an XCD's L2)
  std::vector<int32_t> pc_order(p->n_pairs);
  for (int64_t q = 0; q < p->n_pairs; ++q) pc_order[q] = (int32_t)q;
  std::stable_sort(pc_order.begin(), pc_order.end(), [&](int32_t x, int32_t y) { return pc_cp[x] < pc_cp[y]; });
  if (!p->on_device) return Q4C_OK;
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  // device copies; earlier ones stay allocated until the plan is destroyed
  if ((rc = upload(p, ca, &p->d_cp_a)) != Q4C_OK) return rc;
  if ((rc = upload(p, cb, &p->d_cp_b)) != Q4C_OK) return rc;
  if ((rc = upload(p, coff, &p->d_cp_off)) != Q4C_OK) return rc;
  if ((rc = upload(p, ctoff, &p->d_ct_off)) != Q4C_OK) return rc;
  if ((rc = upload(p, ct_pair, &p->d_ct_pair)) != Q4C_OK) return rc;
  if ((rc = upload(p, ct_flag, &p->d_ct_flag)) != Q4C_OK) return rc;
  if ((rc = upload(p, ct_T, &p->d_ct_T)) != Q4C_OK) return rc;
  if ((rc = upload(p, pc_cp, &p->d_pc_cp)) != Q4C_OK) return rc;
  if ((rc = upload(p, pc_flag, &p->d_pc_flag)) != Q4C_OK) return rc;
  if ((rc = upload(p, pc_T, &p->d_pc_T)) != Q4C_OK) return rc;
  if ((rc = upload(p, pc_order, &p->d_pc_order)) != Q4C_OK) return rc;
  return Q4C_OK;
}

int q4c_plan_cell_pairs(const q4c_plan *p, int64_t *n_cell_pairs, int32_t *pair_atoms, int64_t *pair_off) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (p->n_cell_atoms == 0) return fail(Q4C_EINVAL, "no periodic cell set (q4c_plan_set_cells)");
  if (n_cell_pairs) *n_cell_pairs = (int64_t)p->cp_a.size();
  if (pair_atoms)
    for (size_t c = 0; c < p->cp_a.size(); ++c) {
      pair_atoms[2 * c] = p->cp_a[c];
      pair_atoms[2 * c + 1] = p->cp_b[c];
    }
  if (pair_off) std::copy(p->cp_off.begin(), p->cp_off.end(), pair_off);
  return Q4C_OK;
}

// Copies n_k k-points (and weights) into the plan's k buffer [3 n_k points,
// n_k weights], grows the phase table to a chunk of the larger of the
// contribution and pair counts, and waits for the copy (the host arrays may
// go away after the call).
static int stage_kpoints(const q4c_plan *p, int32_t n_k, const double *k_points, const double *k_weights,
                         void *stream) {
  int rc;
  if (p->kpts_cap < 4 * (int64_t)n_k) {
    void *ptr = nullptr;
    if ((rc = device_alloc(const_cast<q4c_plan *>(p), (size_t)(4 * n_k) * sizeof(double), &ptr)) != Q4C_OK)
      return rc;
    p->d_kpts = (double *)ptr;
    p->kpts_cap = 4 * (int64_t)n_k;
  }
  const int64_t ph_len = 2 * (int64_t)q4c::kBlochKChunk * std::max<int64_t>(p->n_contrib, p->n_pairs);
  if (p->bloch_ph_cap < ph_len) {
    void *ptr = nullptr;
    if ((rc = device_alloc(const_cast<q4c_plan *>(p), (size_t)ph_len * sizeof(double), &ptr)) != Q4C_OK) return rc;
    p->d_bloch_ph = (double *)ptr;
    p->bloch_ph_cap = ph_len;
  }
  if (n_k == 0) return Q4C_OK;
  hipError_t e = hipMemcpyAsync(p->d_kpts, k_points, (size_t)(3 * n_k) * sizeof(double), hipMemcpyHostToDevice,
                                (hipStream_t)stream);
  if (e != hipSuccess) return q4c::hip_fail(e, "hipMemcpyAsync k-points");
  if (k_weights) {
    e = hipMemcpyAsync(p->d_kpts + 3 * (int64_t)n_k, k_weights, (size_t)n_k * sizeof(double), hipMemcpyHostToDevice,
                       (hipStream_t)stream);
    if (e != hipSuccess) return q4c::hip_fail(e, "hipMemcpyAsync k-weights");
  }
  e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return q4c::hip_fail(e, "hipStreamSynchronize");
  return Q4C_OK;
}

int q4c_bloch_sum(const q4c_plan *p, int32_t n_parts, const double *store_dev, int32_t n_k, const double *k_points,
                  double *out_dev, void *stream) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  // 3 or 4 parts would cut the spin-orbit triple of a five-part store
  if (n_parts != 1 && n_parts != 2 && n_parts != 5) return fail(Q4C_EINVAL, "n_parts must be 1, 2 or 5");
  if (n_k < 0) return fail(Q4C_EINVAL, "negative n_k");
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  if (p->n_cell_atoms == 0) return fail(Q4C_EINVAL, "no periodic cell set (q4c_plan_set_cells)");
  if (n_k == 0 || p->cp_a.empty()) return Q4C_OK;
  if (!k_points || !store_dev || !out_dev) return fail(Q4C_EINVAL, "NULL argument");
  if (!finite_all(k_points, 3 * (int64_t)n_k)) return fail(Q4C_EINVAL, "non-finite k-point");
  if ((rc = stage_kpoints(p, n_k, k_points, nullptr, stream)) != Q4C_OK) return rc;
  return q4c::launch_bloch_sum(p, n_parts, store_dev, n_k, p->d_kpts, p->d_bloch_ph, out_dev, (hipStream_t)stream);
}

int q4c_bloch_sum_noalloc(const q4c_plan *p, int32_t n_parts, const double *store_dev, int32_t n_k,
                          const double *k_points_dev, double *out_dev, void *stream) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (n_parts != 1 && n_parts != 2 && n_parts != 5) return fail(Q4C_EINVAL, "n_parts must be 1, 2 or 5");
  if (n_k < 0) return fail(Q4C_EINVAL, "negative n_k");
  int rc = check_plan_dev(p);  // makes the plan's device current
  if (rc != Q4C_OK) return rc;
  if (p->n_cell_atoms == 0) return fail(Q4C_EINVAL, "no periodic cell set (q4c_plan_set_cells)");
  if (n_k == 0 || p->cp_a.empty()) return Q4C_OK;
  if (!k_points_dev || !store_dev || !out_dev) return fail(Q4C_EINVAL, "NULL argument");
  return q4c::launch_bloch_sum_noalloc(p, n_parts, store_dev, n_k, k_points_dev, out_dev, (hipStream_t)stream);
}

int q4c_bloch_density(const q4c_plan *p, int32_t n_parts, const double *rho_dev, int32_t n_k, const double *k_points,
                      const double *k_weights, double *coef_out_dev, void *stream) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (n_parts != 1 && n_parts != 2) return fail(Q4C_EINVAL, "n_parts must be 1 or 2 (Hermitian parts)");
  if (n_k < 0) return fail(Q4C_EINVAL, "negative n_k");
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  if (p->n_cell_atoms == 0) return fail(Q4C_EINVAL, "no periodic cell set (q4c_plan_set_cells)");
  if (p->store_len == 0) return Q4C_OK;
  if (!coef_out_dev || (n_k > 0 && (!rho_dev || !k_points || !k_weights))) return fail(Q4C_EINVAL, "NULL argument");
  if (n_k > 0 && !finite_all(k_points, 3 * (int64_t)n_k)) return fail(Q4C_EINVAL, "non-finite k-point");
  if (n_k > 0 && !finite_all(k_weights, (int64_t)n_k)) return fail(Q4C_EINVAL, "non-finite k-weight");
  if ((rc = stage_kpoints(p, n_k, k_points, k_weights, stream)) != Q4C_OK) return rc;
  return q4c::launch_bloch_density(p, n_parts, rho_dev, n_k, p->d_kpts, p->d_kpts + 3 * (int64_t)n_k, p->d_bloch_ph,
                                   coef_out_dev, (hipStream_t)stream);
}

int q4c_integrate_HS(const q4c_plan *p, const double *v_dev, uint32_t flags, double *hs_dev, void *stream) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (flags & ~(uint32_t)(Q4C_ACCUMULATE | Q4C_CHECK_FINITE)) return fail(Q4C_EINVAL, "unknown flag");
  if (p->n_points > 0 && !v_dev) return fail(Q4C_EINVAL, "NULL potential");
  if (p->store_len > 0 && !hs_dev) return fail(Q4C_EINVAL, "NULL H/S output");
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  if (p->n_shells > 0 && !p->d_ucoef) return fail(Q4C_EINVAL, "no ket potential set (q4c_plan_set_ket_potential)");
  if (flags & Q4C_CHECK_FINITE) {
    bool ok = true;
    rc = q4c::launch_check_finite(p, v_dev, (hipStream_t)stream, &ok);
    if (rc != Q4C_OK) return rc;
    if (!ok) return fail(Q4C_ENONFINITE, "potential contains NaN or Inf");
  }
  p->panel_pass = -1;  // the H/S panels replace the W-path panels
  const uint32_t f = flags & ~(uint32_t)Q4C_CHECK_FINITE;
  if (p->use_graphs && !p->profiling)
    return run_graph(p, 2, v_dev, hs_dev, nullptr, nullptr, f, 0, 0, (hipStream_t)stream,
                     [&](hipStream_t cs) { return q4c::launch_integrate_hs(p, v_dev, f, hs_dev, cs); });
  return q4c::launch_integrate_hs(p, v_dev, f, hs_dev, (hipStream_t)stream);
}

int density_on_grid(const q4c_plan *p, const double *coef_dev, uint32_t terms, int32_t precision, int32_t weight_mode,
                    double *out_dev, void *stream) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (terms == 0 || (terms & ~(uint32_t)Q4C_TERM_ALL)) return fail(Q4C_EINVAL, "bad term selection");
  if (precision != Q4C_PREC_F64 && precision != Q4C_PREC_F32)
    return fail(Q4C_EINVAL, "density_on_grid precision must be Q4C_PREC_F64 or Q4C_PREC_F32");
  if (weight_mode != 0 && weight_mode != 1) return fail(Q4C_EINVAL, "weight_mode must be 0 or 1");
  if (p->store_len > 0 && !coef_dev) return fail(Q4C_EINVAL, "NULL coefficients");
  if (p->n_points > 0 && !out_dev) return fail(Q4C_EINVAL, "NULL output");
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  // panels the previous call left resident are used, not tabulated again;
  // only the first pass this call runs (the last one) can find its own: any
  // pass it tabulates may overwrite another pass's region
  const int64_t resident = p->panel_pass == (int64_t)p->passes.size() - 1 ? p->panel_pass : -1;
  p->panel_pass = -1;
  if (p->use_graphs && !p->profiling)
    rc = run_graph(p, 1, coef_dev, out_dev, nullptr, nullptr, terms | ((int64_t)precision << 8), weight_mode, resident,
                   (hipStream_t)stream, [&](hipStream_t cs) {
                     return q4c::launch_density(p, coef_dev, terms, precision, weight_mode, out_dev, resident, cs);
                   });
  else
    rc = q4c::launch_density(p, coef_dev, terms, precision, weight_mode, out_dev, resident, (hipStream_t)stream);
  // the passes ran from the last one down: pass 0's panels are resident
  if (rc == Q4C_OK && !p->passes.empty()) p->panel_pass = 0;
  return rc;
}

int q4c_plan_set_graphs(q4c_plan *p, int enable) {
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  drop_graphs(p);
  p->use_graphs = enable != 0;
  return Q4C_OK;
}

int q4c_plan_set_launch(q4c_plan *p, int32_t kernel, int32_t order, int32_t persistent) {
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  if (kernel != Q4C_KERNEL_CONTRACT && kernel != Q4C_KERNEL_DENSITY && kernel != Q4C_KERNEL_HS)
    return fail(Q4C_EINVAL, "unknown kernel");
  if (order != 0 && order != 1) return fail(Q4C_EINVAL, "order must be 0 or 1");
  if (persistent < 0 || persistent > 65535) return fail(Q4C_EINVAL, "persistent workgroups must be in 0..65535");
  drop_graphs(p);
  q4c::LaunchCfg &c = kernel == Q4C_KERNEL_CONTRACT ? p->cfg_contract
                      : kernel == Q4C_KERNEL_DENSITY ? p->cfg_density
                                                     : p->cfg_hs;
  c.order = order;
  c.persistent = persistent;
  return Q4C_OK;
}

int q4c_plan_get_launch(const q4c_plan *p, int32_t kernel, int32_t *order, int32_t *persistent) {
  if (!p || !order || !persistent) return fail(Q4C_EINVAL, "NULL argument");
  if (kernel != Q4C_KERNEL_CONTRACT && kernel != Q4C_KERNEL_DENSITY && kernel != Q4C_KERNEL_HS)
    return fail(Q4C_EINVAL, "unknown kernel");
  const q4c::LaunchCfg &c = kernel == Q4C_KERNEL_CONTRACT ? p->cfg_contract
                            : kernel == Q4C_KERNEL_DENSITY ? p->cfg_density
                                                           : p->cfg_hs;
  *order = c.order;
  *persistent = c.persistent;
  return Q4C_OK;
}

int q4c_plan_autotune(q4c_plan *p, const double *v_dev, int32_t precision, double *store_dev, const double *coef_dev,
                      double *out_dev, int32_t reps, q4c_tune_entry *table, int32_t table_len, int32_t *n_entries,
                      void *stream) {
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  if (precision != Q4C_PREC_F64 && precision != Q4C_PREC_SPLIT_F32 && precision != Q4C_PREC_F32 &&
      precision != Q4C_PREC_BF16X3 && precision != Q4C_PREC_F64_VALU)
    return fail(Q4C_EINVAL, "unknown precision");
  if ((p->n_points > 0 && !v_dev) || (p->store_len > 0 && !store_dev))
    return fail(Q4C_EINVAL, "the potential and a store buffer are required");
  if ((coef_dev == nullptr) != (out_dev == nullptr)) return fail(Q4C_EINVAL, "coef_dev and out_dev go together");
  if (reps < 1) reps = 3;
  const hipStream_t s = (hipStream_t)stream;
  const bool prof = p->profiling, graphs = p->use_graphs;
  p->profiling = false;
  p->use_graphs = false;
  drop_graphs(p);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return q4c::hip_fail(hipGetLastError(), "hipEventCreate");
  int n_out = 0;
  auto time_call = [&](const std::function<int()> &call, double *ms) -> int {
    int r = call();  // warm-up
    if (r != Q4C_OK) return r;
    std::vector<double> t;
    for (int i = 0; i < reps; ++i) {
      hipError_t e = hipEventRecord(e0, s);
      if (e != hipSuccess) return q4c::hip_fail(e, "hipEventRecord");
      r = call();
      if (r != Q4C_OK) return r;
      e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float f = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
      if (e != hipSuccess) return q4c::hip_fail(e, "hipEvent timing");
      t.push_back(f);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return Q4C_OK;
  };
  for (int kernel = 0; kernel < 2 && rc == Q4C_OK; ++kernel) {
    if (kernel == Q4C_KERNEL_DENSITY && !coef_dev) break;
    // workgroups that fit on the chip at once: two per CU for every
    // contraction kernel and the adjoint
    const int occ = 2;
    const int cand_p[3] = {0, occ * p->n_cu, 2 * occ * p->n_cu};
    q4c::LaunchCfg best{};
    double best_ms = 1e300;
    q4c::LaunchCfg best0{};  // fastest in batch order
    double best0_ms = 1e300;
    for (int order = 0; order < 2 && rc == Q4C_OK; ++order)
      for (int ip = 0; ip < 3 && rc == Q4C_OK; ++ip) {
        q4c::LaunchCfg &c = kernel == Q4C_KERNEL_CONTRACT ? p->cfg_contract : p->cfg_density;
        c.order = order;
        c.persistent = cand_p[ip];
        double ms = 0.0;
        if (kernel == Q4C_KERNEL_CONTRACT)
          rc = time_call([&] {
            return q4c::launch_integrate(p, v_dev, precision, Q4C_PART_ALL, 0, store_dev, nullptr, nullptr, s);
          }, &ms);
        else
          rc = time_call([&] { return q4c::launch_density(p, coef_dev, Q4C_TERM_ALL, Q4C_PREC_F64, 1, out_dev, -1, s); },
                         &ms);
        if (rc != Q4C_OK) break;
        if (table && n_out < table_len) table[n_out] = q4c_tune_entry{kernel, order, cand_p[ip], ms};
        ++n_out;
        if (ms < best_ms) {
          best_ms = ms;
          best = c;
        }
        if (order == 0 && ms < best0_ms) {
          best0_ms = ms;
          best0 = c;
        }
      }
    // Batch order keeps a batch's tiles on one XCD's L2 and reads far less
    // HBM than the cost-sorted queue; it is kept unless the other order is
    // faster by more than the run-to-run spread of the timings (2%).
    if (best.order != 0 && best0_ms <= 1.02 * best_ms) best = best0;
    (kernel == Q4C_KERNEL_CONTRACT ? p->cfg_contract : p->cfg_density) = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->panel_pass = -1;
  p->profiling = prof;
  p->use_graphs = graphs;
  if (n_entries) *n_entries = n_out;
  return rc;
}

int q4c_coef_from_spinor(const q4c_plan *p, const double *spin_d_dev, double *coef_out_dev, void *stream) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (p->store_len > 0 && (!spin_d_dev || !coef_out_dev)) return fail(Q4C_EINVAL, "NULL buffer");
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  return q4c::launch_coef_from_spinor(p, spin_d_dev, coef_out_dev, (hipStream_t)stream);
}

int q4c_plan_sync(const q4c_plan *p, void *stream) {
  int rc = check_plan_dev(p);
  if (rc != Q4C_OK) return rc;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return q4c::hip_fail(e, "hipStreamSynchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return q4c::hip_fail(e, "asynchronous kernel error");
  return Q4C_OK;
}

int q4c_plan_profile(q4c_plan *p, int enable) {
  if (!p) return fail(Q4C_EINVAL, "NULL plan");
  if (!p->on_device) return fail(Q4C_ENODEV, "plan has no device data");
  p->profiling = enable != 0;
  return Q4C_OK;
}

int q4c_plan_timers(q4c_plan *p, double *ms, int64_t *launches) {
  if (!p || !ms || !launches) return fail(Q4C_EINVAL, "NULL argument");
  for (int k = 0; k < Q4C_NTIMERS; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  if (!p->on_device) return Q4C_OK;
  (void)hipSetDevice(p->device);
  int rc = Q4C_OK;
  for (auto &x : p->ev_live) {
    float t = 0.0f;
    hipError_t e = hipEventSynchronize(x.second.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, x.second.first, x.second.second);
    if (e != hipSuccess && rc == Q4C_OK) rc = q4c::hip_fail(e, "hipEventElapsedTime");
    if (x.first >= 0 && x.first < Q4C_NTIMERS) {
      ms[x.first] += t;
      launches[x.first] += 1;
    }
    p->ev_pool.push_back(x.second.first);
    p->ev_pool.push_back(x.second.second);
  }
  p->ev_live.clear();
  return rc;
}

const char *q4c_status_string(int s) {
  switch (s) {
    case Q4C_OK: return "ok";
    case Q4C_EINVAL: return "invalid argument";
    case Q4C_ENOMEM: return "out of memory";
    case Q4C_EHIP: return "HIP runtime error";
    case Q4C_ENOTIMPL: return "not implemented";
    case Q4C_EUNSUPPORTED: return "unsupported input";
    case Q4C_ESIZE: return "buffer too small";
    case Q4C_ENONFINITE: return "non-finite input";
    case Q4C_ENODEV: return "no device data";
    default: return "unknown status";
  }
}

const char *q4c_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
