/*
 * q4c.h -- C ABI of libq4c, MI355X (gfx950) real-space grid integration of
 * quasi-four-component (Q4C) Hamiltonian matrix elements over numeric
 * atom-centred orbitals (NAOs).
 *
 * Problem statement (paper Sec. III A): overlapping atom-centred integration
 * grids with partition weights w(r), scalar NAOs
 *     phi_i(r) = Rt_i(s) S_lm(r - R_A),  s = |r - R_A|            (Eq. 12a)
 * (S_lm = s^l Y_lm, real Y_lm of App. B), the potential v on the grid, and the
 * matrix elements integrated as weighted grid sums over batches of points
 *     F_ij = sum_B sum_{r in B} w(r) phi_i(r) F phi_j(r)           (Eq. 29, 31)
 * with F = v for the large-large block V and F = (sigma.p) v (sigma.p)/4c^2
 * for the small-small block W (Eq. 16a with the kinetic balance of Eq. 8b at
 * V_A -> 0).  For real phi the Pauli identity splits W into a scalar part and
 * three spin-orbit parts:
 *     V_ij      = sum_g w_g v_g phi_i phi_j
 *     Ws_ij     = c' sum_g w_g v_g grad phi_i . grad phi_j
 *     Wso_m,ij  = c' sum_g w_g v_g (grad phi_i x grad phi_j)_m,   c' = 1/(4c^2)
 * and the 2x2-spinor blocks are V (x) I2 and Ws (x) I2 + i sum_m Wso_m (x) sigma_m.
 *
 * Conventions
 *  - Units: bohr, hartree.  All floating point arguments are IEEE binary64.
 *  - Functions are numbered atom-major, then shell order, then m = -l..l.
 *  - Sparse atom-pair store: the pairs (A, B), A <= B, with
 *    |R_A - R_B| < rcut_A + rcut_B (rcut_A = largest shell cutoff of A), in
 *    (A, B) order.  Pair p owns nA x nB row-major doubles at pair_off[p]
 *    (rows = functions of A).  Diagonal pairs (A, A) hold the full block.
 *    A real part is store_len doubles; a store of all five parts is
 *    5 * store_len doubles, part-major: V, Ws, Wso_x, Wso_y, Wso_z.
 *  - Spinor blocks: pair p owns a (2 nA) x (2 nB) row-major complex128 block
 *    at complex offset 4 * pair_off[p]; rows (spin, function of A) spin-major,
 *    i.e. [[uu, ud], [du, dd]] sub-blocks.
 *  - Host pointers are read during the call only; nothing is retained.
 *  - Device pointers ("_dev") must be device memory of the plan's device.
 *  - Calls taking a stream are asynchronous on that stream (NULL = default
 *    stream).  Calls on one plan use the plan's scratch buffers and must not
 *    overlap in time (serialise them on one stream).
 *  - Every call returns Q4C_OK (0) or a negative status; no C++ exception or
 *    abort crosses the ABI.  q4c_last_error() gives a message for the last
 *    failure on the calling thread.
 */
#ifndef Q4C_H
#define Q4C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  Q4C_OK = 0,
  Q4C_EINVAL = -1,       /* invalid argument (NULL, negative size, bad layout) */
  Q4C_ENOMEM = -2,       /* host or device allocation failed */
  Q4C_EHIP = -3,         /* HIP runtime error (message via q4c_last_error) */
  Q4C_ENOTIMPL = -4,     /* option not implemented */
  Q4C_EUNSUPPORTED = -5, /* unsupported input, e.g. l > 4 */
  Q4C_ESIZE = -6,        /* output buffer too small */
  Q4C_ENONFINITE = -7,   /* non-finite input detected (Q4C_CHECK_FINITE) */
  Q4C_ENODEV = -8        /* plan has no device data (host-only plan or no GPU) */
};

/* precision of the per-batch contractions (paper Sec. III A, Eq. 29/31):
 * V always runs on FP64 MFMA (its elements reach ~1e2 Ha, beyond what FP32
 * accumulation can hold to 1e-8 Ha).  The W parts (9 of the 10 P n^2 flops
 * of a batch):
 *   Q4C_PREC_F64        FP64 MFMA, FP64 accumulation.
 *   Q4C_PREC_F32        FP32 MFMA on FP32 operands (sqrt|w v| times the
 *                       gradient, formed in FP64 and rounded once; the row
 *                       operand carries the sign of w v);
 *                       every element's FP32 partial sum covers 16 points (at
 *                       most 48 products) and is then added to an FP64 sum.
 *                       Bound: |error| <= gamma_52 A_ij + (FP32 underflow:
 *                       below 1e-25 Ha) + FP64 rounding, with
 *                       gamma_k = k u / (1 - k u), u = 2^-24 (gamma_52 ~ 3.1e-6)
 *                       and A_ij the sum over all points of the magnitudes of
 *                       the element's terms (c' sum_g |w_g v_g| sum |d phi_i|
 *                       |d phi_j| over the products entering it).
 *   Q4C_PREC_SPLIT_F32  FP32 MFMA with each operand (the gradient for rows,
 *                       w v times it, formed in FP64, for columns) split into
 *                       hi = fl32(x) and lo = fl32(x - hi), FP32 sums over
 *                       16 points as for F32, and every product taken as
 *                       hi hi + hi lo + lo hi (three FP32 MFMAs): operand
 *                       rounding drops to about 2^-48, and a 16-point partial
 *                       sum has up to 144 products: gamma_150 A_ij.
 *   Q4C_PREC_BF16X3     BF16 MFMA (16 times the FP32 MFMA rate) with each
 *                       operand split into three BF16 parts x1 + x2 + x3
 *                       (|x - x1 - x2 - x3| <= 2^-23 |x|) and every product
 *                       taken as its six terms of order 2^-16 and above
 *                       (a1 b1 + a2 b1 + a1 b2 + a1 b3 + a2 b2 + a3 b1, within
 *                       3 2^-23 |a b|); both operands are sqrt|w v| times
 *                       the gradient, formed in FP64 before the split, and
 *                       the row operand takes the sign of w v.  FP32
 *                       accumulation over one 16-point chunk (9 MFMAs of
 *                       K = 32 per element at most), then added to an FP64
 *                       sum.  The BF16 MFMA sums each group of 8 products
 *                       aligned to the largest of them, dropping what falls
 *                       below its last place (up to 7 units of the last place
 *                       per group), and adds each group to the accumulator
 *                       (at most 1 unit); with 2^-23 per unit,
 *                       |error| <= 48 2^-23 A_ij (about 5.7e-6 A_ij), plus
 *                       FP32 underflow (below 1e-25 Ha) and FP64 rounding.
 *                       V runs in the same kernel on FP64 MFMA, in the same
 *                       order as Q4C_PREC_F64 (bitwise the same V).
 *   Q4C_PREC_F64_VALU   all five parts in FP64 on the vector ALU, no matrix
 *                       cores: the plain FP64 baseline the reduced
 *                       precisions are compared with (FP64 bar, summation
 *                       point by point; not bitwise Q4C_PREC_F64).
 * Batch partial sums are added to the store in FP64 in a fixed order. */
enum {
  Q4C_PREC_F64 = 0,
  Q4C_PREC_SPLIT_F32 = 1,
  Q4C_PREC_F32 = 2,
  Q4C_PREC_BF16X3 = 3,
  Q4C_PREC_F64_VALU = 4
};

/* parts of q4c_integrate_H (bit set): V, the scalar W part Ws, the three
 * spin-orbit parts Wso_x,y,z.  Parts not selected are neither computed nor
 * written (their store elements keep their values). */
enum { Q4C_PART_V = 1u, Q4C_PART_WS = 2u, Q4C_PART_WSO = 4u, Q4C_PART_ALL = 7u };

/* flags of q4c_integrate_H */
enum {
  Q4C_ACCUMULATE = 1u,     /* add into the store instead of overwriting it */
  Q4C_ASSEMBLE_W = 2u,     /* also write the W spinor blocks */
  Q4C_ASSEMBLE_V = 4u,     /* also write the V spinor blocks (V (x) I2) */
  Q4C_CHECK_FINITE = 8u    /* reject a potential with NaN/Inf (synchronises) */
};

/* plan option flags */
enum {
  Q4C_PLAN_HOST_ONLY = 1   /* build host structures only (no device upload) */
};

typedef struct q4c_plan q4c_plan;

/* Basis set: per-atom shells with piecewise-cubic radial tables.
 * Shell s: angular momentum shell_l[s] in 0..4, cutoff shell_rcut[s] > 0,
 * nint = shell_nint[s] >= 1 intervals on knots r_j = rcut (j / nint)^2,
 * coefficients coef[shell_coef_off[s] + 4 j + k], k = 0..3, such that for
 * r_j <= s < r_{j+1} and t = (s - r_j) / (r_{j+1} - r_j):
 *     Rt(s) = c0 + c1 t + c2 t^2 + c3 t^3,   Rt(s) = 0 for s >= rcut.
 * Rt is the radial function divided by s^l (paper Eq. 12a: P(r)/r = Rt s^l),
 * so phi = Rt(s) s^l Y_lm.  Shells may share coefficient ranges. */
typedef struct {
  int32_t n_atoms;
  const double *R;               /* [3 n_atoms] positions, xyz interleaved */
  const int32_t *atom_shell_off; /* [n_atoms + 1], non-decreasing, from 0 */
  int32_t n_shells;
  const int32_t *shell_l;        /* [n_shells] */
  const double *shell_rcut;      /* [n_shells] */
  const int32_t *shell_nint;     /* [n_shells] */
  const int64_t *shell_coef_off; /* [n_shells] offsets into coef (doubles) */
  int64_t n_coef;                /* length of coef */
  const double *coef;
} q4c_basis;

/* Integration grid in the caller's point order ("user order"). */
typedef struct {
  int64_t n_points;
  const double *x, *y, *z;  /* [n_points] bohr */
  const double *w;          /* [n_points] quadrature x partition weight, finite */
} q4c_grid;

typedef struct {
  double c_light;           /* speed of light in a.u.; <= 0 selects 137.035999084 */
  int32_t p_max;            /* max points per batch; <= 0 selects 300 */
  int32_t flags;            /* Q4C_PLAN_* */
  int64_t staging_bytes;    /* per-plan scratch budget (staged batch results and
                               operand panels); <= 0 selects 32 GiB.  Batches are
                               processed in passes that fit the budget. */
} q4c_opts;

typedef struct {
  int32_t n_atoms, n_fn;
  int64_t n_points;        /* input points */
  int64_t n_active;        /* points inside at least one basis support */
  int64_t n_batches;
  int64_t n_pairs;
  int64_t store_len;       /* doubles per real part */
  int64_t fn_entries;      /* sum over batches of relevant functions */
  int64_t max_batch_points, max_batch_fn;
  int64_t n_work;          /* contraction work items (batch, tile, tile) */
  int64_t n_passes;        /* staging passes per call */
  int64_t device_bytes;    /* device memory owned by the plan */
  double flops_alg;        /* sum_B 10 P_B n_B^2, the algorithmic flop count of one H build */
  int32_t n_systems;       /* independent systems (1 unless q4c_plan_create_batched) */
  int64_t scratch_bytes;   /* device scratch of the plan (largest pass: staging, partials, panels) */
  double flops_alg_hs;     /* sum_B 3 P_B n_B^2: the three contractions of one q4c_integrate_HS */
  int64_t staging_bytes;   /* per-batch partial blocks of one q4c_integrate_H, all passes: written by the
                              contraction, read once by the batch-to-global sum */
  int64_t tab_elems;       /* sum_B P_B n_B: (point, relevant function) pairs of all batches */
} q4c_info;

/* Build a plan: batching (recursive median bisection of the active points to
 * at most p_max points), per-batch relevant functions, the pair store layout,
 * scatter maps and device buffers.  Paper Sec. III A: batches B_v (Eq. 31)
 * and the reduced index set nnz(B_v).  Inputs are copied.  Returns
 * Q4C_EUNSUPPORTED for l > 4 and Q4C_EINVAL for malformed descriptors. */
int q4c_plan_create(const q4c_basis *basis, const q4c_grid *grid, const q4c_opts *opts, q4c_plan **out);

/* One plan over n_systems independent systems (e.g. many molecules): every
 * call then runs all systems' batches in the same launches.  The union is
 * system-major: atoms, functions, grid points (user order = the systems'
 * points concatenated), pairs and store blocks of system 0, then system 1, ...
 * Batches, relevant functions and pairs never mix systems, so each system's
 * batches, pairs and results are exactly those of q4c_plan_create on that
 * system alone (same batch contents, same summation order: bitwise equal).
 * Systems passing the same coef pointer and n_coef share radial tables.
 * Paper Sec. III A (Eq. 31): batches are independent work units. */
int q4c_plan_create_batched(int32_t n_systems, const q4c_basis *bases, const q4c_grid *grids, const q4c_opts *opts,
                            q4c_plan **out);

/* Offsets of every system in the union ([n_systems + 1] each, NULL to skip):
 * atoms, user-order grid points, batches, pairs and store elements (doubles
 * per real part). */
int q4c_plan_systems(const q4c_plan *plan, int64_t *atom_off, int64_t *point_off, int64_t *batch_off,
                     int64_t *pair_off, int64_t *store_off);

/* Free a plan and its device memory; NULL is a no-op.  Synchronises the device. */
void q4c_plan_destroy(q4c_plan *plan);

int q4c_plan_info(const q4c_plan *plan, q4c_info *info);

/* Pair list: pair_atoms[2p], pair_atoms[2p+1] = (A, B); pair_off[n_pairs + 1]
 * offsets (doubles) into one real part.  Host buffers of the sizes in q4c_info. */
int q4c_plan_pairs(const q4c_plan *plan, int32_t *pair_atoms, int64_t *pair_off);

/* Batches: batch b holds points point_index[pt_off[b] .. pt_off[b+1]) (user
 * indices) and functions fn_index[fn_off[b] .. fn_off[b+1]) (global indices,
 * ascending).  Sizes: n_batches + 1, n_active, n_batches + 1, fn_entries.
 * Any pointer may be NULL to skip it. */
int q4c_plan_batches(const q4c_plan *plan, int64_t *pt_off, int64_t *point_index, int64_t *fn_off,
                     int32_t *fn_index);

/* Sparse pair store layout of a plan (the outputs the caller allocates). */
typedef struct {
  int64_t n_pairs;
  int64_t store_len;     /* doubles per real part (sum over pairs of nA nB) */
  int64_t part_bytes;    /* one real part: 8 store_len */
  int64_t store_bytes;   /* the five real parts of q4c_integrate_H: 40 store_len */
  int64_t hs_bytes;      /* the two parts (H, S) of q4c_integrate_HS: 16 store_len */
  int64_t spinor_bytes;  /* one set of complex128 spinor blocks (2 nA x 2 nB per pair): 64 store_len */
} q4c_layout;

/* q4c_store_layout: sizes of the store, and (each optional, NULL to skip)
 * the pair list (pair_atoms[2p], pair_atoms[2p+1] = (A, B), A <= B, in (A, B)
 * order), the block offsets pair_off[n_pairs + 1] (doubles into one real
 * part; spinor blocks start at complex offset 4 pair_off[p]) and the block
 * shapes pair_nfn[2p], pair_nfn[2p+1] = (nA, nB).  Host buffers.  Paper
 * Sec. III A: the locally indexed dense blocks of the sparse matrices. */
int q4c_store_layout(const q4c_plan *plan, q4c_layout *layout, int32_t *pair_atoms, int64_t *pair_off,
                     int32_t *pair_nfn);

/* Element types of nao_tabulate. */
enum {
  Q4C_DTYPE_F64 = 0,      /* binary64 values */
  Q4C_DTYPE_F32_HILO = 1  /* each value x as two binary32: hi = fl32(x), lo = fl32(x - hi)
                             (x = hi + lo to about 2^-48 relative), the split operands of
                             FP32 MFMA products */
};

/* Number of values nao_tabulate writes for batches [b0, b1) (8 bytes each
 * for both element types). */
int q4c_tabulate_size(const q4c_plan *plan, int64_t b0, int64_t b1, int32_t deriv, int64_t *n_values);

/* nao_tabulate: values (deriv = 0) or values and gradients (deriv = 1) of the
 * relevant functions of batches [b0, b1) at their points (Eq. 12a, App. B),
 * computed as the integration calls compute them (one workgroup per batch
 * and 64-function tile, the tile's shell data staged in LDS).
 * Output (device): batch after batch, ncomp = 1 or 4 components (phi, d/dx,
 * d/dy, d/dz), points in the batch order of q4c_plan_batches, functions in
 * the order of fn_index:
 *   Q4C_DTYPE_F64:      double [ncomp][P_b][n_b]
 *   Q4C_DTYPE_F32_HILO: float  [ncomp][2][P_b][n_b] (the hi plane, then the lo plane)
 * Both use 8 q4c_tabulate_size() bytes; out_bytes below that gives
 * Q4C_ESIZE, an unknown dtype Q4C_EINVAL. */
int nao_tabulate(const q4c_plan *plan, int64_t b0, int64_t b1, int32_t deriv, int32_t dtype, void *out_dev,
                 int64_t out_bytes, void *stream);

/* q4c_integrate_H: the selected real parts of the atom-pair store from the
 * potential v (device, [n_points], user order, hartree) (Eq. 29 summed over
 * batches, Eq. 31; W from Eq. 16a with the kinetic balance of Eq. 8b):
 * store_dev[0..5 store_len) = V, Ws, Wso_x, Wso_y, Wso_z with c' applied,
 * parts not in `parts` untouched.  precision: Q4C_PREC_* (see there; V is
 * FP64 in every precision).  Batch partial sums are added to the store in
 * FP64 in a fixed order, so repeated calls are bitwise identical.  With
 * Q4C_ASSEMBLE_W / _V the spinor blocks are written to spin_w_dev /
 * spin_v_dev (complex128, 4 store_len elements each); ASSEMBLE_W needs Ws and
 * Wso selected, ASSEMBLE_V needs V (else Q4C_EINVAL, as for parts = 0). */
int q4c_integrate_H(const q4c_plan *plan, const double *v_dev, int32_t precision, uint32_t parts, uint32_t flags,
                    double *store_dev, double *spin_w_dev, double *spin_v_dev, void *stream);

/* density_on_grid: for coefficients C on the stored elements (device,
 * 5 store_len doubles, same layout as the store, c' NOT included),
 *   n_g = sum_{stored ij} [ C^V_ij phi_i phi_j + c' C^Ws_ij grad phi_i . grad phi_j
 *                            + c' sum_m C^m_ij (grad phi_i x grad phi_j)_m ]
 * (paper Eq. 39 on the scalar basis).  out_dev[g] (device, [n_points], user
 * order) = n_g (weight_mode 0) or w_g n_g (weight_mode 1).  With weight_mode 1
 * and C = dL/d(store), out is dL/dv: the exact adjoint of q4c_integrate_H.
 * terms selects Q4C_TERM_* (bit set).  precision: Q4C_PREC_F64 (FP64 MFMA),
 * or Q4C_PREC_F32: the SS and SO terms (nine of the ten products) on FP32
 * MFMA with coefficients and row values rounded to FP32, each 16-point
 * chunk's FP32 sums over 32 rows (at most 96 products) drained into FP64:
 * per point |error| <= gamma_98 (u = 2^-24, gamma_k = k u / (1 - k u),
 * about 5.8e-6) times the magnitudes of its SS and SO terms (c' sum |C|
 * |d phi_i| |d phi_j|, times |w_g| in weight mode 1), plus FP64 rounding and
 * FP32 underflow below 2^-126; the LL term stays FP64.  Q4C_PREC_SPLIT_F32 is
 * not offered here (Q4C_EINVAL). */
enum { Q4C_TERM_LL = 1u, Q4C_TERM_SS = 2u, Q4C_TERM_SO = 4u, Q4C_TERM_ALL = 7u };
int density_on_grid(const q4c_plan *plan, const double *coef_dev, uint32_t terms, int32_t precision,
                    int32_t weight_mode, double *out_dev, void *stream);

/* The paper's own Q4C Hamiltonian integrand (Sec. II, Eq. 19), evaluated on
 * the scalar functions of one component as in Eq. 29.  A plan built from the
 * large-component basis (P(r)/r Y_lm, Eq. 12a) or from the small-component
 * basis (Q(r)/r Y_{l~m~}, l~ = l +- 1, Eq. 12b; the i of Eq. 12b cancels
 * between bra and ket) gives that component's H and S.
 *
 * q4c_plan_set_ket_potential: the ket potential u_s(r) = eps_s - V_s(r) of
 * every shell s (eps_s, V_s: the orbital energy and defining radial
 * potential of the spinor function the shell belongs to), as a piecewise
 * cubic on the shell's own radial knots, in the radial-table format:
 * u_coef[shell_u_off[s] + 4 j + k] (host arrays, n_shells offsets, n_u
 * doubles; copied).  Replaces an earlier table.  Q4C_EINVAL for a table
 * outside u_coef, an offset not a multiple of 4, or non-finite values. */
int q4c_plan_set_ket_potential(q4c_plan *plan, const int64_t *shell_u_off, int64_t n_u, const double *u_coef);

/* q4c_integrate_HS: for the potential v (device, [n_points], user order,
 * hartree; V_eff of Eq. 19), the symmetrised ket-dependent Hamiltonian and
 * the overlap of the plan's component on the atom-pair store layout:
 *   H_ij = sum_g w_g phi_i phi_j (v_g + (u_i + u_j) / 2)
 *        = (F_ij + F_ji) / 2,  F_ij = sum_g w_g phi_i (eps_j - V_j + v_g) phi_j
 *   S_ij = sum_g w_g phi_i phi_j
 * hs_dev (device): 2 store_len doubles, H then S, each part laid out like one
 * part of the q4c_integrate_H store.  FP64 MFMA; batch sums added in a fixed
 * order (bitwise repeatable).  flags: Q4C_ACCUMULATE adds to hs_dev,
 * Q4C_CHECK_FINITE rejects a non-finite v (Q4C_ENONFINITE).  Q4C_EINVAL if no
 * ket potential is set.  With graphs on (q4c_plan_set_graphs) each distinct
 * (v_dev, hs_dev, flags) is captured once and replayed. */
int q4c_integrate_HS(const q4c_plan *plan, const double *v_dev, uint32_t flags, double *hs_dev, void *stream);

/* q4c_spinor_transform: the scalar -> spinor transformation of H and S
 * (paper Sec. III A, Eq. 33, with the matrices of Eq. 14 built from the
 * Clebsch-Gordan coefficients of Eq. 10 / App. A and the complex harmonics
 * of Eq. 13), summed over the two components and the two spins:
 *   H+_AB = sum_c sum_s G^c_A[s]^H H^c_AB G^c_B[s],  S+ likewise.
 * plan_large: plan over the large-component basis; plan_small: over its
 * small-component partners on the same atoms and grid, listed per atom as
 * two shells l + 1 and l - 1 (one for l = 0) right after one another for
 * every large shell of l, in the large shells' order.  hs_large_dev,
 * hs_small_dev: the q4c_integrate_HS outputs of the two plans (device).
 * Spinor functions per atom: large shells in order; for each,
 * kappa = -(l+1) (j = l + 1/2), then kappa = l (j = l - 1/2, l >= 1); m_j
 * ascending; the small component of (kappa, m_j) lies on the shell of
 * l~ = 2j - l.  Complex harmonics are the Condon-Shortley ones (in terms of
 * the App. B real harmonics, which carry (-1)^m already, Eq. 13 without its
 * own (-1)^m); the i of Eq. 12b cancels.
 * h_dev, s_dev (device, complex128 as interleaved re, im): 4 store_len of
 * the large plan each; pair block (2 n_A) x (2 n_B) row-major at complex
 * offset 4 pair_off[p] (large plan's pairs).  Q4C_EINVAL if the small plan
 * does not pair with the large one (atoms, atom pairs, shells).  The first
 * call with a given small plan builds and uploads its tables on the large
 * plan. */
int q4c_spinor_transform(const q4c_plan *plan_large, const q4c_plan *plan_small, const double *hs_large_dev,
                         const double *hs_small_dev, double *h_dev, double *s_dev, void *stream);

/* q4c_spinor_density_to_scalar: the reverse of q4c_spinor_transform for a
 * density (the paper's D'_ij = sum_mu,nu D_mu,nu G*_i,mu G_j,nu, summed over
 * spins, for each component; Sec. III A, density update): from a spinor
 * density matrix D on the pair blocks (device complex128, the layout of the
 * q4c_spinor_transform outputs; D_BA = D_AB^H implied), the scalar density
 * matrices of the large and small components on their plans' pair layouts,
 *   C^c_AB = f Re sum_s conj(G^c_A[s]) D_AB G^c_B[s]^T,  f = 2 if A != B,
 * so that summing every stored element once gives the full density.
 * cl_dev: store_len (large plan) doubles; cs_dev: store_len (small plan).
 * Same plan pairing rules and tables as q4c_spinor_transform. */
int q4c_spinor_density_to_scalar(const q4c_plan *plan_large, const q4c_plan *plan_small, const double *d_dev,
                                 double *cl_dev, double *cs_dev, void *stream);

/* density_gradient_on_grid: the density and its gradient, as a GGA
 * functional needs them, from one coefficient part C (device, store_len
 * doubles, e.g. a component's scalar density matrix from
 * q4c_spinor_density_to_scalar; each stored element counted once):
 *   n_g = sum_ij C_ij phi_i phi_j,  d n_g / d x_a = sum_ij C_ij (d_a phi_i phi_j + phi_i d_a phi_j)
 * out_dev (device): [4][n_points] in user order: n, dn/dx, dn/dy, dn/dz
 * (zero outside every support).  FP64 MFMA; fixed-order sums (bitwise
 * repeatable).  Uses the launch shape of density_on_grid; the first call
 * allocates the plan's gradient partials (4x the adjoint partials of the
 * largest pass). */
int density_gradient_on_grid(const q4c_plan *plan, const double *coef_dev, double *out_dev, void *stream);

/* Periodic systems (paper Sec. II C).  A plan for a solid holds the atoms of
 * a reference cell and those of their periodic images whose functions reach
 * the cell, with a grid that covers the cell once (its own atoms' grids,
 * partitioned over all atoms); its integrals are then the unit-cell
 * integrals O^uc of Eq. 26 between every pair of those functions.
 *
 * q4c_plan_set_cells: for every atom a of the plan, the reference-cell atom
 * it copies (cell_atom[a] in 0..n_cell_atoms-1) and its lattice translation
 * T(a) (shift[3a..3a+2], bohr; zero for the cell's own atoms).  Host arrays,
 * copied.  Q4C_EINVAL if an index is out of range, a shift is not finite, a
 * cell atom has no copy, or an image's basis differs from its cell atom's;
 * Q4C_EUNSUPPORTED on a batched plan. */
int q4c_plan_set_cells(q4c_plan *plan, int32_t n_cell_atoms, const int32_t *cell_atom, const double *shift);

/* The output layout of q4c_bloch_sum: the cell pairs (a, b), a <= b, that at
 * least one stored pair of their images reaches, in ascending (a, b) order,
 * and the offsets of their n_a x n_b blocks (n_cell_pairs + 1 entries).
 * Any pointer may be NULL. */
int q4c_plan_cell_pairs(const q4c_plan *plan, int64_t *n_cell_pairs, int32_t *pair_atoms, int64_t *pair_off);

/* q4c_bloch_sum: the Bloch sums (Eq. 27 with the restricted sum of Eq. 28)
 *   O_ab(k) = sum over pairs (a', b') of images of a and b of
 *             exp(i k.(T(b') - T(a'))) O^uc_a'b'
 * of the first n_parts parts of a store of this plan (device; n_parts 1, 2
 * or 5: a q4c_integrate_H store, whose parts 2..4 are antisymmetric, or a
 * q4c_integrate_HS output, n_parts <= 2; Q4C_EINVAL otherwise), at n_k
 * k-points (host, 3 n_k, bohr^-1).  out_dev (device, complex128 as re, im):
 * [n_k][n_parts][cell store length] with the blocks at the cell-pair
 * offsets, row-major; O_ba(k) = O_ab(k)^H (symmetric parts) is implied.
 * Q4C_EINVAL without q4c_plan_set_cells.  Copies the k-points and waits for
 * that copy.  The k-points and their phases exp(i k.T) (64 k-points at a
 * time, 16 bytes per contribution and k-point) live in plan-owned device
 * buffers, allocated on first use and grown on demand: calls on one plan must
 * not overlap. */
int q4c_bloch_sum(const q4c_plan *plan, int32_t n_parts, const double *store_dev, int32_t n_k,
                  const double *k_points, double *out_dev, void *stream);

/* q4c_bloch_sum_noalloc: q4c_bloch_sum for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): no allocation, no host copy, no synchronisation.
 * The k-points come as a device array (k_points_dev: 3 n_k doubles, bohr^-1;
 * not checked for finiteness), and the phase table of each chunk of
 * k-points lives in a fixed device array of the library
 * (Q4C_NOALLOC_SCRATCH_BYTES = 4 MiB on each device it runs on, held until
 * the process ends): the k-points are processed in chunks whose phases
 * (16 bytes per contribution and k-point) fit, so a plan whose one k-point
 * needs more gives Q4C_ESIZE.  Every call on a GPU shares that GPU's array
 * (each chunk's phases are written before they are read, nothing needs to
 * start at zero): calls that overlap in time on one GPU race, so serialise
 * them (one stream).  Other arguments, layout and results as
 * q4c_bloch_sum (bitwise equal). */
#define Q4C_NOALLOC_SCRATCH_BYTES (4u << 20)
int q4c_bloch_sum_noalloc(const q4c_plan *plan, int32_t n_parts, const double *store_dev, int32_t n_k,
                          const double *k_points_dev, double *out_dev, void *stream);

/* q4c_bloch_density: the reverse of q4c_bloch_sum, the periodic density
 * matrix of Sec. II C.  From k-space density matrices rho(k) of the cell's
 * functions (Hermitian, e.g. sum over states of f_l C*_al(k) C_bl(k)), the
 * real-space density matrix of every stored image pair (A', B'),
 *   D_A'B' = sum_k w_k exp(i k.(T(B') - T(A'))) rho_ab(k),
 * a, b the cell atoms of A', B', rho_ab = rho_ba^H when a > b, returned as the
 * coefficients the density calls take: coef = f Re D, f = 2 for A' != B'
 * (the stored block stands for both orders) and 1 for A' = B'.  Then
 * density_gradient_on_grid (n_parts 1) or density_on_grid give the density of
 * the extended system on the cell's grid.
 * rho_dev: device complex128 (re, im) [n_k][n_parts][cell store length] in the
 * layout of q4c_bloch_sum's output (blocks of the cell pairs a <= b only);
 * n_parts 1 or 2 (Hermitian parts, e.g. one scalar density matrix per
 * component), else Q4C_EINVAL.  k_points (host, 3 n_k, bohr^-1), k_weights
 * (host, n_k).  coef_out_dev (device, n_parts store_len doubles) is
 * overwritten; n_k = 0 gives zeros.  Shares the k and phase buffers of
 * q4c_bloch_sum (calls on one plan must not overlap) and waits for the
 * k-point copy. */
int q4c_bloch_density(const q4c_plan *plan, int32_t n_parts, const double *rho_dev, int32_t n_k,
                      const double *k_points, const double *k_weights, double *coef_out_dev, void *stream);

/* Coefficients on the stored elements from a Hermitian spinor density matrix
 * D given as spinor blocks (device complex128, 4 store_len, spinor layout)
 * such that density_on_grid yields Re Tr(D H) derivatives (Eq. 21/39):
 * C^V = C^Ws = f Re tr2 D_ji, C^m = -f Im tr2(D_ji sigma_m), f = 2 on
 * off-diagonal pairs (each stored block stands for its mirror), 1 on diagonal
 * pairs.  coef_out_dev: 5 store_len doubles. */
int q4c_coef_from_spinor(const q4c_plan *plan, const double *spin_d_dev, double *coef_out_dev, void *stream);

/* Per-kernel timing.  While profiling is enabled on a plan, every kernel the
 * plan launches is bracketed by HIP events on the launch stream.
 * q4c_plan_timers waits for those events, returns per-kernel-kind totals
 * (milliseconds, launch counts; arrays of Q4C_NTIMERS) since the last query,
 * and resets them.  Meant for measurement, not for code under graph capture. */
enum {
  Q4C_TIMER_TABULATE = 0,
  Q4C_TIMER_CONTRACT = 1,
  Q4C_TIMER_REDUCE = 2,
  Q4C_TIMER_SPINOR = 3,
  Q4C_TIMER_BLOCH = 4,       /* k_bloch_sum of q4c_bloch_sum (its phase kernel counts as other) */
  Q4C_TIMER_DENSITY_TILES = 5,
  Q4C_TIMER_DENSITY_POINTS = 6,
  Q4C_TIMER_OTHER = 7,
  Q4C_NTIMERS = 8
};
int q4c_plan_profile(q4c_plan *plan, int enable);

int q4c_plan_timers(q4c_plan *plan, double *ms, int64_t *launches);

/* Launch shape of the contraction kernels (k_contract of q4c_integrate_H,
 * k_density_tiles of density_on_grid, k_contract_hs of q4c_integrate_HS), per
 * plan (the autotuner covers the first two):
 *   order      0: work items in batch order, consecutive items on one XCD;
 *              1: largest items first (estimated cost), longest-first scheduling;
 *   persistent 0: one workgroup per work item;
 *              k > 0: k workgroups loop over the items, taking them from
 *              ticket queues (one per XCD with stealing for order 0, one global
 *              queue for order 1).
 * Results do not depend on the launch shape (each item's arithmetic and the
 * fixed-order sums are unchanged): bitwise equal outputs.  Setting a shape
 * drops the plan's captured graphs. */
enum { Q4C_KERNEL_CONTRACT = 0, Q4C_KERNEL_DENSITY = 1, Q4C_KERNEL_HS = 2 /* k_contract_hs, q4c_integrate_HS */ };
int q4c_plan_set_launch(q4c_plan *plan, int32_t kernel, int32_t order, int32_t persistent);
int q4c_plan_get_launch(const q4c_plan *plan, int32_t kernel, int32_t *order, int32_t *persistent);

/* Autotuner: times every candidate shape (order 0/1 x persistent 0, one and
 * two chip-fills of workgroups) of the contraction kernel on this plan with
 * q4c_integrate_H(v_dev, precision) into store_dev (5 store_len doubles,
 * overwritten), and, when coef_dev / out_dev are given, of the adjoint kernel
 * with density_on_grid(coef_dev, all terms, weight mode 1) into out_dev;
 * median of reps timed calls after one warm-up, HIP events on `stream`.
 * Keeps the fastest shape of each kernel on the plan (a batch-order shape
 * within 2% of the fastest wins over the cost-sorted order, which reads more
 * HBM) and, if table is not
 * NULL, writes up to table_len entries (kernel, order, persistent, ms);
 * *n_entries = number of candidates timed.  Synchronises the stream.  Batch
 * size is a plan-time choice (q4c_opts.p_max): tune it by building plans. */
typedef struct {
  int32_t kernel, order, persistent;
  double ms;
} q4c_tune_entry;
int q4c_plan_autotune(q4c_plan *plan, const double *v_dev, int32_t precision, double *store_dev,
                      const double *coef_dev, double *out_dev, int32_t reps, q4c_tune_entry *table,
                      int32_t table_len, int32_t *n_entries, void *stream);

/* HIP graphs: when enabled, each distinct q4c_integrate_H / density_on_grid
 * call (same buffers, precision, flags or terms) is captured once into a HIP
 * graph on the plan's own stream and replayed on the caller's stream on every
 * later call: the whole launch sequence of a call is one graph launch.  Up to
 * 16 graphs are kept per plan.  Disabled while profiling.  Buffers must stay
 * allocated while graphs that use them may be replayed. */
int q4c_plan_set_graphs(q4c_plan *plan, int enable);

/* Block until the plan's queued work is done; reports asynchronous HIP errors. */
int q4c_plan_sync(const q4c_plan *plan, void *stream);

const char *q4c_status_string(int status);
const char *q4c_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* Q4C_H */
