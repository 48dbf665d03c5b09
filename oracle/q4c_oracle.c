/*
 * ORACLE -- test infrastructure, not part of the library.
 *
 * A plain, slow FP64 CPU implementation of what Q4C real-space grid
 * integration computes.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code with the HIP library.
 *
 * What it computes (paper, Sec. III A, Eq. 29 and Eq. 31; Eq. 39 for the
 * density):
 *
 *   V_ij      = sum_g w_g v_g phi_i(r_g) phi_j(r_g)
 *   Ws_ij     = c' sum_g w_g v_g grad phi_i . grad phi_j
 *   Wso_m,ij  = c' sum_g w_g v_g (grad phi_i x grad phi_j)_m ,  c' = 1/(4 c^2)
 *
 * W = (sigma.p) v (sigma.p) / 4c^2 is the small-small block <chi^S|V|chi^S>
 * (Eq. 16a) with the kinetic-balance operator of Eq. 8b taken with V_A -> 0,
 * K = sigma.p / 2c.  For real phi and p = -i grad, the Pauli identity
 * (sigma.a)(sigma.b) = a.b + i sigma.(a x b) splits it into the scalar part
 * Ws and the three spin-orbit parts Wso_m.
 *
 * The sums run over the whole grid (no batching): batching in the paper
 * (Eq. 31) only regroups the same terms.  Sums are compensated (Neumaier).
 *
 * The paper's own Q4C integrand (Sec. II, Eq. 19, evaluated on scalar
 * functions as in Eq. 29) is also stated here, for one component X (large
 * or small) whose scalar functions are given as a basis of their own:
 *
 *   F_ij = sum_g w_g phi_i (eps_j - V_j(|r_g - R_B(j)|) + v_g) phi_j
 *   H_ij = (F_ij + F_ji) / 2
 *        = sum_g w_g phi_i phi_j (v_g + (u_i + u_j) / 2),  u_k = eps_k - V_k
 *   S_ij = sum_g w_g phi_i phi_j
 *
 * with u_k the per-shell "ket potential" given as a table like the radials.
 * Small-component functions Q(r)/r Y_{l~m~} (Eq. 12b) are real: the i of
 * Eq. 12b cancels between bra and ket.
 *
 * Basis functions (Eq. 12a): phi(r) = R(s)/s^l * S_lm(r - R_A), where
 * S_lm = s^l Y_lm is the real solid harmonic with the real Y_lm of App. B
 * (Condon-Shortley convention as written there), and the radial part
 * Rt(s) = R(s)/s^l is given as a piecewise cubic on knots
 * r_j = rcut (j/nint)^2, coefficients (c0..c3) per interval in t in [0,1).
 * phi = 0 for s >= rcut.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t n_atoms;
  const double *R;              /* [3*n_atoms] */
  const int32_t *atom_shell_off; /* [n_atoms+1] */
  const int32_t *shell_l;        /* [n_shells] */
  const double *shell_rcut;      /* [n_shells] */
  const int32_t *shell_nint;     /* [n_shells] */
  const int64_t *shell_coef_off; /* [n_shells] */
  const double *coef;            /* 4 doubles per interval */
} orc_basis;

/* ------------------------------------------------------------------ */
/* Real spherical harmonics, App. B                                    */
/* ------------------------------------------------------------------ */

static double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

static double ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

/* Coefficients a[j] (j = 0..l-m) of the m-th derivative of the Legendre
 * polynomial P_l(t) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) t^(l-2k). */
static void legendre_deriv(int l, int m, double *a) {
  for (int j = 0; j <= l; ++j) a[j] = 0.0;
  for (int k = 0; 2 * k <= l; ++k) {
    int p = l - 2 * k;
    if (p < m) continue;
    double c = ipow(0.5, l) * ((k & 1) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l);
    a[p - m] += c * fact(p) / fact(p - m);
  }
}

/*
 * S = s^l Y_lm(theta, phi) at (x, y, z) relative to the centre, and its
 * Cartesian gradient.
 *
 * App. B: P_l^m(cos t) = sin^m(t) d^m/d(cos t)^m P_l(cos t) (no (-1)^m inside),
 *   Y_l^m = (-1)^m sqrt2 K cos(m phi) P_l^m      (m > 0)
 *         = K P_l^0                               (m = 0)
 *         = (-1)^m sqrt2 K sin(|m| phi) P_l^|m|   (m < 0)
 *   K = sqrt((2l+1)(l-|m|)! / (4 pi (l+|m|)!)).
 * With s^m sin^m(t) cos(m phi) = Re (x+iy)^m, s^m sin^m(t) sin(m phi) = Im (x+iy)^m
 * and s^(l-m) P_l^(m)(z/s) = sum_j a_j z^j (s^2)^((l-m-j)/2), S is a polynomial.
 */
void orc_solid_harmonic(int l, int m, double x, double y, double z, double *S, double *g) {
  int am = m < 0 ? -m : m;
  double K = sqrt((2.0 * l + 1.0) * fact(l - am) / (4.0 * M_PI * fact(l + am)));
  double pref = (m == 0) ? K : ((am & 1) ? -1.0 : 1.0) * sqrt(2.0) * K;
  /* (x+iy)^am and (x+iy)^(am-1) */
  double cr = 1.0, ci = 0.0, pr = 0.0, pi_ = 0.0;
  for (int k = 0; k < am; ++k) {
    pr = cr;
    pi_ = ci;
    double nr = cr * x - ci * y, ni = cr * y + ci * x;
    cr = nr;
    ci = ni;
  }
  double A, Ax, Ay;
  if (m >= 0) {
    A = cr;
    Ax = am * pr;
    Ay = -am * pi_;
  } else {
    A = ci;
    Ax = am * pi_;
    Ay = am * pr;
  }
  if (am == 0) {
    Ax = 0.0;
    Ay = 0.0;
  }
  double a[8];
  legendre_deriv(l, am, a);
  double rho = x * x + y * y + z * z;
  double Q = 0.0, Qx = 0.0, Qy = 0.0, Qz = 0.0;
  for (int j = 0; j <= l - am; ++j) {
    if (a[j] == 0.0) continue;
    int e = (l - am - j) / 2;
    double zj = ipow(z, j), re = ipow(rho, e);
    Q += a[j] * zj * re;
    if (e >= 1) {
      double re1 = ipow(rho, e - 1);
      Qx += a[j] * zj * e * re1 * 2.0 * x;
      Qy += a[j] * zj * e * re1 * 2.0 * y;
      Qz += a[j] * zj * e * re1 * 2.0 * z;
    }
    if (j >= 1) Qz += a[j] * j * ipow(z, j - 1) * re;
  }
  *S = pref * A * Q;
  g[0] = pref * (Ax * Q + A * Qx);
  g[1] = pref * (Ay * Q + A * Qy);
  g[2] = pref * (A * Qz);
}

/*
 * Magnitude bounds of S_lm and grad S_lm at (x, y, z): the sums of |terms|
 * of their polynomials in x, y, z.  With the factorisation above,
 * S = pref A Q, every monomial of Re/Im (x+iy)^m is bounded in sum by
 * (|x|+|y|)^m and every monomial of Q = sum_j a_j z^j rho^e (rho = x^2 + y^2
 * + z^2, whose terms are all positive) by sum_j |a_j| |z|^j rho^e; the same
 * holds term by term for the derivatives.  A value computed from any
 * expansion of S then carries a rounding error of a few ulps of Sm (resp.
 * gm), also where S itself cancels (near its nodal planes).
 */
static void solid_harmonic_mag(int l, int m, double x, double y, double z, double *Sm, double *gm) {
  int am = m < 0 ? -m : m;
  double K = sqrt((2.0 * l + 1.0) * fact(l - am) / (4.0 * M_PI * fact(l + am)));
  double pref = (m == 0) ? K : sqrt(2.0) * K;
  double ax = fabs(x), ay = fabs(y), az = fabs(z);
  double Am = ipow(ax + ay, am), Ad = am > 0 ? am * ipow(ax + ay, am - 1) : 0.0;
  double a[8];
  legendre_deriv(l, am, a);
  double rho = x * x + y * y + z * z;
  double Q = 0.0, Qx = 0.0, Qy = 0.0, Qz = 0.0;
  for (int j = 0; j <= l - am; ++j) {
    if (a[j] == 0.0) continue;
    int e = (l - am - j) / 2;
    double c = fabs(a[j]), zj = ipow(az, j), re = ipow(rho, e);
    Q += c * zj * re;
    if (e >= 1) {
      double re1 = ipow(rho, e - 1);
      Qx += c * zj * e * re1 * 2.0 * ax;
      Qy += c * zj * e * re1 * 2.0 * ay;
      Qz += c * zj * e * re1 * 2.0 * az;
    }
    if (j >= 1) Qz += c * j * ipow(az, j - 1) * re;
  }
  *Sm = pref * Am * Q;
  gm[0] = pref * (Ad * Q + Am * Qx);
  gm[1] = pref * (Ad * Q + Am * Qy);
  gm[2] = pref * Am * Qz;
}

/* ------------------------------------------------------------------ */
/* Radial table                                                        */
/* ------------------------------------------------------------------ */

/* Rt(s) and Rt'(s); with cval/cder non-NULL also the evaluation scales
 * sum_k |c_k t^k| and sum_k k |c_k t^(k-1)| / h (the size of the terms the
 * cubic is summed from, which bounds its rounding error). */
static void radial_eval(const double *tab, int nint, double rcut, double s, double *val, double *der, double *cval,
                        double *cder) {
  if (!(s < rcut)) {
    *val = 0.0;
    *der = 0.0;
    if (cval) *cval = 0.0;
    if (cder) *cder = 0.0;
    return;
  }
  int j = (int)floor(nint * sqrt(s / rcut));
  if (j > nint - 1) j = nint - 1;
  if (j < 0) j = 0;
  double rj = rcut * ((double)j / nint) * ((double)j / nint);
  double rj1 = rcut * ((double)(j + 1) / nint) * ((double)(j + 1) / nint);
  double h = rj1 - rj;
  double t = (s - rj) / h;
  const double *c = tab + 4 * (int64_t)j;
  *val = c[0] + c[1] * t + c[2] * t * t + c[3] * t * t * t;
  *der = (c[1] + 2.0 * c[2] * t + 3.0 * c[3] * t * t) / h;
  if (cval) *cval = fabs(c[0]) + fabs(c[1] * t) + fabs(c[2] * t * t) + fabs(c[3] * t * t * t);
  if (cder) *cder = (fabs(c[1]) + fabs(2.0 * c[2] * t) + fabs(3.0 * c[3] * t * t)) / h;
}

/* Magnitude of the terms of Rt''(s): sum_k k (k-1) |c_k t^(k-2)| / h^2. */
static double radial_d2_mag(const double *tab, int nint, double rcut, double s) {
  if (!(s < rcut)) return 0.0;
  int j = (int)floor(nint * sqrt(s / rcut));
  if (j > nint - 1) j = nint - 1;
  if (j < 0) j = 0;
  double rj = rcut * ((double)j / nint) * ((double)j / nint);
  double rj1 = rcut * ((double)(j + 1) / nint) * ((double)(j + 1) / nint);
  double h = rj1 - rj;
  double t = (s - rj) / h;
  const double *c = tab + 4 * (int64_t)j;
  return (fabs(2.0 * c[2]) + fabs(6.0 * c[3] * t)) / (h * h);
}

void orc_radial(const double *tab, int nint, double rcut, double s, double *val, double *der) {
  radial_eval(tab, nint, rcut, s, val, der, NULL, NULL);
}

/* number of functions on atom a */
static int atom_nfn(const orc_basis *b, int a) {
  int n = 0;
  for (int s = b->atom_shell_off[a]; s < b->atom_shell_off[a + 1]; ++s) n += 2 * b->shell_l[s] + 1;
  return n;
}

static double atom_rcut(const orc_basis *b, int a) {
  double r = 0.0;
  for (int s = b->atom_shell_off[a]; s < b->atom_shell_off[a + 1]; ++s)
    if (b->shell_rcut[s] > r) r = b->shell_rcut[s];
  return r;
}

/*
 * Values and gradients of every function of atom a at point (px,py,pz).
 * phi = Rt(s) S_lm(d), grad phi = Rt'(s) (d/s) S_lm + Rt(s) grad S_lm, d = p - R_a.
 * At s = 0 the first gradient term is 0 (Rt'(s) d/s -> 0 for a smooth radial).
 */
static void atom_functions_c(const orc_basis *b, int a, double px, double py, double pz, double *phi,
                             double *grad, double *aphi, double *agrad) {
  double dx = px - b->R[3 * a], dy = py - b->R[3 * a + 1], dz = pz - b->R[3 * a + 2];
  double s = sqrt(dx * dx + dy * dy + dz * dz);
  int f = 0;
  for (int sh = b->atom_shell_off[a]; sh < b->atom_shell_off[a + 1]; ++sh) {
    int l = b->shell_l[sh];
    double Rt, dRt, cR, cdR;
    radial_eval(b->coef + b->shell_coef_off[sh], b->shell_nint[sh], b->shell_rcut[sh], s, &Rt, &dRt, &cR, &cdR);
    double u[3] = {0.0, 0.0, 0.0}, au[3] = {0.0, 0.0, 0.0};
    if (s > 0.0) {
      u[0] = dRt * dx / s;
      u[1] = dRt * dy / s;
      u[2] = dRt * dz / s;
      au[0] = cdR * fabs(dx) / s;
      au[1] = cdR * fabs(dy) / s;
      au[2] = cdR * fabs(dz) / s;
    }
    for (int m = -l; m <= l; ++m, ++f) {
      double S, gS[3];
      orc_solid_harmonic(l, m, dx, dy, dz, &S, gS);
      phi[f] = Rt * S;
      for (int c = 0; c < 3; ++c) grad[3 * f + c] = u[c] * S + Rt * gS[c];
      if (aphi) {
        aphi[f] = cR * fabs(S);
        for (int c = 0; c < 3; ++c) agrad[3 * f + c] = au[c] * fabs(S) + cR * fabs(gS[c]);
      }
    }
  }
}

/*
 * As atom_functions_c, with the magnitudes of the terms each value is summed
 * from: the radial cubic's sum_k |c_k t^k| (and derivative analogue) times
 * the magnitude bound of S_lm (and of its gradient) from solid_harmonic_mag,
 * plus the value's sensitivity to the rounding of the distance: a distance
 * s known to a few ulps moves Rt by Rt'(s) s u, which dominates in the steep
 * tails of tight functions (|Rt'/Rt| = 2 alpha s for a Gaussian), so the
 * scale of phi adds |Rt'| s |S| and that of d_c phi adds
 * (|Rt''| s + |Rt'|) |d_c| / s |S| + |Rt'| s |d_c S| (term magnitudes
 * again).  These bound the rounding of a value computed in any order at any
 * point, including near the nodal planes of S_lm; they are the error scale
 * of a single tabulated value and of the density at one point.
 */
static void atom_functions_m(const orc_basis *b, int a, double px, double py, double pz, double *phi,
                             double *grad, double *aphi, double *agrad) {
  double dx = px - b->R[3 * a], dy = py - b->R[3 * a + 1], dz = pz - b->R[3 * a + 2];
  double s = sqrt(dx * dx + dy * dy + dz * dz);
  int f = 0;
  for (int sh = b->atom_shell_off[a]; sh < b->atom_shell_off[a + 1]; ++sh) {
    int l = b->shell_l[sh];
    double Rt, dRt, cR, cdR;
    const double *tab = b->coef + b->shell_coef_off[sh];
    radial_eval(tab, b->shell_nint[sh], b->shell_rcut[sh], s, &Rt, &dRt, &cR, &cdR);
    const double cd2R = radial_d2_mag(tab, b->shell_nint[sh], b->shell_rcut[sh], s);
    double u[3] = {0.0, 0.0, 0.0}, au[3] = {0.0, 0.0, 0.0};
    if (s > 0.0) {
      u[0] = dRt * dx / s;
      u[1] = dRt * dy / s;
      u[2] = dRt * dz / s;
      /* term magnitudes of Rt'(s) d_c / s and their sensitivity to s */
      au[0] = (cdR + cd2R * s + cdR) * fabs(dx) / s;
      au[1] = (cdR + cd2R * s + cdR) * fabs(dy) / s;
      au[2] = (cdR + cd2R * s + cdR) * fabs(dz) / s;
    }
    const double cRs = cR + cdR * s; /* term magnitudes of Rt(s) and its sensitivity to s */
    for (int m = -l; m <= l; ++m, ++f) {
      double S, gS[3], Sm, gm[3];
      orc_solid_harmonic(l, m, dx, dy, dz, &S, gS);
      solid_harmonic_mag(l, m, dx, dy, dz, &Sm, gm);
      phi[f] = Rt * S;
      for (int c = 0; c < 3; ++c) grad[3 * f + c] = u[c] * S + Rt * gS[c];
      aphi[f] = cRs * Sm;
      for (int c = 0; c < 3; ++c) agrad[3 * f + c] = au[c] * Sm + cRs * gm[c];
    }
  }
}

static void atom_functions(const orc_basis *b, int a, double px, double py, double pz, double *phi,
                           double *grad) {
  atom_functions_c(b, a, px, py, pz, phi, grad, NULL, NULL);
}

int orc_n_functions(const orc_basis *b) {
  int n = 0;
  for (int a = 0; a < b->n_atoms; ++a) n += atom_nfn(b, a);
  return n;
}

/* phi[g*nfn + i], grad[(g*nfn + i)*3 + c] for all functions at all points;
 * aphi / agrad (optional, same layout): the magnitudes of atom_functions_m. */
void orc_tabulate(const orc_basis *b, int64_t npts, const double *x, const double *y, const double *z,
                  double *phi, double *grad, double *aphi, double *agrad) {
  int nfn = orc_n_functions(b);
  for (int64_t g = 0; g < npts; ++g) {
    int f0 = 0;
    for (int a = 0; a < b->n_atoms; ++a) {
      if (aphi)
        atom_functions_m(b, a, x[g], y[g], z[g], phi + g * nfn + f0, grad + (g * nfn + f0) * 3,
                         aphi + g * nfn + f0, agrad + (g * nfn + f0) * 3);
      else
        atom_functions(b, a, x[g], y[g], z[g], phi + g * nfn + f0, grad + (g * nfn + f0) * 3);
      f0 += atom_nfn(b, a);
    }
  }
}

/* ------------------------------------------------------------------ */
/* Compensated summation                                               */
/* ------------------------------------------------------------------ */

static inline void neu_add(double *s, double *c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x))
    *c += (*s - t) + x;
  else
    *c += (x - t) + *s;
  *s = t;
}

/*
 * Pair blocks of the five real parts for the listed atom pairs.
 * out for pair p: 5 consecutive nA x nB row-major blocks (V, Ws, Wso_x,
 * Wso_y, Wso_z), rows = functions of A, columns = functions of B.  Blocks of
 * successive pairs follow each other.
 * screened != 0 skips points outside the support of A or of B (exact zeros);
 * screened == 0 evaluates every point (brute force).
 * absout (optional, same layout) receives the error scale of each element:
 * sum_g |w_g v_g| times the sum of the magnitudes of the products that enter
 * the term (|phi_i||phi_j|, sum_a |d_a phi_i||d_a phi_j|, and
 * |d_b phi_i||d_c phi_j| + |d_c phi_i||d_b phi_j| for the spin-orbit parts),
 * where each magnitude is that of the terms the function value is computed
 * from: the radial cubic contributes sum_k |c_k t^k| (resp. its derivative
 * analogue) instead of |Rt|, so tail values that arise from cancellation in
 * the table carry their rounding scale.
 */
int orc_pair_blocks(const orc_basis *b, int64_t npts, const double *x, const double *y, const double *z,
                    const double *w, const double *v, double c_light, int npairs, const int32_t *pa,
                    const int32_t *pb, int screened, double *out, double *absout) {
  const double cp = 1.0 / (4.0 * c_light * c_light);
  int64_t *offs = (int64_t *)malloc(sizeof(int64_t) * (npairs + 1));
  offs[0] = 0;
  for (int p = 0; p < npairs; ++p) offs[p + 1] = offs[p] + 5 * (int64_t)atom_nfn(b, pa[p]) * atom_nfn(b, pb[p]);
  /* pairs are independent: one thread per pair, each element summed in point order */
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < npairs; ++p) {
    int A = pa[p], B = pb[p];
    int nA = atom_nfn(b, A), nB = atom_nfn(b, B);
    double rA = atom_rcut(b, A), rB = atom_rcut(b, B);
    int64_t blk = (int64_t)nA * nB;
    const int64_t off = offs[p];
    double *sum = (double *)calloc(5 * blk, sizeof(double));
    double *cmp = (double *)calloc(5 * blk, sizeof(double));
    double *abs_ = (double *)calloc(5 * blk, sizeof(double));
    double *fa = (double *)malloc(sizeof(double) * nA * 8);
    double *fb = (double *)malloc(sizeof(double) * nB * 8);
    double *ga = fa + nA, *gb = fb + nB;
    double *xa = fa + 4 * nA, *xb = fb + 4 * nB;  /* magnitudes */
    double *ya = xa + nA, *yb = xb + nB;
    for (int64_t g = 0; g < npts; ++g) {
      if (screened) {
        double ax = x[g] - b->R[3 * A], ay = y[g] - b->R[3 * A + 1], az = z[g] - b->R[3 * A + 2];
        double bx = x[g] - b->R[3 * B], by = y[g] - b->R[3 * B + 1], bz = z[g] - b->R[3 * B + 2];
        if (!(ax * ax + ay * ay + az * az < rA * rA)) continue;
        if (!(bx * bx + by * by + bz * bz < rB * rB)) continue;
      }
      double om = w[g] * v[g];
      atom_functions_c(b, A, x[g], y[g], z[g], fa, ga, xa, ya);
      atom_functions_c(b, B, x[g], y[g], z[g], fb, gb, xb, yb);
      for (int i = 0; i < nA; ++i) {
        const double *gi = ga + 3 * i, *hi = ya + 3 * i;
        for (int j = 0; j < nB; ++j) {
          const double *gj = gb + 3 * j, *hj = yb + 3 * j;
          int64_t e = (int64_t)i * nB + j;
          double t[5];
          t[0] = om * fa[i] * fb[j];
          t[1] = om * (gi[0] * gj[0] + gi[1] * gj[1] + gi[2] * gj[2]);
          t[2] = om * (gi[1] * gj[2] - gi[2] * gj[1]);
          t[3] = om * (gi[2] * gj[0] - gi[0] * gj[2]);
          t[4] = om * (gi[0] * gj[1] - gi[1] * gj[0]);
          double ao = fabs(om), a[5];
          a[0] = ao * xa[i] * xb[j];
          a[1] = ao * (hi[0] * hj[0] + hi[1] * hj[1] + hi[2] * hj[2]);
          a[2] = ao * (hi[1] * hj[2] + hi[2] * hj[1]);
          a[3] = ao * (hi[2] * hj[0] + hi[0] * hj[2]);
          a[4] = ao * (hi[0] * hj[1] + hi[1] * hj[0]);
          for (int q = 0; q < 5; ++q) {
            neu_add(sum + q * blk + e, cmp + q * blk + e, t[q]);
            abs_[q * blk + e] += a[q];
          }
        }
      }
    }
    for (int q = 0; q < 5; ++q) {
      double sc = (q == 0) ? 1.0 : cp;
      for (int64_t e = 0; e < blk; ++e) {
        out[off + q * blk + e] = (sum[q * blk + e] + cmp[q * blk + e]) * sc;
        if (absout) absout[off + q * blk + e] = abs_[q * blk + e] * sc;
      }
    }
    free(sum);
    free(cmp);
    free(abs_);
    free(fa);
    free(fb);
  }
  free(offs);
  return 0;
}

/*
 * H and S of one component for the listed atom pairs (the Q4C integrand,
 * Eq. 19 in the scalar form of Eq. 29, symmetrised):
 *
 *   H_ij = sum_g w_g phi_i phi_j (v_g + (u_i(s_A) + u_j(s_B)) / 2)
 *   S_ij = sum_g w_g phi_i phi_j
 *
 * u of shell sh is the piecewise cubic at u_coef + shell_u_off[sh] on the
 * shell's own knots (same format as the radial tables).
 * out for pair p: 2 consecutive nA x nB row-major blocks (H, S).
 * absout (optional): error scales sum_g |w_g| |phi_i| |phi_j| (|v_g| +
 * (|u_i| + |u_j|) / 2) for H and sum_g |w_g| |phi_i| |phi_j| for S, with the
 * magnitudes of the terms the values are summed from (see orc_pair_blocks).
 */
static void atom_ket(const orc_basis *b, const int64_t *shell_u_off, const double *u_coef, int a, double px,
                     double py, double pz, double *u, double *au) {
  double dx = px - b->R[3 * a], dy = py - b->R[3 * a + 1], dz = pz - b->R[3 * a + 2];
  double s = sqrt(dx * dx + dy * dy + dz * dz);
  int f = 0;
  for (int sh = b->atom_shell_off[a]; sh < b->atom_shell_off[a + 1]; ++sh) {
    int l = b->shell_l[sh];
    double val, der, cval, cder;
    radial_eval(u_coef + shell_u_off[sh], b->shell_nint[sh], b->shell_rcut[sh], s, &val, &der, &cval, &cder);
    for (int m = -l; m <= l; ++m, ++f) {
      u[f] = val;
      au[f] = cval;
    }
  }
}

int orc_pair_blocks_hs(const orc_basis *b, const int64_t *shell_u_off, const double *u_coef, int64_t npts,
                       const double *x, const double *y, const double *z, const double *w, const double *v,
                       int npairs, const int32_t *pa, const int32_t *pb, int screened, double *out,
                       double *absout) {
  int64_t *offs = (int64_t *)malloc(sizeof(int64_t) * (npairs + 1));
  offs[0] = 0;
  for (int p = 0; p < npairs; ++p) offs[p + 1] = offs[p] + 2 * (int64_t)atom_nfn(b, pa[p]) * atom_nfn(b, pb[p]);
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < npairs; ++p) {
    int A = pa[p], B = pb[p];
    int nA = atom_nfn(b, A), nB = atom_nfn(b, B);
    double rA = atom_rcut(b, A), rB = atom_rcut(b, B);
    int64_t blk = (int64_t)nA * nB;
    const int64_t off = offs[p];
    double *sum = (double *)calloc(2 * blk, sizeof(double));
    double *cmp = (double *)calloc(2 * blk, sizeof(double));
    double *abs_ = (double *)calloc(2 * blk, sizeof(double));
    /* per side: phi, gradient (unused), magnitudes, u, |u| terms */
    double *fa = (double *)malloc(sizeof(double) * nA * 11);
    double *fb = (double *)malloc(sizeof(double) * nB * 11);
    double *ga = fa + nA, *gb = fb + nB;
    double *xa = fa + 4 * nA, *xb = fb + 4 * nB;
    double *ya = xa + nA, *yb = xb + nB;
    double *ua = ya + 3 * nA, *ub = yb + 3 * nB;
    double *va = ua + nA, *vb = ub + nB;
    for (int64_t g = 0; g < npts; ++g) {
      if (screened) {
        double ax = x[g] - b->R[3 * A], ay = y[g] - b->R[3 * A + 1], az = z[g] - b->R[3 * A + 2];
        double bx = x[g] - b->R[3 * B], by = y[g] - b->R[3 * B + 1], bz = z[g] - b->R[3 * B + 2];
        if (!(ax * ax + ay * ay + az * az < rA * rA)) continue;
        if (!(bx * bx + by * by + bz * bz < rB * rB)) continue;
      }
      atom_functions_c(b, A, x[g], y[g], z[g], fa, ga, xa, ya);
      atom_functions_c(b, B, x[g], y[g], z[g], fb, gb, xb, yb);
      atom_ket(b, shell_u_off, u_coef, A, x[g], y[g], z[g], ua, va);
      atom_ket(b, shell_u_off, u_coef, B, x[g], y[g], z[g], ub, vb);
      for (int i = 0; i < nA; ++i) {
        for (int j = 0; j < nB; ++j) {
          int64_t e = (int64_t)i * nB + j;
          double wpp = w[g] * fa[i] * fb[j];
          double aw = fabs(w[g]) * xa[i] * xb[j];
          neu_add(sum + e, cmp + e, wpp * (v[g] + 0.5 * (ua[i] + ub[j])));
          neu_add(sum + blk + e, cmp + blk + e, wpp);
          abs_[e] += aw * (fabs(v[g]) + 0.5 * (va[i] + vb[j]));
          abs_[blk + e] += aw;
        }
      }
    }
    for (int64_t e = 0; e < 2 * blk; ++e) {
      out[off + e] = sum[e] + cmp[e];
      if (absout) absout[off + e] = abs_[e];
    }
    free(sum);
    free(cmp);
    free(abs_);
    free(fa);
    free(fb);
  }
  free(offs);
  return 0;
}

/*
 * Density / adjoint at the listed points (Eq. 39 with the coefficient
 * matrices given on the same pair blocks as the integrals):
 *
 *   nL_g  = sum_pairs sum_ij C^V_ij phi_i phi_j
 *   nSs_g = c' sum_pairs sum_ij C^Ws_ij grad phi_i . grad phi_j
 *   nSo_g = c' sum_pairs sum_m sum_ij C^m_ij (grad phi_i x grad phi_j)_m
 *
 * coef: per pair 5 blocks nA x nB in the order V, Ws, x, y, z (same layout as
 * orc_pair_blocks output).  Each stored element counts once.
 * out[g] = (weight_mode ? w_g : 1) * (nL + nSs + nSo); parts (optional)
 * receives [g*3 + 0..2] = nL, nSs, nSo (unweighted).
 * scale (optional, [g*3 + 0..2], unweighted): the error scale of each part at
 * the point, the sum over its terms of |C| times the magnitudes of the two
 * function factors (atom_functions_m): |C^V| |phi_i| |phi_j|,
 * c' |C^Ws| sum_a |d_a phi_i| |d_a phi_j| and
 * c' |C^m| (|d_b phi_i| |d_c phi_j| + |d_c phi_i| |d_b phi_j|).  Any order of
 * summing the terms stays within a small multiple of unit roundoff times it.
 */
int orc_density_points(const orc_basis *b, int64_t npts, const double *x, const double *y, const double *z,
                       const double *w, double c_light, int npairs, const int32_t *pa, const int32_t *pb,
                       const double *coef, int weight_mode, double *out, double *parts, double *scale) {
  const double cp = 1.0 / (4.0 * c_light * c_light);
  int na = b->n_atoms;
  int64_t *poff = (int64_t *)malloc(sizeof(int64_t) * (npairs + 1));
  poff[0] = 0;
  for (int p = 0; p < npairs; ++p) poff[p + 1] = poff[p] + 5 * (int64_t)atom_nfn(b, pa[p]) * atom_nfn(b, pb[p]);
  int maxfn = 0;
  for (int a = 0; a < na; ++a)
    if (atom_nfn(b, a) > maxfn) maxfn = atom_nfn(b, a);
  /* points are independent: each thread sums its points' terms in pair order */
#pragma omp parallel
  {
  double *fa = (double *)malloc(sizeof(double) * maxfn * 8);
  double *fb = (double *)malloc(sizeof(double) * maxfn * 8);
#pragma omp for schedule(dynamic, 16)
  for (int64_t g = 0; g < npts; ++g) {
    double sL = 0, cL = 0, sS = 0, cS = 0, sO = 0, cO = 0;
    double mL = 0, mS = 0, mO = 0;
    for (int p = 0; p < npairs; ++p) {
      int A = pa[p], B = pb[p];
      double rA = atom_rcut(b, A), rB = atom_rcut(b, B);
      double ax = x[g] - b->R[3 * A], ay = y[g] - b->R[3 * A + 1], az = z[g] - b->R[3 * A + 2];
      double bx = x[g] - b->R[3 * B], by = y[g] - b->R[3 * B + 1], bz = z[g] - b->R[3 * B + 2];
      if (!(ax * ax + ay * ay + az * az < rA * rA)) continue;
      if (!(bx * bx + by * by + bz * bz < rB * rB)) continue;
      int nA = atom_nfn(b, A), nB = atom_nfn(b, B);
      int64_t blk = (int64_t)nA * nB;
      double *ga = fa + nA, *gb = fb + nB;
      double *xa = fa + 4 * nA, *xb = fb + 4 * nB; /* magnitudes */
      double *ya = xa + nA, *yb = xb + nB;
      if (scale) {
        atom_functions_m(b, A, x[g], y[g], z[g], fa, ga, xa, ya);
        atom_functions_m(b, B, x[g], y[g], z[g], fb, gb, xb, yb);
      } else {
        atom_functions(b, A, x[g], y[g], z[g], fa, ga);
        atom_functions(b, B, x[g], y[g], z[g], fb, gb);
      }
      const double *C = coef + poff[p];
      for (int i = 0; i < nA; ++i) {
        const double *gi = ga + 3 * i;
        for (int j = 0; j < nB; ++j) {
          const double *gj = gb + 3 * j;
          int64_t e = (int64_t)i * nB + j;
          neu_add(&sL, &cL, C[e] * fa[i] * fb[j]);
          neu_add(&sS, &cS, C[blk + e] * (gi[0] * gj[0] + gi[1] * gj[1] + gi[2] * gj[2]));
          neu_add(&sO, &cO, C[2 * blk + e] * (gi[1] * gj[2] - gi[2] * gj[1]));
          neu_add(&sO, &cO, C[3 * blk + e] * (gi[2] * gj[0] - gi[0] * gj[2]));
          neu_add(&sO, &cO, C[4 * blk + e] * (gi[0] * gj[1] - gi[1] * gj[0]));
          if (scale) {
            const double *hi = ya + 3 * i, *hj = yb + 3 * j;
            mL += fabs(C[e]) * xa[i] * xb[j];
            mS += fabs(C[blk + e]) * (hi[0] * hj[0] + hi[1] * hj[1] + hi[2] * hj[2]);
            mO += fabs(C[2 * blk + e]) * (hi[1] * hj[2] + hi[2] * hj[1]) +
                  fabs(C[3 * blk + e]) * (hi[2] * hj[0] + hi[0] * hj[2]) +
                  fabs(C[4 * blk + e]) * (hi[0] * hj[1] + hi[1] * hj[0]);
          }
        }
      }
    }
    double nL = sL + cL, nS = cp * (sS + cS), nO = cp * (sO + cO);
    double f = weight_mode ? w[g] : 1.0;
    out[g] = f * (nL + nS + nO);
    if (parts) {
      parts[3 * g] = nL;
      parts[3 * g + 1] = nS;
      parts[3 * g + 2] = nO;
    }
    if (scale) {
      scale[3 * g] = mL;
      scale[3 * g + 1] = cp * mS;
      scale[3 * g + 2] = cp * mO;
    }
  }
  free(fa);
  free(fb);
  }
  free(poff);
  return 0;
}

/*
 * Density and its gradient at the listed points from one real coefficient
 * block per atom pair (the scalar density matrix of one component, each
 * stored element counted once):
 *   n_g     = sum_pairs sum_ij C_ij phi_i phi_j
 *   dn_g/da = sum_pairs sum_ij C_ij (d_a phi_i phi_j + phi_i d_a phi_j)
 * (the density of Sec. II B / III A on the scalar basis, with the gradient a
 * GGA functional needs).  coef: per pair nA x nB row-major.  out[4 g + k]:
 * k = 0 n, 1..3 the x, y, z derivatives.  Sums are compensated.
 * scale (optional, same layout): the error scale of each output, the sum over
 * its terms of |C_ij| times the magnitudes of the factors (atom_functions_m):
 * |phi_i| |phi_j| for n, |d_a phi_i| |phi_j| + |phi_i| |d_a phi_j| for dn/da.
 */
int orc_density_grad_points(const orc_basis *b, int64_t npts, const double *x, const double *y, const double *z,
                            int npairs, const int32_t *pa, const int32_t *pb, const double *coef, double *out,
                            double *scale) {
  int na = b->n_atoms;
  int64_t *poff = (int64_t *)malloc(sizeof(int64_t) * (npairs + 1));
  poff[0] = 0;
  for (int p = 0; p < npairs; ++p) poff[p + 1] = poff[p] + (int64_t)atom_nfn(b, pa[p]) * atom_nfn(b, pb[p]);
  int maxfn = 0;
  for (int a = 0; a < na; ++a)
    if (atom_nfn(b, a) > maxfn) maxfn = atom_nfn(b, a);
  /* points are independent: each thread sums its points' terms in pair order */
#pragma omp parallel
  {
  double *fa = (double *)malloc(sizeof(double) * maxfn * 8);
  double *fb = (double *)malloc(sizeof(double) * maxfn * 8);
#pragma omp for schedule(dynamic, 16)
  for (int64_t g = 0; g < npts; ++g) {
    double s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0}, m[4] = {0, 0, 0, 0};
    for (int p = 0; p < npairs; ++p) {
      int A = pa[p], B = pb[p];
      double rA = atom_rcut(b, A), rB = atom_rcut(b, B);
      double ax = x[g] - b->R[3 * A], ay = y[g] - b->R[3 * A + 1], az = z[g] - b->R[3 * A + 2];
      double bx = x[g] - b->R[3 * B], by = y[g] - b->R[3 * B + 1], bz = z[g] - b->R[3 * B + 2];
      if (!(ax * ax + ay * ay + az * az < rA * rA)) continue;
      if (!(bx * bx + by * by + bz * bz < rB * rB)) continue;
      int nA = atom_nfn(b, A), nB = atom_nfn(b, B);
      double *ga = fa + nA, *gb = fb + nB;
      double *xa = fa + 4 * nA, *xb = fb + 4 * nB; /* magnitudes */
      double *ya = xa + nA, *yb = xb + nB;
      if (scale) {
        atom_functions_m(b, A, x[g], y[g], z[g], fa, ga, xa, ya);
        atom_functions_m(b, B, x[g], y[g], z[g], fb, gb, xb, yb);
      } else {
        atom_functions(b, A, x[g], y[g], z[g], fa, ga);
        atom_functions(b, B, x[g], y[g], z[g], fb, gb);
      }
      const double *C = coef + poff[p];
      for (int i = 0; i < nA; ++i)
        for (int j = 0; j < nB; ++j) {
          double cij = C[(int64_t)i * nB + j];
          neu_add(&s[0], &c[0], cij * fa[i] * fb[j]);
          for (int k = 0; k < 3; ++k) neu_add(&s[k + 1], &c[k + 1], cij * (ga[3 * i + k] * fb[j] + fa[i] * gb[3 * j + k]));
          if (scale) {
            double ac = fabs(cij);
            m[0] += ac * xa[i] * xb[j];
            for (int k = 0; k < 3; ++k) m[k + 1] += ac * (ya[3 * i + k] * xb[j] + xa[i] * yb[3 * j + k]);
          }
        }
    }
    for (int k = 0; k < 4; ++k) {
      out[4 * g + k] = s[k] + c[k];
      if (scale) scale[4 * g + k] = m[k];
    }
  }
  free(fa);
  free(fb);
  }
  free(poff);
  return 0;
}

/* Threads used by the parallel loops above (OpenMP; 1 without it), and a
 * way to set them: the CPU baseline is timed on all host cores and on one. */
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
