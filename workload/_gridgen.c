/*
 * Input-generation helpers for the seeded synthetic workloads.
 *
 * These produce INPUT data only (partition weights and a model potential on
 * the grid).  They contain none of the Hamiltonian-integration arithmetic;
 * both the library under test and the oracle receive their results as plain
 * arrays.
 *
 *  - becke_weights: Becke (1988) fuzzy-cell partition of unity.  The cell
 *    function is s(mu) = (1 - p(p(p(mu)))) / 2 with p(mu) = 1.5 mu - 0.5 mu^3
 *    and no atomic-size adjustment.  The competing set of a point is the set
 *    of atoms closer than `r_comp` (plus the point's own centre), so the
 *    weights of one point sum to exactly one over that set.
 *  - model_potential: v(r) = sum_A -Z_A erf(|r-R_A|/a)/|r-R_A|, with the
 *    r -> 0 limit -2 Z_A / (a sqrt(pi)).  With r_cut > 0 each term is shifted
 *    by +Z_A/r_cut and dropped beyond r_cut (continuous at r_cut).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double cell_s(double mu) {
  double p = mu;
  for (int k = 0; k < 3; ++k) p = 1.5 * p - 0.5 * p * p * p;
  return 0.5 * (1.0 - p);
}

/* atoms sorted into a uniform cell list for neighbour search */
typedef struct {
  double lo[3], h;
  int n[3];
  int *head, *next;
} cells_t;

static void cells_build(cells_t *c, int na, const double *R, double h) {
  for (int d = 0; d < 3; ++d) c->lo[d] = 1e300;
  double hi[3] = {-1e300, -1e300, -1e300};
  for (int a = 0; a < na; ++a)
    for (int d = 0; d < 3; ++d) {
      if (R[3 * a + d] < c->lo[d]) c->lo[d] = R[3 * a + d];
      if (R[3 * a + d] > hi[d]) hi[d] = R[3 * a + d];
    }
  c->h = h;
  for (int d = 0; d < 3; ++d) c->n[d] = (int)((hi[d] - c->lo[d]) / h) + 1;
  int64_t nc = (int64_t)c->n[0] * c->n[1] * c->n[2];
  c->head = (int *)malloc(sizeof(int) * nc);
  c->next = (int *)malloc(sizeof(int) * (na > 0 ? na : 1));
  for (int64_t i = 0; i < nc; ++i) c->head[i] = -1;
  for (int a = na - 1; a >= 0; --a) {
    int ix[3];
    for (int d = 0; d < 3; ++d) ix[d] = (int)((R[3 * a + d] - c->lo[d]) / h);
    int64_t id = ((int64_t)ix[2] * c->n[1] + ix[1]) * c->n[0] + ix[0];
    c->next[a] = c->head[id];
    c->head[id] = a;
  }
}

static void cells_free(cells_t *c) {
  free(c->head);
  free(c->next);
}

/* collect atoms within rc of p into out (capacity cap); returns count */
static int cells_query(const cells_t *c, const double *R, const double *p, double rc, int *out, int cap) {
  int lo[3], hi[3], cnt = 0;
  for (int d = 0; d < 3; ++d) {
    lo[d] = (int)floor((p[d] - rc - c->lo[d]) / c->h);
    hi[d] = (int)floor((p[d] + rc - c->lo[d]) / c->h);
    if (lo[d] < 0) lo[d] = 0;
    if (hi[d] > c->n[d] - 1) hi[d] = c->n[d] - 1;
    if (lo[d] > hi[d]) return 0;
  }
  double rc2 = rc * rc;
  for (int iz = lo[2]; iz <= hi[2]; ++iz)
    for (int iy = lo[1]; iy <= hi[1]; ++iy)
      for (int ix = lo[0]; ix <= hi[0]; ++ix) {
        int64_t id = ((int64_t)iz * c->n[1] + iy) * c->n[0] + ix;
        for (int a = c->head[id]; a >= 0; a = c->next[a]) {
          double dx = p[0] - R[3 * a], dy = p[1] - R[3 * a + 1], dz = p[2] - R[3 * a + 2];
          if (dx * dx + dy * dy + dz * dz < rc2 && cnt < cap) out[cnt++] = a;
        }
      }
  return cnt;
}

/* w_out[g] = Becke weight of atom owner[g] at point g (quadrature weight not included). */
int becke_weights(int na, const double *R, int64_t npts, const double *x, const double *y, const double *z,
                  const int32_t *owner, double r_comp, double *w_out) {
  cells_t c;
  cells_build(&c, na, R, r_comp > 1.0 ? r_comp : 1.0);
  int err = 0;
#pragma omp parallel
  {
    int cap = na + 1;
    int *nb = (int *)malloc(sizeof(int) * cap);
    double *dist = (double *)malloc(sizeof(double) * cap);
    double *P = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 4096)
    for (int64_t g = 0; g < npts; ++g) {
      double p[3] = {x[g], y[g], z[g]};
      int m = cells_query(&c, R, p, r_comp, nb, cap);
      int own = owner[g], has = 0;
      for (int k = 0; k < m; ++k) has |= (nb[k] == own);
      if (!has) nb[m++] = own;
      for (int k = 0; k < m; ++k) {
        int a = nb[k];
        double dx = p[0] - R[3 * a], dy = p[1] - R[3 * a + 1], dz = p[2] - R[3 * a + 2];
        dist[k] = sqrt(dx * dx + dy * dy + dz * dz);
      }
      double sum = 0.0, pown = 0.0;
      for (int k = 0; k < m; ++k) {
        double prod = 1.0;
        int a = nb[k];
        for (int l = 0; l < m && prod != 0.0; ++l) {
          if (l == k) continue;
          int b = nb[l];
          double rx = R[3 * a] - R[3 * b], ry = R[3 * a + 1] - R[3 * b + 1], rz = R[3 * a + 2] - R[3 * b + 2];
          double rab = sqrt(rx * rx + ry * ry + rz * rz);
          prod *= cell_s((dist[k] - dist[l]) / rab);
        }
        P[k] = prod;
        sum += prod;
        if (a == own) pown = prod;
      }
      w_out[g] = sum > 0.0 ? pown / sum : 0.0;
    }
    free(nb);
    free(dist);
    free(P);
  }
  cells_free(&c);
  return err;
}

int model_potential(int na, const double *R, const double *Z, int64_t npts, const double *x, const double *y,
                    const double *z, double a_smear, double r_cut, double *v_out) {
  const double lim_fac = 2.0 / (a_smear * sqrt(M_PI));
  if (r_cut <= 0.0) {
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < npts; ++g) {
      double acc = 0.0;
      for (int a = 0; a < na; ++a) {
        double dx = x[g] - R[3 * a], dy = y[g] - R[3 * a + 1], dz = z[g] - R[3 * a + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        acc += (r > 0.0) ? -Z[a] * erf(r / a_smear) / r : -Z[a] * lim_fac;
      }
      v_out[g] = acc;
    }
    return 0;
  }
  cells_t c;
  cells_build(&c, na, R, r_cut);
#pragma omp parallel
  {
    int *nb = (int *)malloc(sizeof(int) * (na + 1));
#pragma omp for schedule(dynamic, 4096)
    for (int64_t g = 0; g < npts; ++g) {
      double p[3] = {x[g], y[g], z[g]};
      int m = cells_query(&c, R, p, r_cut, nb, na + 1);
      double acc = 0.0;
      for (int k = 0; k < m; ++k) {
        int a = nb[k];
        double dx = p[0] - R[3 * a], dy = p[1] - R[3 * a + 1], dz = p[2] - R[3 * a + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        acc += ((r > 0.0) ? -Z[a] * erf(r / a_smear) / r : -Z[a] * lim_fac) + Z[a] / r_cut;
      }
      v_out[g] = acc;
    }
    free(nb);
  }
  cells_free(&c);
  return 0;
}
