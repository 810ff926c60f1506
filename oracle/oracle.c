/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, FP64 CPU statement of what the mapping hot path computes,
 * used by the tests, the smoke check and the benchmark's CPU baseline to
 * check the device library.  It shares no code with the device library and
 * must never be called by it.
 *
 * What it computes (SPH-to-Voronoi "Exact" mapping, Sec. 1 and Sec. 2.3, with
 * the M4 cubic-spline kernel truncated at 2h, Sec. 2.4.2):
 *   w_ic = integral over Voronoi cell c of W(|r - x_i|, h_i) dV
 *   M_c  = sum_i m_i w_ic,  rho_c = M_c / V_c          (forward mapping)
 *   c_i  = sum_c w_ic                                   (coverage)
 *   q_i  = sum_c w_ic q_c / c_i                         (inverse mapping)
 * and the tree-node pseudo-particle builder of Sec. 2.4 (tree walk with the
 * opening-angle criterion, eq. opening_angle; node smoothing lengths from
 * eqs. h_node, n_node, hnode_func, hnode_func_deriv, hnode_newton_raphson and
 * hnode_estval with the bisection and fallback rules of Sec. 2.4.2).
 *
 * Route for w_ic (the paper cites the analytic solution but does not print
 * it): the cell is a convex polyhedron, so w = sum_f sgn(d_f) I_f where I_f is
 * the kernel integral over the cone with apex x and base face f and d_f the
 * signed distance from x to the face plane (positive on the cell side).  In
 * spherical coordinates about x, I_f = (1/4pi) int_{Omega_f} Phi(R(Omega))
 * dOmega with Phi(q) the fraction of kernel mass inside radius q.  Writing the
 * face in polar coordinates about the foot point P0 and splitting it into the
 * signed triangles (P0, A, B) of its edges gives
 *   I_f = (1/4pi) sum_e sgn(p_e) int_{phi_A}^{phi_B} Psi_d(U(phi)) dphi,
 *   U(phi) = sqrt(d^2 + p_e^2 sec^2 phi),
 *   Psi_d(U) = |d| int_{|d|}^{U} Phi(u)/u^2 du,
 * (lengths in units of h).  Psi is taken in closed form from the radial
 * antiderivative of Phi(u)/u^2; the angular integral is done by adaptive
 * Gauss-Kronrod (7/15) with breakpoints where U crosses 1 and 2.
 *
 * Parity-pinned by the tests against: the kernel normalisation and Phi, an
 * independent slab integral of the half-space, 3-D quadrature of a cube,
 * Monte-Carlo sampling of the kernel over random convex cells, partition of
 * unity over tessellations, symmetry (edge 1/4, corner 1/8), additivity under
 * plane splits and the exact 0/1 limits.
 *
 * Build: gcc -O2 -std=c99 -fopenmp -ffp-contract=off -shared -fPIC oracle.c -lm
 * (no FMA contraction: the candidate-pair test and the tree sums are defined
 * operation by operation).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* OpenMP threads the oracle's parallel loops use. */
int ora_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ kernel */
/* M4 cubic spline shape, W(r,h) = w(r/h) / (pi h^3), zero beyond 2h. */
double ora_w(double q) {
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) return 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
  return 0.0;
}

/* dw/dq */
double ora_dw(double q) {
  if (q < 1.0) return -3.0 * q + 2.25 * q * q;
  if (q < 2.0) return -0.75 * (2.0 - q) * (2.0 - q);
  return 0.0;
}

/* Phi(q) = 4 int_0^q s^2 w(s) ds, the fraction of kernel mass within q. */
double ora_Phi(double q) {
  if (q <= 0.0) return 0.0;
  if (q < 1.0) return (4.0 / 3.0) * q * q * q - 1.2 * pow(q, 5) + 0.5 * pow(q, 6);
  if (q < 2.0)
    return -1.0 / 15.0 + (8.0 / 3.0) * q * q * q - 3.0 * pow(q, 4) + 1.2 * pow(q, 5) - pow(q, 6) / 6.0;
  return 1.0;
}

/* A continuous antiderivative of Phi(u)/u^2 on u > 0. */
double ora_G(double u) {
  if (u < 1.0) return (2.0 / 3.0) * u * u - 0.3 * pow(u, 4) + 0.1 * pow(u, 5);
  if (u < 2.0)
    return 1.0 / (15.0 * u) + (4.0 / 3.0) * u * u - u * u * u + 0.3 * pow(u, 4) - pow(u, 5) / 30.0 - 0.2;
  return 1.4 - 1.0 / u;
}

/* Psi_d(U) = |d| int_{|d|}^{U} Phi(u)/u^2 du  (ad = |d| > 0, U >= ad). */
double ora_Psi(double ad, double U) { return ad * (ora_G(U) - ora_G(ad)); }

/* ---------------------------------------------------- adaptive quadrature */
static const double gk_x[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                               0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                               0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                               0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double gk_wk[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                                0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                                0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                                0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double gk_wg[4] = {0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
                                0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

typedef struct {
  double ad, p2, d2;
} edge_t;

/* Integrand of one right-triangle fan written in the coordinate tau along
   the edge (tau = |p| tan phi, dphi = |p| dtau / (p^2 + tau^2)):
   Psi_d(U) |p| / (p^2 + tau^2) with U = sqrt(d^2 + p^2 + tau^2).  In tau the
   integrand stays smooth when the foot point nears the edge line (p -> 0),
   where the same integral in phi narrows to a spike next to +-pi/2. */
static double fan_integrand(const edge_t *e, double tau) {
  double r2 = e->p2 + tau * tau;
  double U = sqrt(e->d2 + r2);
  return ora_Psi(e->ad, U) * sqrt(e->p2) / r2;
}

static double gk15(const edge_t *e, double a, double b, double *err) {
  double c = 0.5 * (a + b), hw = 0.5 * (b - a);
  double fc = fan_integrand(e, c);
  double rk = fc * gk_wk[7], rg = fc * gk_wg[3];
  for (int j = 0; j < 7; ++j) {
    double dx = hw * gk_x[j];
    double f1 = fan_integrand(e, c - dx), f2 = fan_integrand(e, c + dx);
    rk += gk_wk[j] * (f1 + f2);
    if (j % 2 == 1) rg += gk_wg[j / 2] * (f1 + f2);
  }
  *err = fabs((rk - rg) * hw);
  return rk * hw;
}

static double adapt(const edge_t *e, double a, double b, double tol, int depth) {
  double err;
  double r = gk15(e, a, b, &err);
  if (err <= tol || depth >= 50 || b - a < 1e-15) return r;
  double m = 0.5 * (a + b);
  return adapt(e, a, m, 0.5 * tol, depth + 1) + adapt(e, m, b, 0.5 * tol, depth + 1);
}

/* int_{tA}^{tB} Psi_d(U) |p| dtau / (p^2 + tau^2), i.e. the fan integral
   int Psi_d(U(phi)) dphi over the same triangle, with breakpoints at tau = 0
   and where U = 1 or U = 2. */
static double fan_integral_tau(double ad, double p, double pa, double pb) {
  edge_t e = {ad, p * p, ad * ad};
  double bp[8];
  int nb = 0;
  bp[nb++] = pa;
  double cand[5];
  int nc = 0;
  cand[nc++] = 0.0;
  for (int k = 1; k <= 2; ++k) {
    double r2 = (double)(k * k) - e.d2 - e.p2; /* tau^2 = k^2 - d^2 - p^2 */
    if (r2 > 0.0) {
      double t = sqrt(r2);
      cand[nc++] = t;
      cand[nc++] = -t;
    }
  }
  /* sort candidates ascending */
  for (int i = 1; i < nc; ++i)
    for (int j = i; j > 0 && cand[j] < cand[j - 1]; --j) {
      double t = cand[j];
      cand[j] = cand[j - 1];
      cand[j - 1] = t;
    }
  for (int i = 0; i < nc; ++i)
    if (cand[i] > pa && cand[i] < pb) bp[nb++] = cand[i];
  bp[nb++] = pb;
  double s = 0.0;
  for (int i = 0; i + 1 < nb; ++i) s += adapt(&e, bp[i], bp[i + 1], 1e-14, 0);
  return s;
}

/* ------------------------------------------------------------ geometry */
static void v_sub(const double *a, const double *b, double *o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
static double v_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void v_cross(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Area vector (Newell) of a polygon and its vertex centroid. */
static void poly_area_vec(int nv, const double *const *V, double *avec, double *cen) {
  cen[0] = cen[1] = cen[2] = 0.0;
  for (int k = 0; k < nv; ++k)
    for (int j = 0; j < 3; ++j) cen[j] += V[k][j];
  for (int j = 0; j < 3; ++j) cen[j] /= nv;
  avec[0] = avec[1] = avec[2] = 0.0;
  for (int k = 0; k < nv; ++k) {
    double a[3], b[3], c[3];
    v_sub(V[k], cen, a);
    v_sub(V[(k + 1) % nv], cen, b);
    v_cross(a, b, c);
    for (int j = 0; j < 3; ++j) avec[j] += 0.5 * c[j];
  }
}

/* Kernel integral of particle (x, h) over the cone with apex x and base the
   convex polygon V[0..nv-1], whose orientation gives the outward normal n
   (CCW seen from outside).  Returns sgn(d) I_f. */
static double face_term(const double *x, double h, int nv, const double *const *V, const double *nhat,
                        const double *cen) {
  double xc[3];
  v_sub(cen, x, xc);
  double d = v_dot(nhat, xc); /* > 0: x on the inner side */
  if (d == 0.0) return 0.0;
  double ad = fabs(d) / h;
  double P0[3] = {x[0] + d * nhat[0], x[1] + d * nhat[1], x[2] + d * nhat[2]};
  double sum = 0.0;
  for (int k = 0; k < nv; ++k) {
    const double *A = V[k], *B = V[(k + 1) % nv];
    double ab[3];
    v_sub(B, A, ab);
    double len = sqrt(v_dot(ab, ab));
    if (len == 0.0) continue;
    double e[3] = {ab[0] / len, ab[1] / len, ab[2] / len};
    double mvec[3];
    v_cross(nhat, e, mvec); /* in-plane normal pointing into the polygon */
    double pa[3], pb[3];
    v_sub(P0, A, pa);
    double p = v_dot(pa, mvec) / h; /* > 0: foot on the inner side */
    if (p == 0.0) continue;
    double ta[3];
    v_sub(A, P0, ta);
    v_sub(B, P0, pb);
    double tA = v_dot(ta, e) / h, tB = v_dot(pb, e) / h;
    double s = fan_integral_tau(ad, p, tA, tB);
    sum += (p > 0 ? 1.0 : -1.0) * s;
  }
  return (d > 0 ? 1.0 : -1.0) * sum / (4.0 * M_PI);
}

/* w = integral of W(|r-x|,h) over one convex cell given as faces.
   cell_ref: a point strictly inside the cell (used to orient the faces). */
static double cell_weight_faces(const double *x, double h, int nf, const int *fsz,
                                const double *const *fv /* concatenated vertex pointers */,
                                const double *inside) {
  double w = 0.0;
  int off = 0;
  for (int f = 0; f < nf; ++f) {
    int nv = fsz[f];
    const double *const *V = fv + off;
    off += nv;
    if (nv < 3) continue;
    double avec[3], cen[3];
    poly_area_vec(nv, V, avec, cen);
    double an = sqrt(v_dot(avec, avec));
    if (an == 0.0) continue;
    double nhat[3] = {avec[0] / an, avec[1] / an, avec[2] / an};
    double gc[3];
    v_sub(cen, inside, gc);
    if (v_dot(nhat, gc) < 0.0) {
      /* reversed orientation: walk the polygon backwards */
      const double *R[512];
      if (nv > 512) continue;
      for (int k = 0; k < nv; ++k) R[k] = V[nv - 1 - k];
      double nn[3] = {-nhat[0], -nhat[1], -nhat[2]};
      w += face_term(x, h, nv, R, nn, cen);
    } else {
      w += face_term(x, h, nv, V, nhat, cen);
    }
  }
  return w;
}

/* ----------------------------------------------- tessellation accessors */
typedef struct {
  int64_t n_cells;
  const double *gen;      /* [C][3] */
  const double *vert;     /* [V][3] */
  const int64_t *cfo;     /* [C+1]  */
  const int64_t *fvo;     /* [F+1]  */
  const int32_t *fv;      /* [FV]   */
} tess_t;

static double cell_weight(const tess_t *T, int64_t c, const double *x, double h) {
  int64_t f0 = T->cfo[c], f1 = T->cfo[c + 1];
  int nf = (int)(f1 - f0);
  int tot = (int)(T->fvo[f1] - T->fvo[f0]);
  int *fsz = (int *)malloc(sizeof(int) * (nf > 0 ? nf : 1));
  const double **fvp = (const double **)malloc(sizeof(double *) * (tot > 0 ? tot : 1));
  double inside[3] = {0, 0, 0};
  int k = 0;
  for (int64_t f = f0; f < f1; ++f) {
    fsz[f - f0] = (int)(T->fvo[f + 1] - T->fvo[f]);
    for (int64_t t = T->fvo[f]; t < T->fvo[f + 1]; ++t) {
      fvp[k] = T->vert + 3 * (int64_t)T->fv[t];
      for (int j = 0; j < 3; ++j) inside[j] += fvp[k][j];
      ++k;
    }
  }
  /* the vertex-incidence average of a convex cell lies strictly inside */
  for (int j = 0; j < 3; ++j) inside[j] /= (k > 0 ? k : 1);
  double w = cell_weight_faces(x, h, nf, fsz, fvp, inside);
  free(fsz);
  free(fvp);
  return w;
}

/* Volume by the divergence theorem over the (outward-oriented) faces. */
double ora_cell_volume_t(const tess_t *T, int64_t c) {
  int64_t f0 = T->cfo[c], f1 = T->cfo[c + 1];
  double inside[3] = {0, 0, 0};
  int k = 0;
  for (int64_t t = T->fvo[f0]; t < T->fvo[f1]; ++t, ++k)
    for (int j = 0; j < 3; ++j) inside[j] += T->vert[3 * (int64_t)T->fv[t] + j];
  for (int j = 0; j < 3; ++j) inside[j] /= (k > 0 ? k : 1);
  double vol = 0.0;
  for (int64_t f = f0; f < f1; ++f) {
    int nv = (int)(T->fvo[f + 1] - T->fvo[f]);
    if (nv < 3 || nv > 512) continue;
    const double *V[512];
    for (int q = 0; q < nv; ++q) V[q] = T->vert + 3 * (int64_t)T->fv[T->fvo[f] + q];
    double avec[3], cen[3];
    poly_area_vec(nv, V, avec, cen);
    double gc[3];
    v_sub(cen, inside, gc);
    vol += fabs(v_dot(gc, avec)) / 3.0;
  }
  return vol;
}

/* --------------------------------------------- canonical candidate pairs */
/* Bounding radius of cell c about its generator: the smallest binary32 R
   with R*R >= max_v |v - g|^2 (FP64, (dx*dx + dy*dy) + dz*dz). */
float ora_cell_radius_t(const tess_t *T, int64_t c) {
  const double *g = T->gen + 3 * c;
  double r2 = 0.0;
  for (int64_t t = T->fvo[T->cfo[c]]; t < T->fvo[T->cfo[c + 1]]; ++t) {
    const double *v = T->vert + 3 * (int64_t)T->fv[t];
    double dx = v[0] - g[0], dy = v[1] - g[1], dz = v[2] - g[2];
    double s = (dx * dx + dy * dy) + dz * dz;
    if (s > r2) r2 = s;
  }
  float R = (float)sqrt(r2);
  while ((double)R * (double)R < r2) R = nextafterf(R, INFINITY);
  while (R > 0.0f) {
    float Rm = nextafterf(R, 0.0f);
    if ((double)Rm * (double)Rm >= r2) R = Rm;
    else break;
  }
  return R;
}

/* The canonical binary32 test: (c,i) is a candidate pair iff
   d2 < s*s with dx = fl(x_i) - fl(g_x) (likewise y, z),
   d2 = (dx*dx + dy*dy) + dz*dz and s = R_c + 2 fl(h_i). */
static int canon_pair(const double *x, double h, const double *g, float R) {
  float dx = (float)x[0] - (float)g[0];
  float dy = (float)x[1] - (float)g[1];
  float dz = (float)x[2] - (float)g[2];
  float d2 = (dx * dx + dy * dy) + dz * dz;
  float s = R + 2.0f * (float)h;
  return d2 < s * s;
}

/* ------------------------------------------------------------ public API */

/* Candidate pairs and weights of the listed cells (brute force over all
   particles).  Pass 1 (w == NULL): counts[k] = number of pairs of cells[k].
   Pass 2: for each listed cell, in order, particle indices ascending into
   idx[] and weights into w[] (offsets are the running sum of counts). */
void ora_pairs_weights(int64_t n_cells, const double *gen, const double *vert, const int64_t *cfo,
                       const int64_t *fvo, const int32_t *fv, int64_t n_part, const double *xyz,
                       const double *h, int64_t n_list, const int64_t *cells, int64_t *counts,
                       const int64_t *offsets, int32_t *idx, double *w) {
  tess_t T = {n_cells, gen, vert, cfo, fvo, fv};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n_list; ++k) {
    int64_t c = cells[k];
    float R = ora_cell_radius_t(&T, c);
    const double *g = gen + 3 * c;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n_part; ++i) {
      if (!canon_pair(xyz + 3 * i, h[i], g, R)) continue;
      if (idx) {
        int64_t o = offsets[k] + cnt;
        idx[o] = (int32_t)i;
        if (w) w[o] = cell_weight(&T, c, xyz + 3 * i, h[i]);
      }
      ++cnt;
    }
    if (!idx) counts[k] = cnt;
  }
}

/* Weight of one particle over one cell, regardless of the pair test. */
double ora_weight(int64_t n_cells, const double *gen, const double *vert, const int64_t *cfo,
                  const int64_t *fvo, const int32_t *fv, int64_t c, const double *x, double h) {
  tess_t T = {n_cells, gen, vert, cfo, fvo, fv};
  return cell_weight(&T, c, x, h);
}

/* Cell volumes and canonical radii of the listed cells. */
void ora_cell_info(int64_t n_cells, const double *gen, const double *vert, const int64_t *cfo,
                   const int64_t *fvo, const int32_t *fv, int64_t n_list, const int64_t *cells,
                   double *vol, float *radius) {
  tess_t T = {n_cells, gen, vert, cfo, fvo, fv};
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n_list; ++k) {
    if (vol) vol[k] = ora_cell_volume_t(&T, cells[k]);
    if (radius) radius[k] = ora_cell_radius_t(&T, cells[k]);
  }
}

/* Forward mapping of the listed cells: M_c = sum_i m_i w_ic over the
   canonical pairs in ascending particle order, rho_c = M_c / V_c.
   Also returns the number of pairs per listed cell. */
void ora_map_cells(int64_t n_cells, const double *gen, const double *vert, const int64_t *cfo,
                   const int64_t *fvo, const int32_t *fv, int64_t n_part, const double *xyz,
                   const double *h, const double *m, int64_t n_list, const int64_t *cells, double *mass,
                   double *rho, int64_t *npairs) {
  tess_t T = {n_cells, gen, vert, cfo, fvo, fv};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n_list; ++k) {
    int64_t c = cells[k];
    float R = ora_cell_radius_t(&T, c);
    const double *g = gen + 3 * c;
    double M = 0.0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n_part; ++i) {
      if (!canon_pair(xyz + 3 * i, h[i], g, R)) continue;
      M += m[i] * cell_weight(&T, c, xyz + 3 * i, h[i]);
      ++cnt;
    }
    mass[k] = M;
    rho[k] = M / ora_cell_volume_t(&T, c);
    if (npairs) npairs[k] = cnt;
  }
}

/* Coverage c_i = sum_c w_ic and inverse mapping q_i = sum_c w_ic q_c / c_i
   (q_i = 0 when c_i = 0) of the listed particles, brute force over cells.
   q (nullable): [n_cells][ncomp] cell values; out_q [n_list][ncomp]. */
void ora_particles(int64_t n_cells, const double *gen, const double *vert, const int64_t *cfo,
                   const int64_t *fvo, const int32_t *fv, int64_t n_part, const double *xyz,
                   const double *h, int64_t n_list, const int64_t *parts, const double *q, int32_t ncomp,
                   double *cov, double *out_q) {
  tess_t T = {n_cells, gen, vert, cfo, fvo, fv};
  float *R = (float *)malloc(sizeof(float) * (n_cells > 0 ? n_cells : 1));
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n_cells; ++c) R[c] = ora_cell_radius_t(&T, c);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n_list; ++k) {
    int64_t i = parts[k];
    double ci = 0.0;
    double acc[16];
    for (int j = 0; j < ncomp && j < 16; ++j) acc[j] = 0.0;
    for (int64_t c = 0; c < n_cells; ++c) {
      if (!canon_pair(xyz + 3 * i, h[i], gen + 3 * c, R[c])) continue;
      double w = cell_weight(&T, c, xyz + 3 * i, h[i]);
      ci += w;
      if (q)
        for (int j = 0; j < ncomp && j < 16; ++j) acc[j] += w * q[c * ncomp + j];
    }
    cov[k] = ci;
    if (q && out_q)
      for (int j = 0; j < ncomp && j < 16; ++j) out_q[k * ncomp + j] = ci > 0.0 ? acc[j] / ci : 0.0;
  }
  free(R);
}

/* Weight of a particle over a single convex cell given as explicit faces:
   nf faces, fsz[f] vertices each, verts concatenated [sum fsz][3];
   `inside` is a point strictly inside the cell. */
double ora_weight_poly(const double *x, double h, int nf, const int *fsz, const double *verts,
                       const double *inside) {
  int tot = 0;
  for (int f = 0; f < nf; ++f) tot += fsz[f];
  const double **fvp = (const double **)malloc(sizeof(double *) * (tot > 0 ? tot : 1));
  for (int k = 0; k < tot; ++k) fvp[k] = verts + 3 * k;
  double w = cell_weight_faces(x, h, nf, fsz, fvp, inside);
  free(fvp);
  return w;
}

/* ------------------------------------------- distance of a point to a cell */
/* Distance from x to the segment [A, B] in space. */
static double seg_dist(const double *x, const double *A, const double *B) {
  double ab[3], ax[3];
  v_sub(B, A, ab);
  v_sub(x, A, ax);
  double L2 = v_dot(ab, ab);
  double t = L2 > 0.0 ? v_dot(ax, ab) / L2 : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double d[3] = {ax[0] - t * ab[0], ax[1] - t * ab[1], ax[2] - t * ab[2]};
  return sqrt(v_dot(d, d));
}

/* Signed distance of x to cell c, the quantity that decides the exact 0/1
   shortcuts of the mapping (a kernel support of radius 2h that stays clear
   of every face gives w = 0 outside the cell and 1 inside):
     outside the cell: the distance to the nearest point of the cell
                       (positive), i.e. the smallest distance to a face
                       polygon;
     inside:           minus the distance to the nearest face plane (for a
                       convex cell that is the distance to the boundary).
   Faces are oriented outwards from the vertex-incidence average, as in the
   weight; a face polygon's distance is |d| when the foot point lies inside
   it, else the smallest edge-segment distance. */
static double cell_distance(const tess_t *T, int64_t c, const double *x) {
  int64_t f0 = T->cfo[c], f1 = T->cfo[c + 1];
  double inside[3] = {0, 0, 0};
  int64_t k = 0;
  for (int64_t t = T->fvo[f0]; t < T->fvo[f1]; ++t, ++k)
    for (int j = 0; j < 3; ++j) inside[j] += T->vert[3 * (int64_t)T->fv[t] + j];
  for (int j = 0; j < 3; ++j) inside[j] /= (k > 0 ? (double)k : 1.0);
  double smax = -HUGE_VAL, dmin = HUGE_VAL;
  for (int64_t f = f0; f < f1; ++f) {
    int nv = (int)(T->fvo[f + 1] - T->fvo[f]);
    if (nv < 3) continue;
    const double *V[512];
    if (nv > 512) continue;
    for (int q = 0; q < nv; ++q) V[q] = T->vert + 3 * (int64_t)T->fv[T->fvo[f] + q];
    double avec[3], cen[3];
    poly_area_vec(nv, V, avec, cen);
    double an = sqrt(v_dot(avec, avec));
    if (an == 0.0) continue;
    double n[3] = {avec[0] / an, avec[1] / an, avec[2] / an};
    double gc[3];
    v_sub(cen, inside, gc);
    if (v_dot(n, gc) < 0.0)
      for (int j = 0; j < 3; ++j) n[j] = -n[j];
    double xc[3];
    v_sub(x, cen, xc);
    double s = v_dot(n, xc); /* > 0: x beyond this face's plane */
    if (s > smax) smax = s;
    /* the foot point lies inside the polygon iff it is on the inner side of
       every edge line (the polygon is convex) */
    double P0[3] = {x[0] - s * n[0], x[1] - s * n[1], x[2] - s * n[2]};
    int in = 1;
    double emin = HUGE_VAL;
    for (int q = 0; q < nv; ++q) {
      const double *A = V[q], *B = V[(q + 1) % nv];
      double ab[3], ap[3], cr[3], ac[3];
      v_sub(B, A, ab);
      v_sub(P0, A, ap);
      v_sub(cen, A, ac);
      v_cross(ab, ap, cr);
      double side = v_dot(cr, n);
      v_cross(ab, ac, cr);
      double ref = v_dot(cr, n); /* the centroid's side of this edge */
      if (side * ref < 0.0) in = 0;
      double e = seg_dist(x, A, B);
      if (e < emin) emin = e;
    }
    double dp = in ? fabs(s) : emin;
    if (dp < dmin) dmin = dp;
  }
  if (smax <= 0.0) return smax; /* inside: minus the distance to the nearest plane */
  return dmin;
}

void ora_cell_distance(int64_t n_cells, const double *gen, const double *vert, const int64_t *cfo,
                       const int64_t *fvo, const int32_t *fv, int64_t n_list, const int64_t *cells,
                       const double *xyz, double *out) {
  tess_t T = {n_cells, gen, vert, cfo, fvo, fv};
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n_list; ++k) out[k] = cell_distance(&T, cells[k], xyz + 3 * k);
}

/* ----------------------------------------------- algorithmic work counts */
/* What the Exact integral of the canonical pairs of the listed cells must
   evaluate, in exact (binary64) geometry, summed over the pairs:
     out[0] pairs
     out[1] faces of the pairs' cells
     out[2] faces the support reaches (face polygon closer than 2h)
     out[3] edges of those faces
     out[4] edges the support reaches (edge segment closer than 2h)
     out[5] inner pieces, out[6] outer pieces: the part of a reached edge
            inside the support splits where U = |r - x|/h crosses 1; a part
            with U < 1 is an inner piece, one with 1 <= U < 2 an outer piece
            (a range crossing U = 1 on both sides counts one of each: the
            outer form over the whole range plus twice the difference over
            the inner stretch).
   Each face is oriented outwards as in the weight.  With nbr (the cell on
   the other side of each face, negative for a wall; nullable), a face shared
   by two cells is one polygon whose term of the weight is the same from both
   sides up to its sign, so it is counted (with its edges and pieces) only
   for the lower-numbered of its cells: the work of evaluating each
   (particle, face) once. */
void ora_work_counts(int64_t n_cells, const double *gen, const double *vert, const int64_t *cfo,
                     const int64_t *fvo, const int32_t *fv, int64_t n_part, const double *xyz,
                     const double *h, int64_t n_list, const int64_t *cells, const int32_t *nbr, int64_t *out) {
  tess_t T = {n_cells, gen, vert, cfo, fvo, fv};
  int64_t tot[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma omp parallel
  {
    int64_t loc[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < n_list; ++k) {
      int64_t c = cells[k];
      float R = ora_cell_radius_t(&T, c);
      const double *g = gen + 3 * c;
      int64_t f0 = cfo[c], f1 = cfo[c + 1];
      double inside[3] = {0, 0, 0};
      int64_t nvtot = 0;
      for (int64_t t = fvo[f0]; t < fvo[f1]; ++t, ++nvtot)
        for (int j = 0; j < 3; ++j) inside[j] += vert[3 * (int64_t)fv[t] + j];
      for (int j = 0; j < 3; ++j) inside[j] /= (nvtot > 0 ? (double)nvtot : 1.0);
      for (int64_t i = 0; i < n_part; ++i) {
        const double *x = xyz + 3 * i;
        if (!canon_pair(x, h[i], g, R)) continue;
        const double hh = h[i], r2 = 4.0 * hh * hh;
        loc[0] += 1;
        loc[1] += f1 - f0;
        for (int64_t f = f0; f < f1; ++f) {
          if (nbr && nbr[f] >= 0 && nbr[f] < c) continue; /* the other cell's */
          int nv = (int)(fvo[f + 1] - fvo[f]);
          if (nv < 3 || nv > 512) continue;
          const double *V[512];
          for (int q = 0; q < nv; ++q) V[q] = vert + 3 * (int64_t)fv[fvo[f] + q];
          double avec[3], cen[3];
          poly_area_vec(nv, V, avec, cen);
          double an = sqrt(v_dot(avec, avec));
          if (an == 0.0) continue;
          double n[3] = {avec[0] / an, avec[1] / an, avec[2] / an};
          double gc[3];
          v_sub(cen, inside, gc);
          if (v_dot(n, gc) < 0.0)
            for (int j = 0; j < 3; ++j) n[j] = -n[j];
          double xc[3];
          v_sub(x, cen, xc);
          double sd = v_dot(n, xc);
          if (sd * sd >= r2) continue; /* the plane is beyond the support */
          double P0[3] = {x[0] - sd * n[0], x[1] - sd * n[1], x[2] - sd * n[2]};
          int in = 1;
          double emin = HUGE_VAL;
          for (int q = 0; q < nv; ++q) {
            const double *A = V[q], *B = V[(q + 1) % nv];
            double ab[3], ap[3], ac[3], cr[3];
            v_sub(B, A, ab);
            v_sub(P0, A, ap);
            v_sub(cen, A, ac);
            v_cross(ab, ap, cr);
            double side = v_dot(cr, n);
            v_cross(ab, ac, cr);
            if (side * v_dot(cr, n) < 0.0) in = 0;
            double e = seg_dist(x, A, B);
            if (e < emin) emin = e;
          }
          double dp = in ? fabs(sd) : emin;
          if (dp * dp >= r2) continue; /* the face polygon is beyond the support */
          loc[2] += 1;
          for (int q = 0; q < nv; ++q) {
            const double *A = V[q], *B = V[(q + 1) % nv];
            double ab[3], ax[3];
            v_sub(B, A, ab);
            double L2 = v_dot(ab, ab);
            if (L2 == 0.0) continue;
            loc[3] += 1;
            if (seg_dist(x, A, B) >= 2.0 * hh) continue;
            loc[4] += 1;
            /* along the edge line, in units of h: U^2 = a^2 + t^2, t from
               the foot of x on the line; the segment is [ta, tb] */
            v_sub(x, A, ax);
            double L = sqrt(L2);
            double tf = v_dot(ax, ab) / L; /* foot along the edge from A */
            double a2 = (v_dot(ax, ax) - tf * tf) / (hh * hh);
            if (a2 < 0.0) a2 = 0.0;
            double ta = -tf / hh, tb = (L - tf) / hh;
            double t2 = sqrt(fmax(4.0 - a2, 0.0));
            double ca = fmin(fmax(ta, -t2), t2), cb = fmin(fmax(tb, -t2), t2);
            if (a2 < 1.0) {
              double t1 = sqrt(1.0 - a2);
              int lo = ca < -t1 && cb > -t1, hi = ca < t1 && cb > t1;
              if (lo || hi) {
                loc[5] += 1;
                loc[6] += 1;
              } else {
                double mid = 0.5 * (ca + cb);
                if (fabs(mid) < t1) loc[5] += 1;
                else loc[6] += 1;
              }
            } else {
              loc[6] += 1;
            }
          }
        }
      }
    }
#pragma omp critical
    for (int j = 0; j < 7; ++j) tot[j] += loc[j];
  }
  for (int j = 0; j < 7; ++j) out[j] = tot[j];
}

/* Angular fan integral, exposed for unit tests:
   int_{pa}^{pb} Psi_{ad}(sqrt(ad^2 + p^2 sec^2 phi)) dphi. */
double ora_fan_integral(double ad, double p, double pa, double pb) {
  return fan_integral_tau(ad, p, fabs(p) * tan(pa), fabs(p) * tan(pb));
}

/* ================================================= pseudo-particle builder */
/*
 * Sec. 2.4.1-2.4.2 with the octree variant of the gravity tree: cubic
 * subdivision of the box, leaves hold at most leaf_max particles (or sit at
 * max_depth).  Node position = centre of mass, size s = distance from the
 * centre of mass to the furthest member (Sec. 2.2.1).  Node sums are formed
 * bottom-up: a leaf sums its members in ascending particle index, an internal
 * node sums its children in octant order (x bit, then y bit, then z bit as
 * 1, 2, 4).
 *
 * Walk (Sec. 2.2.2, 2.4.1): depth first from the root.  A node is accepted
 * when for every source r - s > r_part and not (theta^2 r^2 < s^2)
 * (eq. opening_angle); an accepted node with one member is emitted as that
 * real particle, otherwise as a pseudo-particle (mass, centre of mass).  A
 * rejected leaf is opened: its members are emitted as real particles with
 * their own h (ascending index).
 *
 * Node smoothing lengths (Sec. 2.4.2): for each pseudo-particle a,
 * n(h) = sum_b W(|r_a - r_b|, h) over every emitted unit b (accepted nodes and
 * the opened leaves standing in for their particles), self term included;
 * f(h) = hfact n^(-1/3) - h, f'(h) = -(1/3) hfact n' n^(-4/3) - 1; Newton from
 * h0 = hfact 2 s until |h_new - h| / h0 < eps.  Newton fails after 30 steps,
 * when an iterate leaves [1e-2 h0, 1e2 h0] or when |f'| < 1e-12; then
 * bisection on [1e-2 h0, 1e2 h0] to a bracket below eps h0 if f changes sign
 * there, else h = h0.  Above `bypass` pseudo-particles every h = h0.
 * Branch codes: 0 Newton, 1 bisection, 2 fallback h0, 3 bypass.
 */
typedef struct {
  int64_t first;   /* first member in the tree's particle order */
  int64_t count;
  uint64_t label;  /* 1 followed by the node's octant digits, root first */
  int32_t child[8];
  int32_t is_leaf;
  double M, S[3];  /* mass and sum of m x */
  double com[3];
  double s2;       /* max squared member distance from the com */
} onode_t;

typedef struct {
  const double *x;
  const double *m;
  int leaf_max, max_depth;
  int64_t *order; /* particle order (grouped by node) */
  onode_t *nodes;
  int64_t n_nodes, cap;
} otree_t;

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

static int32_t otree_build(otree_t *T, int64_t first, int64_t count, const double lo[3], double size,
                           int depth, uint64_t label) {
  if (T->n_nodes == T->cap) {
    T->cap = T->cap * 2 + 64;
    T->nodes = (onode_t *)realloc(T->nodes, sizeof(onode_t) * T->cap);
  }
  int32_t id = (int32_t)T->n_nodes++;
  onode_t nd;
  memset(&nd, 0, sizeof nd);
  nd.first = first;
  nd.count = count;
  nd.label = label;
  for (int k = 0; k < 8; ++k) nd.child[k] = -1;
  int64_t *ord = T->order + first;
  if (count <= T->leaf_max || depth >= T->max_depth) {
    nd.is_leaf = 1;
    qsort(ord, (size_t)count, sizeof(int64_t), cmp_i64);
    for (int64_t t = 0; t < count; ++t) {
      int64_t j = ord[t];
      nd.M += T->m[j];
      for (int k = 0; k < 3; ++k) nd.S[k] += T->m[j] * T->x[3 * j + k];
    }
  } else {
    double half = 0.5 * size;
    double mid[3] = {lo[0] + half, lo[1] + half, lo[2] + half};
    /* stable partition into octants (ascending index preserved) */
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * count);
    int64_t cnt[8] = {0}, off[8];
    for (int64_t t = 0; t < count; ++t) {
      const double *p = T->x + 3 * ord[t];
      int o = (p[0] >= mid[0]) | ((p[1] >= mid[1]) << 1) | ((p[2] >= mid[2]) << 2);
      cnt[o]++;
    }
    off[0] = 0;
    for (int o = 1; o < 8; ++o) off[o] = off[o - 1] + cnt[o - 1];
    int64_t pos[8];
    memcpy(pos, off, sizeof pos);
    for (int64_t t = 0; t < count; ++t) {
      const double *p = T->x + 3 * ord[t];
      int o = (p[0] >= mid[0]) | ((p[1] >= mid[1]) << 1) | ((p[2] >= mid[2]) << 2);
      tmp[pos[o]++] = ord[t];
    }
    memcpy(ord, tmp, sizeof(int64_t) * count);
    free(tmp);
    for (int o = 0; o < 8; ++o) {
      if (!cnt[o]) continue;
      double clo[3] = {(o & 1) ? mid[0] : lo[0], (o & 2) ? mid[1] : lo[1], (o & 4) ? mid[2] : lo[2]};
      int32_t c = otree_build(T, first + off[o], cnt[o], clo, half, depth + 1, (label << 3) | (uint64_t)o);
      nd.child[o] = c;
      nd.M += T->nodes[c].M;
      for (int k = 0; k < 3; ++k) nd.S[k] += T->nodes[c].S[k];
    }
  }
  for (int k = 0; k < 3; ++k) nd.com[k] = nd.S[k] / nd.M;
  nd.s2 = 0.0;
  for (int64_t t = 0; t < count; ++t) {
    const double *p = T->x + 3 * ord[t];
    double dx = p[0] - nd.com[0], dy = p[1] - nd.com[1], dz = p[2] - nd.com[2];
    double s = (dx * dx + dy * dy) + dz * dz;
    if (s > nd.s2) nd.s2 = s;
  }
  T->nodes[id] = nd;
  return id;
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

/* label in the sorted list of nodes to open (Sec. 2.4.1: nodes that failed
   the resolution check are opened in the next walk) */
static int forced_open(uint64_t label, int64_t n_open, const uint64_t *open_sorted) {
  return n_open > 0 && bsearch(&label, open_sorted, (size_t)n_open, sizeof(uint64_t), cmp_u64) != NULL;
}

static int accepted(const onode_t *nd, int n_src, const double *src, double r_part, double theta) {
  double s = sqrt(nd->s2);
  for (int k = 0; k < n_src; ++k) {
    double dx = nd->com[0] - src[3 * k], dy = nd->com[1] - src[3 * k + 1], dz = nd->com[2] - src[3 * k + 2];
    double r2 = (dx * dx + dy * dy) + dz * dz;
    double r = sqrt(r2);
    if (!(r - s > r_part)) return 0;
    if ((theta * theta) * r2 < nd->s2) return 0;
  }
  return 1;
}

typedef struct {
  int64_t n;
  int64_t n_open;
  const uint64_t *open;  /* sorted labels of nodes to open */
  uint64_t *label;  /* node label of the entry's unit */
  int32_t *kind;    /* 0 real particle, 1 pseudo-particle */
  int64_t *first;   /* lowest member particle index */
  int64_t *count;   /* members */
  double *pos;      /* [][3] */
  double *mass, *h, *s;
  int32_t *unit;    /* h-solve unit of the entry */
  int64_t *owner;   /* [n particles] entry that holds the particle */
  /* h-solve units: accepted nodes and opened leaves */
  int64_t n_units;
  double *upos;     /* [][3] */
} emit_t;

static void walk(const otree_t *T, int32_t id, int n_src, const double *src, double r_part, double theta,
                 const double *hp, emit_t *E) {
  const onode_t *nd = &T->nodes[id];
  if (accepted(nd, n_src, src, r_part, theta) && !forced_open(nd->label, E->n_open, E->open)) {
    int64_t u = E->n_units++;
    for (int k = 0; k < 3; ++k) E->upos[3 * u + k] = nd->com[k];
    int64_t e = E->n++;
    E->unit[e] = (int32_t)u;
    E->label[e] = nd->label;
    E->count[e] = nd->count;
    for (int64_t t = 0; t < nd->count; ++t) E->owner[T->order[nd->first + t]] = e;
    if (nd->count == 1) {
      int64_t j = T->order[nd->first];
      E->kind[e] = 0;
      E->first[e] = j;
      for (int k = 0; k < 3; ++k) E->pos[3 * e + k] = T->x[3 * j + k];
      E->mass[e] = T->m[j];
      E->h[e] = hp[j];
      E->s[e] = 0.0;
    } else {
      int64_t mn = T->order[nd->first];
      for (int64_t t = 1; t < nd->count; ++t)
        if (T->order[nd->first + t] < mn) mn = T->order[nd->first + t];
      E->kind[e] = 1;
      E->first[e] = mn;
      for (int k = 0; k < 3; ++k) E->pos[3 * e + k] = nd->com[k];
      E->mass[e] = nd->M;
      E->h[e] = 0.0;
      E->s[e] = sqrt(nd->s2);
    }
    return;
  }
  if (nd->is_leaf) {
    int64_t u = E->n_units++;
    for (int k = 0; k < 3; ++k) E->upos[3 * u + k] = nd->com[k];
    for (int64_t t = 0; t < nd->count; ++t) { /* members are in ascending index */
      int64_t j = T->order[nd->first + t];
      int64_t e = E->n++;
      E->unit[e] = (int32_t)u;
      E->label[e] = nd->label;
      E->owner[j] = e;
      E->kind[e] = 0;
      E->first[e] = j;
      E->count[e] = 1;
      for (int k = 0; k < 3; ++k) E->pos[3 * e + k] = T->x[3 * j + k];
      E->mass[e] = T->m[j];
      E->h[e] = hp[j];
      E->s[e] = 0.0;
    }
    return;
  }
  for (int o = 0; o < 8; ++o)
    if (nd->child[o] >= 0) walk(T, nd->child[o], n_src, src, r_part, theta, hp, E);
}

/* n(h) and dn/dh at node position a over the units */
static void node_sums(const double *a, double h, int64_t nu, const double *upos, double *n, double *dn) {
  double sw = 0.0, sd = 0.0, ih = 1.0 / h;
  for (int64_t b = 0; b < nu; ++b) {
    double dx = a[0] - upos[3 * b], dy = a[1] - upos[3 * b + 1], dz = a[2] - upos[3 * b + 2];
    double q = sqrt((dx * dx + dy * dy) + dz * dz) * ih;
    if (q >= 2.0) continue;
    double w = ora_w(q);
    sw += w;
    sd += -(3.0 * w + q * ora_dw(q));
  }
  *n = sw * ih * ih * ih / M_PI;
  *dn = sd * ih * ih * ih * ih / M_PI;
}

static double hfun(const double *a, double h, int64_t nu, const double *upos, double hfact) {
  double n, dn;
  node_sums(a, h, nu, upos, &n, &dn);
  return hfact * pow(n, -1.0 / 3.0) - h;
}

/* The node h-solve for one pseudo-particle; returns the branch code. */
int ora_node_h(const double *a, double s, int64_t nu, const double *upos, double hfact, double eps,
               double *h_out, int *iters) {
  double h0 = hfact * 2.0 * s;
  double lo = 1e-2 * h0, hi = 1e2 * h0;
  double h = h0;
  int it;
  for (it = 0; it < 30; ++it) {
    double n, dn;
    node_sums(a, h, nu, upos, &n, &dn);
    double f = hfact * pow(n, -1.0 / 3.0) - h;
    double fp = -(1.0 / 3.0) * hfact * dn * pow(n, -4.0 / 3.0) - 1.0;
    if (!(fabs(fp) >= 1e-12)) break;
    double hn = h - f / fp;
    if (!(hn >= lo && hn <= hi)) break;
    if (fabs(hn - h) / h0 < eps) {
      *h_out = hn;
      if (iters) *iters = it + 1;
      return 0;
    }
    h = hn;
  }
  if (iters) *iters = it;
  double flo = hfun(a, lo, nu, upos, hfact), fhi = hfun(a, hi, nu, upos, hfact);
  if (flo == 0.0) {
    *h_out = lo;
    return 1;
  }
  if (fhi == 0.0) {
    *h_out = hi;
    return 1;
  }
  if ((flo < 0.0) == (fhi < 0.0)) {
    *h_out = h0;
    return 2;
  }
  while (hi - lo >= eps * h0) {
    double mid = 0.5 * (lo + hi);
    double fm = hfun(a, mid, nu, upos, hfact);
    if (fm == 0.0) {
      *h_out = mid;
      return 1;
    }
    if ((fm < 0.0) == (flo < 0.0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  *h_out = 0.5 * (lo + hi);
  return 1;
}

/* Full builder.  Outputs (capacity n entries each; pos [n][3]):
   kind, first (lowest member index), count, pos, mass, h, s (node size),
   branch (-1 for real particles), unit (h-solve unit of the entry), label
   (node label of the entry's unit: a 1 followed by the octant digits from
   the root down, 3 bits per level), owner ([n]: the entry that holds each
   particle, itself or its pseudo-particle).  Nodes whose labels are among the
   n_open labels in open (any order) are opened whatever the walk criterion
   says.  Returns the number of emitted entries; *n_units_out = number of
   units, upos_out (capacity n*3) their positions; *n_nodes_out = tree size;
   *s_root_out = size of the root node. */
int64_t ora_pseudo_build(int64_t n, const double *x, const double *m, const double *hp, int32_t n_src,
                         const double *src, double r_part, double theta, double hfact, double eps,
                         int32_t leaf_max, int32_t max_depth, int64_t bypass, int64_t n_open, const uint64_t *open,
                         int32_t *kind, int64_t *first, int64_t *count, double *pos, double *mass, double *h,
                         double *s, int32_t *branch, int32_t *unit, uint64_t *label, int64_t *owner,
                         int64_t *n_units_out, double *upos_out, int64_t *n_nodes_out, double *s_root_out) {
  otree_t T;
  T.x = x;
  T.m = m;
  T.leaf_max = leaf_max;
  T.max_depth = max_depth;
  T.order = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) T.order[i] = i;
  T.nodes = NULL;
  T.n_nodes = T.cap = 0;
  double lo[3] = {0.0, 0.0, 0.0};
  otree_build(&T, 0, n, lo, 1.0, 0, 1);
  uint64_t *open_sorted = (uint64_t *)malloc(sizeof(uint64_t) * (n_open > 0 ? n_open : 1));
  if (n_open > 0) memcpy(open_sorted, open, sizeof(uint64_t) * n_open);
  qsort(open_sorted, (size_t)n_open, sizeof(uint64_t), cmp_u64);
  emit_t E;
  E.n = 0;
  E.n_open = n_open;
  E.open = open_sorted;
  E.label = label;
  E.kind = kind;
  E.first = first;
  E.count = count;
  E.pos = pos;
  E.mass = mass;
  E.h = h;
  E.s = s;
  E.unit = unit;
  E.owner = owner;
  E.n_units = 0;
  E.upos = upos_out;
  walk(&T, 0, n_src, src, r_part, theta, hp, &E);
  int64_t n_pseudo = 0;
  for (int64_t e = 0; e < E.n; ++e) n_pseudo += kind[e] == 1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t e = 0; e < E.n; ++e) {
    if (kind[e] != 1) {
      branch[e] = -1;
      continue;
    }
    if (n_pseudo > bypass) {
      h[e] = hfact * 2.0 * s[e];
      branch[e] = 3;
      continue;
    }
    branch[e] = ora_node_h(pos + 3 * e, s[e], E.n_units, E.upos, hfact, eps, &h[e], NULL);
  }
  *n_units_out = E.n_units;
  *n_nodes_out = T.n_nodes;
  *s_root_out = n > 0 ? sqrt(T.nodes[0].s2) : 0.0;
  free(open_sorted);
  free(T.order);
  free(T.nodes);
  return E.n;
}

/* Resolution parameter (eq. resol_param): the neutral-fraction threshold of a
   node of size s_node, f_neu,limit = (1/K) (K - 1 / (s_node / s_root)). */
double ora_fneu_limit(double s_ratio, double K) { return (K - 1.0 / s_ratio) / K; }

/* Pseudo-particles whose neutral fraction is below the threshold of their
   size (under-resolved, Sec. 2.4.1): their labels, in entry order.  Real
   particles are never checked.  Returns the count. */
int64_t ora_underresolved(int64_t n, const int32_t *kind, const uint64_t *label, const double *s,
                          const double *fneu, double s_root, double K, uint64_t *out) {
  int64_t k = 0;
  for (int64_t e = 0; e < n; ++e)
    if (kind[e] == 1 && fneu[e] < ora_fneu_limit(s[e] / s_root, K)) out[k++] = label[e];
  return k;
}

/* Per-particle values from the mixed set (Sec. 3.3: the paper proposes
   interpolating each SPH particle's ionic fraction from the pseudo-particles
   whose smoothing spheres reach it, instead of giving every member its node's
   value).  Reading: the SPH interpolant over the entries, each entry j with
   the volume its smoothing length stands for, V_j = (h_j / h_fact)^3 (the
   h-density relation of eq. h_node for pseudo-particles, and of the SPH
   particles themselves), normalised by the same sum (Shepard):
     q_i = sum_j V_j W(|x_i - x_j|, h_j) q_j / sum_j V_j W(|x_i - x_j|, h_j)
         = sum_j w(r_ij / h_j) q_j / sum_j w(r_ij / h_j)
   over the entries with |x_i - x_j| < 2 h_j (the h^3 and h_fact cancel; w
   is the dimensionless M4 kernel).  A particle that is an entry itself keeps
   that entry's value, one that no sphere reaches its owner's value.  Plain
   O(n E) loop, entries in index order.  values and out are [][ncomp]. */
void ora_interpolate(int64_t n, const double *x, const int64_t *owner, int64_t ne, const double *ex,
                     const double *eh, const int32_t *ekind, const double *val, int32_t ncomp, double *out) {
  if (ncomp < 1 || ncomp > 16) return; /* the per-particle sums hold at most 16 components */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = owner[i];
    double *oi = out + (int64_t)ncomp * i;
    if (ekind[o] == 0) {
      for (int k = 0; k < ncomp; ++k) oi[k] = val[(int64_t)ncomp * o + k];
      continue;
    }
    double den = 0.0;
    double num[16];
    for (int k = 0; k < ncomp; ++k) num[k] = 0.0;
    for (int64_t j = 0; j < ne; ++j) {
      const double dx = x[3 * i] - ex[3 * j], dy = x[3 * i + 1] - ex[3 * j + 1], dz = x[3 * i + 2] - ex[3 * j + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double hj = eh[j];
      if (!(r < 2.0 * hj)) continue;
      const double W = ora_w(r / hj);
      den += W;
      for (int k = 0; k < ncomp; ++k) num[k] += W * val[(int64_t)ncomp * j + k];
    }
    for (int k = 0; k < ncomp; ++k) oi[k] = den > 0.0 ? num[k] / den : val[(int64_t)ncomp * o + k];
  }
}

/* ------------------------------------------------------------------ Voronoi
   The grid the mapping runs on (Sec. 2.3): the Voronoi cell of generator c
   inside the box [lo, hi] is the set of box points at least as close to g_c
   as to any other generator.  Built the textbook way: start from the box as
   six square faces and cut it by the bisector half-space of every other
   generator in turn (n.x <= d with n = g_j - g_c, d = (|g_j|^2 - |g_c|^2) / 2),
   clipping each face polygon against the plane and closing the cut with a
   cap face whose points are ordered by angle about their mean.  Face ids:
   the neighbouring generator, or -1..-6 for the box planes x-, x+, y-, y+,
   z-, z+.  Volume and centroid by the fan of tetrahedra (g_c, v0, v_i,
   v_i+1) over each face. */

typedef struct {
  int nv, cap;
  double *v; /* [cap][3] */
  int64_t id;
} opoly_t;

typedef struct {
  int nf, cap;
  opoly_t *f;
} ocell_t;

static void opoly_push(opoly_t *p, const double *x) {
  if (p->nv == p->cap) {
    p->cap = p->cap ? 2 * p->cap : 8;
    p->v = (double *)realloc(p->v, sizeof(double) * 3 * p->cap);
  }
  memcpy(p->v + 3 * p->nv, x, sizeof(double) * 3);
  p->nv++;
}

static opoly_t *ocell_add(ocell_t *C, int64_t id) {
  if (C->nf == C->cap) {
    C->cap = C->cap ? 2 * C->cap : 16;
    C->f = (opoly_t *)realloc(C->f, sizeof(opoly_t) * C->cap);
  }
  opoly_t *p = &C->f[C->nf++];
  p->nv = p->cap = 0;
  p->v = NULL;
  p->id = id;
  return p;
}

static void ocell_free(ocell_t *C) {
  for (int k = 0; k < C->nf; ++k) free(C->f[k].v);
  free(C->f);
  C->f = NULL;
  C->nf = C->cap = 0;
}

static void ocell_box(ocell_t *C, const double *lo, const double *hi) {
  /* corner (i, j, k) with bits x = 1, y = 2, z = 4 */
  static const int quad[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
  C->nf = C->cap = 0;
  C->f = NULL;
  for (int s = 0; s < 6; ++s) {
    opoly_t *p = ocell_add(C, -1 - s);
    for (int q = 0; q < 4; ++q) {
      const int b = quad[s][q];
      double x[3] = {(b & 1) ? hi[0] : lo[0], (b & 2) ? hi[1] : lo[1], (b & 4) ? hi[2] : lo[2]};
      opoly_push(p, x);
    }
  }
}

/* keep n.x <= d (n unit); returns 1 when a vertex lay beyond eps */
static int ocell_clip(ocell_t *C, const double *n, double d, int64_t id, double eps) {
  opoly_t cap = {0, 0, NULL, id};
  int cut = 0;
  for (int k = 0; k < C->nf; ++k)
    for (int i = 0; i < C->f[k].nv; ++i)
      if (v_dot(n, C->f[k].v + 3 * i) - d > eps) cut = 1;
  if (!cut) return 0;
  int w = 0;
  for (int k = 0; k < C->nf; ++k) {
    opoly_t *f = &C->f[k];
    opoly_t out = {0, 0, NULL, f->id};
    for (int i = 0; i < f->nv; ++i) {
      const double *a = f->v + 3 * i, *b = f->v + 3 * ((i + 1) % f->nv);
      const double sa = v_dot(n, a) - d, sb = v_dot(n, b) - d;
      if (sa <= eps) {
        opoly_push(&out, a);
        if (sa >= -eps) opoly_push(&cap, a);
      }
      if ((sa < -eps && sb > eps) || (sa > eps && sb < -eps)) {
        const double t = sa / (sa - sb);
        double x[3] = {a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1]), a[2] + t * (b[2] - a[2])};
        opoly_push(&out, x);
        opoly_push(&cap, x);
      }
    }
    free(f->v);
    if (out.nv >= 3)
      C->f[w++] = out;
    else
      free(out.v);
  }
  C->nf = w;
  /* cap: distinct points ordered by angle about their mean */
  opoly_t uq = {0, 0, NULL, id};
  for (int i = 0; i < cap.nv; ++i) {
    int dup = 0;
    for (int j = 0; j < uq.nv && !dup; ++j) {
      double e[3];
      v_sub(cap.v + 3 * i, uq.v + 3 * j, e);
      dup = v_dot(e, e) <= 100.0 * eps * eps;
    }
    if (!dup) opoly_push(&uq, cap.v + 3 * i);
  }
  free(cap.v);
  if (uq.nv >= 3) {
    double m[3] = {0, 0, 0}, u[3], t[3], ww[3];
    for (int i = 0; i < uq.nv; ++i)
      for (int q = 0; q < 3; ++q) m[q] += uq.v[3 * i + q] / uq.nv;
    t[0] = fabs(n[0]) < 0.9 ? 1.0 : 0.0;
    t[1] = fabs(n[0]) < 0.9 ? 0.0 : 1.0;
    t[2] = 0.0;
    v_cross(n, t, u);
    const double lu = sqrt(v_dot(u, u));
    for (int q = 0; q < 3; ++q) u[q] /= lu;
    v_cross(n, u, ww);
    double *ang = (double *)malloc(sizeof(double) * uq.nv);
    for (int i = 0; i < uq.nv; ++i) {
      double e[3];
      v_sub(uq.v + 3 * i, m, e);
      ang[i] = atan2(v_dot(e, ww), v_dot(e, u));
    }
    for (int i = 1; i < uq.nv; ++i) /* insertion sort by angle */
      for (int j = i; j > 0 && ang[j] < ang[j - 1]; --j) {
        double ta = ang[j];
        ang[j] = ang[j - 1];
        ang[j - 1] = ta;
        double tv[3];
        memcpy(tv, uq.v + 3 * j, sizeof tv);
        memcpy(uq.v + 3 * j, uq.v + 3 * (j - 1), sizeof tv);
        memcpy(uq.v + 3 * (j - 1), tv, sizeof tv);
      }
    free(ang);
    opoly_t *p = ocell_add(C, id);
    *p = uq;
  } else {
    free(uq.v);
  }
  return 1;
}

static void ocell_build(int64_t n, const double *g, int64_t c, const double *lo, const double *hi, ocell_t *C) {
  ocell_box(C, lo, hi);
  const double L = fmax(hi[0] - lo[0], fmax(hi[1] - lo[1], hi[2] - lo[2]));
  const double eps = 1e-13 * L;
  const double *gc = g + 3 * c;
  double rmax = -1.0; /* largest vertex distance from g_c, refreshed after a cut */
  for (int64_t j = 0; j < n; ++j) {
    if (j == c) continue;
    if (rmax < 0.0) {
      double r2 = 0.0;
      for (int k = 0; k < C->nf; ++k)
        for (int i = 0; i < C->f[k].nv; ++i) {
          double e[3];
          v_sub(C->f[k].v + 3 * i, gc, e);
          r2 = fmax(r2, v_dot(e, e));
        }
      rmax = sqrt(r2);
    }
    double nv[3];
    v_sub(g + 3 * j, gc, nv);
    const double dist = sqrt(v_dot(nv, nv));
    /* the bisector is dist/2 from g_c: it cannot cut when every vertex is closer */
    if (0.5 * dist > rmax + eps) continue;
    for (int q = 0; q < 3; ++q) nv[q] /= dist;
    double mid[3] = {0.5 * (g[3 * j] + gc[0]), 0.5 * (g[3 * j + 1] + gc[1]), 0.5 * (g[3 * j + 2] + gc[2])};
    if (ocell_clip(C, nv, v_dot(nv, mid), j, eps)) rmax = -1.0;
  }
}

static void ocell_moments(const ocell_t *C, const double *gc, double *vol, double *cen) {
  double V = 0.0, S[3] = {0, 0, 0};
  for (int k = 0; k < C->nf; ++k) {
    const opoly_t *f = &C->f[k];
    for (int i = 1; i + 1 < f->nv; ++i) {
      double a[3], b[3], c[3], x[3];
      v_sub(f->v, gc, a);
      v_sub(f->v + 3 * i, gc, b);
      v_sub(f->v + 3 * (i + 1), gc, c);
      v_cross(b, c, x);
      const double t = fabs(v_dot(a, x)) / 6.0;
      V += t;
      for (int q = 0; q < 3; ++q) S[q] += t * (a[q] + b[q] + c[q]) / 4.0;
    }
  }
  *vol = V;
  for (int q = 0; q < 3; ++q) cen[q] = gc[q] + (V > 0.0 ? S[q] / V : 0.0);
}

/* Cells of all generators.  Per cell: volume, centroid [3]; faces as a CSR
   (cell_face_off [n+1]) with the face id, its area and its polygon
   (face_vtx_off [F+1] into face_pts [][3]).  Pass NULL for the face arrays
   to get only the counts: *n_faces_out, *n_fv_out.  Returns 0. */
int ora_voronoi(int64_t n, const double *g, const double *lo, const double *hi, double *volume, double *centroid,
                int64_t *cell_face_off, int64_t *face_id, double *face_area, int64_t *face_vtx_off,
                double *face_pts, int64_t *n_faces_out, int64_t *n_fv_out) {
  int64_t *nf = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t *nfv = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t c = 0; c < n; ++c) {
    ocell_t C;
    ocell_build(n, g, c, lo, hi, &C);
    ocell_moments(&C, g + 3 * c, &volume[c], centroid + 3 * c);
    nf[c] = C.nf;
    for (int k = 0; k < C.nf; ++k) nfv[c] += C.f[k].nv;
    ocell_free(&C);
  }
  int64_t F = 0, FV = 0;
  for (int64_t c = 0; c < n; ++c) {
    int64_t a = nf[c], b = nfv[c];
    nf[c] = F;
    nfv[c] = FV;
    F += a;
    FV += b;
  }
  *n_faces_out = F;
  *n_fv_out = FV;
  if (cell_face_off) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t c = 0; c < n; ++c) {
      ocell_t C;
      ocell_build(n, g, c, lo, hi, &C);
      int64_t f0 = nf[c], p0 = nfv[c];
      cell_face_off[c] = f0;
      for (int k = 0; k < C.nf; ++k) {
        const opoly_t *f = &C.f[k];
        face_id[f0 + k] = f->id;
        face_vtx_off[f0 + k] = p0;
        double A[3] = {0, 0, 0};
        for (int i = 1; i + 1 < f->nv; ++i) {
          double a[3], b[3], x[3];
          v_sub(f->v + 3 * i, f->v, a);
          v_sub(f->v + 3 * (i + 1), f->v, b);
          v_cross(a, b, x);
          for (int q = 0; q < 3; ++q) A[q] += x[q];
        }
        face_area[f0 + k] = 0.5 * sqrt(v_dot(A, A));
        memcpy(face_pts + 3 * p0, f->v, sizeof(double) * 3 * f->nv);
        p0 += f->nv;
      }
      ocell_free(&C);
    }
    cell_face_off[n] = F;
    face_vtx_off[F] = FV;
  }
  free(nf);
  free(nfv);
  return 0;
}

/* Lloyd's iteration (Sec. 2.3): every generator moves to the centroid of its
   cell, iters times.  out [n][3] receives the final generators. */
void ora_lloyd(int64_t n, const double *g, const double *lo, const double *hi, int32_t iters, double *out) {
  double *cur = (double *)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
  memcpy(cur, g, sizeof(double) * 3 * n);
  for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t c = 0; c < n; ++c) {
      ocell_t C;
      double v;
      ocell_build(n, cur, c, lo, hi, &C);
      ocell_moments(&C, cur + 3 * c, &v, out + 3 * c);
      ocell_free(&C);
    }
    memcpy(cur, out, sizeof(double) * 3 * n);
  }
  if (iters <= 0) memcpy(out, g, sizeof(double) * 3 * n);
  free(cur);
}

/* Volume and centroid of the cells listed in cells[m] only (same
   construction as ora_voronoi). */
void ora_voronoi_cells(int64_t n, const double *g, const double *lo, const double *hi, int64_t m,
                       const int64_t *cells, double *volume, double *centroid) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t k = 0; k < m; ++k) {
    ocell_t C;
    ocell_build(n, g, cells[k], lo, hi, &C);
    ocell_moments(&C, g + 3 * cells[k], &volume[k], centroid + 3 * k);
    ocell_free(&C);
  }
}

/* ------------------------------------------------------------- k-d tree
   The paper's own tree (Sec. 2.2.1): a binary k-d tree built top down by
   recursive coordinate bisection.  A node's domain (the root's is the unit
   cube) is split in two through the centre of mass of its particles along
   the domain's longest axis (the first such axis on a tie); particles below
   the split coordinate go left.  Splitting stops when a node holds fewer
   than leaf_split particles (10 in the paper), at max_depth, or when a split
   would leave one side empty.  Labels: root 1, children of n are 2n (left)
   and 2n + 1 (right), so a node of label n lies on level floor(log2 n) and
   its ancestor on level k is n >> (level - k).
   Centres of mass are order-free: each m_i and m_i x_i is rounded to a
   fixed-point integer of 2^-K (K such that every node sum stays below 2^62,
   from n and the largest mass) and the integer sums are exact, so the
   split planes do not depend on summation order.  Node mass = its integer
   sum times 2^-K; size s = largest member distance from the centre of mass.

   Walk (Sec. 2.4.1), depth first, left before right; per source, with
   r = |com - source|: the node reaches r_part when r - s <= r_part, reaches
   r_leaf when r - s <= r_leaf, and fails the opening angle when
   theta^2 r^2 < s^2 (eq. opening_angle).  A node is accepted when it does
   none of these for any source and is not named in open; an accepted node
   is emitted (as itself when it has one particle).  A leaf that is not
   accepted is emitted as its particles (own h) when it reaches r_part, is
   named in open or holds one particle, and otherwise as a leaf
   pseudo-particle (leaves in the annulus between r_part and r_leaf, and
   leaves that fail the opening angle further out).

   Node smoothing lengths: the iteration of eqs. hnode_func to
   hnode_estval (ora_node_h) over the emitted units (accepted nodes and
   leaves).  With more than nf_threshold units the sums run over the trial
   neighbours of the neighbour-find of Sec. 2.4.3 instead of all units:
   k_mid is the level just above the highest unit; for a target a, r_cut is
   sqrt(3) times the size of a's ancestor on k_mid, or, when that is below
   r_2h = 4 h_fact s_a (eq. compact_support_radius), 4 h_fact times the size
   of a's ancestor up_levels above a; the k_mid nodes whose centres of mass
   lie within r_cut of a are flagged, and the trial neighbours are the units
   (in unit order) whose k_mid ancestor is flagged. */

typedef struct {
  uint64_t label;
  int32_t level, parent, left, right;
  int64_t first, count;
  double lo[3], hi[3];
  double com[3], M, s2;
} kdnode_t;

typedef struct {
  const double *x, *m;
  int leaf_split, max_depth, K;
  int64_t *order, *tmp;
  kdnode_t *nodes;
  int64_t n_nodes, cap;
} kdtree_t;

static int kd_scale(int64_t n, const double *m) {
  double mmax = 0.0;
  for (int64_t i = 0; i < n; ++i) mmax = fmax(mmax, m[i]);
  int e = 0;
  frexp((double)n * mmax, &e);
  return 62 - e;
}

static int32_t kd_build(kdtree_t *T, int64_t first, int64_t count, const double lo[3], const double hi[3],
                        int level, uint64_t label, int32_t parent) {
  if (T->n_nodes == T->cap) {
    T->cap = T->cap ? 2 * T->cap : 1024;
    T->nodes = (kdnode_t *)realloc(T->nodes, sizeof(kdnode_t) * T->cap);
  }
  const int32_t id = (int32_t)T->n_nodes++;
  kdnode_t nd;
  nd.label = label;
  nd.level = level;
  nd.parent = parent;
  nd.left = nd.right = -1;
  nd.first = first;
  nd.count = count;
  memcpy(nd.lo, lo, sizeof nd.lo);
  memcpy(nd.hi, hi, sizeof nd.hi);
  int64_t qm = 0, qx[3] = {0, 0, 0};
  for (int64_t t = 0; t < count; ++t) {
    const int64_t j = T->order[first + t];
    qm += llrint(ldexp(T->m[j], T->K));
    for (int k = 0; k < 3; ++k) qx[k] += llrint(ldexp(T->m[j] * T->x[3 * j + k], T->K));
  }
  for (int k = 0; k < 3; ++k) nd.com[k] = (double)qx[k] / (double)qm;
  nd.M = ldexp((double)qm, -T->K);
  nd.s2 = 0.0;
  for (int64_t t = 0; t < count; ++t) {
    const int64_t j = T->order[first + t];
    double e[3];
    v_sub(T->x + 3 * j, nd.com, e);
    nd.s2 = fmax(nd.s2, v_dot(e, e));
  }
  T->nodes[id] = nd;
  if (count < T->leaf_split || level >= T->max_depth) return id;
  int axis = 0;
  for (int k = 1; k < 3; ++k)
    if (hi[k] - lo[k] > hi[axis] - lo[axis]) axis = k;
  const double split = nd.com[axis];
  int64_t nl = 0, nr = 0;
  for (int64_t t = 0; t < count; ++t) {
    const int64_t j = T->order[first + t];
    if (T->x[3 * j + axis] < split) T->order[first + nl++] = j; else T->tmp[nr++] = j;
  }
  memcpy(T->order + first + nl, T->tmp, sizeof(int64_t) * nr);
  if (nl == 0 || nr == 0) return id;
  double llo[3], lhi[3], rlo[3], rhi[3];
  memcpy(llo, lo, sizeof llo);
  memcpy(lhi, hi, sizeof lhi);
  memcpy(rlo, lo, sizeof rlo);
  memcpy(rhi, hi, sizeof rhi);
  lhi[axis] = split;
  rlo[axis] = split;
  const int32_t l = kd_build(T, first, nl, llo, lhi, level + 1, 2 * label, id);
  const int32_t r = kd_build(T, first + nl, nr, rlo, rhi, level + 1, 2 * label + 1, id);
  T->nodes[id].left = l;
  T->nodes[id].right = r;
  return id;
}

typedef struct {
  int n_src;
  const double *src;
  double r_part, r_leaf, theta;
  int64_t n_open;
  const uint64_t *open;
  int64_t n, n_units;
  int32_t *kind, *unit_node, *entry_node;
  int64_t *first, *count, *owner;
  double *pos, *mass, *s;
  uint64_t *label;
  const double *hp;
} kdemit_t;

static void kd_walk(const kdtree_t *T, int32_t id, kdemit_t *E) {
  const kdnode_t *nd = &T->nodes[id];
  const double s = sqrt(nd->s2);
  int part = 0, leafz = 0, angle = 0;
  for (int k = 0; k < E->n_src; ++k) {
    double e[3];
    v_sub(nd->com, E->src + 3 * k, e);
    const double r = sqrt(v_dot(e, e));
    if (r - s <= E->r_part) part = 1;
    if (r - s <= E->r_leaf) leafz = 1;
    if (E->theta * E->theta * r * r < nd->s2) angle = 1;
  }
  const int forced = forced_open(nd->label, E->n_open, E->open);
  const int leaf = nd->left < 0;
  const int accepted = !(part || leafz || angle || forced);
  if (!accepted && !leaf) {
    kd_walk(T, nd->left, E);
    kd_walk(T, nd->right, E);
    return;
  }
  const int64_t u = E->n_units++;
  E->unit_node[u] = id;
  if (nd->count == 1 || (!accepted && (part || forced))) {
    for (int64_t t = 0; t < nd->count; ++t) { /* members are in ascending index */
      const int64_t j = T->order[nd->first + t];
      const int64_t e = E->n++;
      E->kind[e] = 0;
      E->first[e] = j;
      E->count[e] = 1;
      for (int k = 0; k < 3; ++k) E->pos[3 * e + k] = T->x[3 * j + k];
      E->mass[e] = T->m[j];
      E->s[e] = 0.0;
      E->label[e] = nd->label;
      E->entry_node[e] = id;
      E->owner[j] = e;
    }
    return;
  }
  const int64_t e = E->n++;
  E->kind[e] = 1;
  E->first[e] = T->order[nd->first];
  E->count[e] = nd->count;
  for (int k = 0; k < 3; ++k) E->pos[3 * e + k] = nd->com[k];
  E->mass[e] = nd->M;
  E->s[e] = s;
  E->label[e] = nd->label;
  E->entry_node[e] = id;
  for (int64_t t = 0; t < nd->count; ++t) E->owner[T->order[nd->first + t]] = e;
}

static int32_t kd_ancestor(const kdtree_t *T, int32_t id, int level) {
  while (id >= 0 && T->nodes[id].level > level) id = T->nodes[id].parent;
  return id;
}

/* Full k-d builder.  Outputs as ora_pseudo_build (capacity n entries), plus
   level of each entry's node; returns the entry count.  stats_out[4]:
   nodes, units, k_mid (-1: all units summed), pseudo-particles. */
int64_t ora_kd_build(int64_t n, const double *x, const double *m, const double *hp, int32_t n_src,
                     const double *src, double r_part, double r_leaf, double theta, double hfact, double eps,
                     int32_t leaf_split, int32_t max_depth, int64_t nf_threshold, int32_t up_levels,
                     int64_t bypass, int64_t n_open, const uint64_t *open, int32_t *kind, int64_t *first,
                     int64_t *count, double *pos, double *mass, double *h, double *s, int32_t *branch,
                     uint64_t *label, int32_t *level, int64_t *owner, int64_t *stats_out, double *s_root_out) {
  kdtree_t T;
  T.x = x;
  T.m = m;
  T.leaf_split = leaf_split;
  T.max_depth = max_depth;
  T.K = kd_scale(n, m);
  T.order = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  T.tmp = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) T.order[i] = i;
  T.nodes = NULL;
  T.n_nodes = T.cap = 0;
  const double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {1.0, 1.0, 1.0};
  kd_build(&T, 0, n, lo, hi, 0, 1, -1);
  uint64_t *open_sorted = (uint64_t *)malloc(sizeof(uint64_t) * (n_open > 0 ? n_open : 1));
  if (n_open > 0) memcpy(open_sorted, open, sizeof(uint64_t) * n_open);
  qsort(open_sorted, (size_t)n_open, sizeof(uint64_t), cmp_u64);
  kdemit_t E;
  E.n_src = n_src;
  E.src = src;
  E.r_part = r_part;
  E.r_leaf = r_leaf;
  E.theta = theta;
  E.n_open = n_open;
  E.open = open_sorted;
  E.n = E.n_units = 0;
  E.kind = kind;
  E.first = first;
  E.count = count;
  E.pos = pos;
  E.mass = mass;
  E.s = s;
  E.label = label;
  E.owner = owner;
  E.hp = hp;
  E.unit_node = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  E.entry_node = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  kd_walk(&T, 0, &E);
  const int64_t nu = E.n_units;
  double *upos = (double *)malloc(sizeof(double) * 3 * (nu > 0 ? nu : 1));
  int kmin = 1 << 30;
  for (int64_t u = 0; u < nu; ++u) {
    const kdnode_t *nd = &T.nodes[E.unit_node[u]];
    memcpy(upos + 3 * u, nd->com, sizeof(double) * 3);
    if (nd->level < kmin) kmin = nd->level;
  }
  const int use_nf = nu > nf_threshold;
  const int kmid = use_nf ? (kmin > 0 ? kmin - 1 : 0) : -1;
  int64_t n_pseudo = 0;
  for (int64_t e = 0; e < E.n; ++e) {
    level[e] = T.nodes[E.entry_node[e]].level;
    if (kind[e] == 0) h[e] = hp[first[e]];
    n_pseudo += kind[e] == 1;
  }
  /* k_mid ancestor of every unit */
  int32_t *umid = (int32_t *)malloc(sizeof(int32_t) * (nu > 0 ? nu : 1));
  if (use_nf)
    for (int64_t u = 0; u < nu; ++u) umid[u] = kd_ancestor(&T, E.unit_node[u], kmid);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t e = 0; e < E.n; ++e) {
    if (kind[e] != 1) {
      branch[e] = -1;
      continue;
    }
    if (n_pseudo > bypass) {
      h[e] = hfact * 2.0 * s[e];
      branch[e] = 3;
      continue;
    }
    if (!use_nf) {
      branch[e] = ora_node_h(pos + 3 * e, s[e], nu, upos, hfact, eps, &h[e], NULL);
      continue;
    }
    const int32_t na = E.entry_node[e];
    const int32_t mid = kd_ancestor(&T, na, kmid);
    double rcut = sqrt(3.0) * sqrt(T.nodes[mid].s2);
    if (rcut < 4.0 * hfact * s[e]) {
      const int lv = T.nodes[na].level - up_levels;
      rcut = 4.0 * hfact * sqrt(T.nodes[kd_ancestor(&T, na, lv > 0 ? lv : 0)].s2);
    }
    double *sub = (double *)malloc(sizeof(double) * 3 * (nu > 0 ? nu : 1));
    int64_t ns = 0;
    for (int64_t u = 0; u < nu; ++u) {
      double d[3];
      v_sub(pos + 3 * e, T.nodes[umid[u]].com, d);
      if (sqrt(v_dot(d, d)) < rcut) {
        memcpy(sub + 3 * ns, upos + 3 * u, sizeof(double) * 3);
        ++ns;
      }
    }
    branch[e] = ora_node_h(pos + 3 * e, s[e], ns, sub, hfact, eps, &h[e], NULL);
    free(sub);
  }
  stats_out[0] = T.n_nodes;
  stats_out[1] = nu;
  stats_out[2] = kmid;
  stats_out[3] = n_pseudo;
  *s_root_out = n > 0 ? sqrt(T.nodes[0].s2) : 0.0;
  const int64_t n_out = E.n;
  free(umid);
  free(upos);
  free(E.unit_node);
  free(E.entry_node);
  free(open_sorted);
  free(T.order);
  free(T.tmp);
  free(T.nodes);
  return n_out;
}
