// The Exact integral of a particle's M4 kernel over a convex Voronoi cell.
//
// Mathematics (Sec. 1 and Sec. 2.3 name the method -- an analytic volume
// integral of the SPH kernel over a cell of any geometry -- and Sec. 2.4.2
// fixes the kernel: M4 cubic spline truncated at 2h; the closed form below is
// derived for this library).  Lengths are in units of h, the particle at the
// origin.  With Phi(q) the kernel mass inside radius q, the mass of the cone
// from x to face f is (1/4pi) int_{Omega_f} Phi(R) dOmega; writing Phi = 1 -
// (1 - Phi) and using that the signed solid angles of a closed cell sum to
// 4pi [x inside], the weight becomes
//     w = S - sum_f sgn(d_f) C_f,      S = [x inside the cell],
// where C_f = (1/4pi) int_{Omega_f} (1 - Phi(R)) dOmega is the kernel mass
// beyond face f inside its cone.  1 - Phi vanishes beyond 2h, so a face more
// than 2h away contributes exactly 0, and a particle whose support lies inside
// (outside) the cell gets exactly 1 (0).  In polar coordinates about the
// foot P0 of x on the face plane (distance d), each edge e at in-plane
// distance p_e from P0 spans a right-triangle fan; with tau the coordinate
// along the edge from the foot of P0 and U = sqrt(d^2 + p^2 + tau^2),
//     4pi C_f / |d| = sum_e sgn(p_e) [F(tau_B) - F(tau_A)] - H(|d|) theta_f
// where H(u) = -int_u^2 (1 - Phi(s))/s^2 ds, F(tau) = int_0^{phi(tau)} H(U)
// dphi (zero contribution once U >= 2), and theta_f = 2pi when P0 lies inside
// the face polygon, 0 outside.  F is written with
//     phi = atan(tau/p), beta = atan(|d| tau/(p U)), L = asinh(tau/a),
//     a^2 = d^2 + p^2,
// as polynomials in (tau, U, p, |d|) plus multiples of phi, beta and L, one
// form for U < 1 and one for 1 <= U < 2, joined continuously at U = 1.
#include "common.hpp"

namespace sphmap {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv4Pi = 0.079577471545947667884;

// |d| * F_r(tau) for regime r (0: U < 1, 1: 1 <= U < 2).
__device__ inline double Fd64(int reg, double ad, double p, double tau, double a2, double U) {
  const double d2 = ad * ad;
  const double a = sqrt(a2);
  const double phi = atan2(tau, p);
  const double beta = atan2(ad * tau, p * U);
  const double L = asinh(tau / a);
  const double E1 = p * L + ad * beta;
  const double IU = 0.5 * (tau * U + a2 * L);
  const double U2 = U * U;
  const double IU2 = tau * U * (0.25 * U2 - 0.125 * a2) - 0.125 * a2 * a2 * L;
  const double E2 = d2 * phi + p * tau;
  const double E3 = d2 * E1 + p * IU;
  const double E4 = d2 * d2 * phi + 2.0 * d2 * p * tau + p * (p * p * tau + tau * tau * tau * (1.0 / 3.0));
  const double E5 = d2 * d2 * E1 + 2.0 * d2 * p * IU + p * (p * p * IU + IU2);
  if (reg == 0) return ad * (1.4 * phi - (2.0 / 3.0) * E2 + 0.3 * E4 - 0.1 * E5) - beta;
  return ad * (1.6 * phi - (4.0 / 3.0) * E2 + E3 - 0.3 * E4 + E5 * (1.0 / 30.0)) - (16.0 / 15.0) * beta;
}

// |d| H(|d|)
__device__ inline double dH64(double ad) {
  const double a2 = ad * ad, a3 = a2 * ad;
  if (ad < 1.0) return 1.4 * ad - 1.0 - (2.0 / 3.0) * a3 + 0.3 * a3 * a2 - 0.1 * a3 * a3;
  return 1.6 * ad - 16.0 / 15.0 - (4.0 / 3.0) * a3 + a3 * ad - 0.3 * a3 * a2 + a3 * a3 * (1.0 / 30.0);
}

// |d| [F(tB) - F(tA)] for one edge (p > 0, tA < tB).  n0 / n1 count the
// closed-form evaluations in the inner / outer regime.
__device__ double edge64(double ad, double p, double tA, double tB, int &n0, int &n1) {
  const double a2 = ad * ad + p * p;
  if (a2 >= 4.0) return 0.0;
  const double t2 = sqrt(4.0 - a2);
  const double ca = fmin(fmax(tA, -t2), t2), cb = fmin(fmax(tB, -t2), t2);
  if (!(ca < cb)) return 0.0;
  double t1 = -1.0, D = 0.0;
  if (a2 < 1.0) {
    t1 = sqrt(1.0 - a2);
    if (fabs(ca) > t1 || fabs(cb) > t1) {
      D = Fd64(0, ad, p, t1, a2, 1.0) - Fd64(1, ad, p, t1, a2, 1.0);
      ++n0;
      ++n1;
    }
  }
  auto F = [&](double t) -> double {
    const double at = fabs(t);
    if (at <= t1) {
      ++n0;
      return Fd64(0, ad, p, t, a2, sqrt(a2 + t * t));
    }
    ++n1;
    const double U = (at == t2) ? 2.0 : sqrt(a2 + t * t);
    return Fd64(1, ad, p, t, a2, U) + copysign(D, t);
  };
  return F(cb) - F(ca);
}

// Signed solid angle of a planar polygon seen from x (Van Oosterom and
// Strackee 1983 per fan triangle), used only on exact-boundary cases.
__device__ double solid_angle(const double *V, int nv, double x0, double x1, double x2) {
  double om = 0.0;
  const double ax = V[0] - x0, ay = V[1] - x1, az = V[2] - x2;
  const double la = sqrt(ax * ax + ay * ay + az * az);
  for (int k = 1; k + 1 < nv; ++k) {
    const double bx = V[3 * k] - x0, by = V[3 * k + 1] - x1, bz = V[3 * k + 2] - x2;
    const double cx = V[3 * k + 3] - x0, cy = V[3 * k + 4] - x1, cz = V[3 * k + 5] - x2;
    const double lb = sqrt(bx * bx + by * by + bz * bz), lc = sqrt(cx * cx + cy * cy + cz * cz);
    const double num = ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
    const double den = la * lb * lc + (ax * bx + ay * by + az * bz) * lc + (ax * cx + ay * cy + az * cz) * lb +
                       (bx * cx + by * cy + bz * cz) * la;
    om += 2.0 * atan2(num, den);
  }
  return om;
}

__global__ void __launch_bounds__(256) k_exact_fp64(int64_t P, const int32_t *pair_c, const int32_t *pair_p,
                                                   const double *xyz, const double *hh, const double *gen,
                                                   const int64_t *cfo, const int64_t *fvo, const double4 *fplane,
                                                   const double4 *fsphere, const double *fvpos, double *w_out,
                                                   int64_t *counters) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const int64_t c = pair_c[k];
  const int64_t i = pair_p[k];
  const double h = hh[i];
  const double ih = 1.0 / h;
  const double xr0 = xyz[3 * i] - gen[3 * c], xr1 = xyz[3 * i + 1] - gen[3 * c + 1],
               xr2 = xyz[3 * i + 2] - gen[3 * c + 2];
  double acc = 0.0;
  bool inside = true, on_boundary = false;
  int nf_int = 0, ne_vis = 0, ne_int = 0, nfd0 = 0, nfd1 = 0;
  const int64_t f0 = cfo[c], f1 = cfo[c + 1];
  for (int64_t f = f0; f < f1; ++f) {
    const double4 pl = fplane[f];
    if (!(pl.w > 0.0)) continue;
    const double dist = pl.w - (pl.x * xr0 + pl.y * xr1 + pl.z * xr2);
    if (dist < 0.0) inside = false;
    if (dist == 0.0) {
      on_boundary = true;
      continue;
    }
    const double d = dist * ih, ad = fabs(d);
    if (ad >= 2.0) continue;
    const double4 sp = fsphere[f];
    const double sx = xr0 - sp.x, sy = xr1 - sp.y, sz = xr2 - sp.z;
    const double reach = sp.w + 2.0 * h;
    if (sx * sx + sy * sy + sz * sz >= reach * reach) continue;
    ++nf_int;
    const double P0x = xr0 + dist * pl.x, P0y = xr1 + dist * pl.y, P0z = xr2 + dist * pl.z;
    const int64_t vs = fvo[f], ve = fvo[f + 1];
    const int nv = (int)(ve - vs);
    const double *V = fvpos + 3 * vs;
    double sum = 0.0;
    bool allpos = true, anyzero = false;
    for (int q = 0; q < nv; ++q) {
      const int q1 = (q + 1 == nv) ? 0 : q + 1;
      const double Ax = V[3 * q], Ay = V[3 * q + 1], Az = V[3 * q + 2];
      const double abx = V[3 * q1] - Ax, aby = V[3 * q1 + 1] - Ay, abz = V[3 * q1 + 2] - Az;
      const double len2 = abx * abx + aby * aby + abz * abz;
      if (len2 == 0.0) continue;
      const double len = sqrt(len2), il = 1.0 / len;
      const double ex = abx * il, ey = aby * il, ez = abz * il;
      // in-plane normal of the edge pointing into the polygon: n x e
      const double mx = pl.y * ez - pl.z * ey, my = pl.z * ex - pl.x * ez, mz = pl.x * ey - pl.y * ex;
      const double p = ((P0x - Ax) * mx + (P0y - Ay) * my + (P0z - Az) * mz) * ih;
      if (p <= 0.0) allpos = false;
      if (p == 0.0) {
        anyzero = true;
        continue;
      }
      ++ne_vis;
      const double tA = ((Ax - P0x) * ex + (Ay - P0y) * ey + (Az - P0z) * ez) * ih;
      const double tB = tA + len * ih;
      if (d * d + p * p >= 4.0) continue;
      ++ne_int;
      const double v = edge64(ad, fabs(p), tA, tB, nfd0, nfd1);
      sum += p > 0.0 ? v : -v;
    }
    double theta;
    if (anyzero) {
      // P0 on an edge line: total signed angle from the edges with p != 0
      theta = 0.0;
      for (int q = 0; q < nv; ++q) {
        const int q1 = (q + 1 == nv) ? 0 : q + 1;
        const double Ax = V[3 * q], Ay = V[3 * q + 1], Az = V[3 * q + 2];
        const double abx = V[3 * q1] - Ax, aby = V[3 * q1 + 1] - Ay, abz = V[3 * q1 + 2] - Az;
        const double len2 = abx * abx + aby * aby + abz * abz;
        if (len2 == 0.0) continue;
        const double len = sqrt(len2), il = 1.0 / len;
        const double ex = abx * il, ey = aby * il, ez = abz * il;
        const double mx = pl.y * ez - pl.z * ey, my = pl.z * ex - pl.x * ez, mz = pl.x * ey - pl.y * ex;
        const double p = (P0x - Ax) * mx + (P0y - Ay) * my + (P0z - Az) * mz;
        if (p == 0.0) continue;
        const double tA = (Ax - P0x) * ex + (Ay - P0y) * ey + (Az - P0z) * ez;
        const double dphi = atan2(tA + len, fabs(p)) - atan2(tA, fabs(p));
        theta += p > 0.0 ? dphi : -dphi;
      }
    } else {
      theta = allpos ? 2.0 * kPi : 0.0;
    }
    const double Cf = (sum - dH64(ad) * theta) * kInv4Pi;
    acc += d > 0.0 ? Cf : -Cf;
  }
  double S;
  if (!inside) {
    S = 0.0;
  } else if (!on_boundary) {
    S = 1.0;
  } else {
    // particle exactly on the cell boundary: signed solid angles of the
    // faces it is not on
    double om = 0.0;
    for (int64_t f = f0; f < f1; ++f) {
      const double4 pl = fplane[f];
      if (!(pl.w > 0.0)) continue;
      const double dist = pl.w - (pl.x * xr0 + pl.y * xr1 + pl.z * xr2);
      if (dist == 0.0) continue;
      const int64_t vs = fvo[f], ve = fvo[f + 1];
      om += fabs(solid_angle(fvpos + 3 * vs, (int)(ve - vs), xr0, xr1, xr2));
    }
    S = om * kInv4Pi;
  }
  w_out[k] = S - acc;
  if (counters) {
    atomicAdd((unsigned long long *)&counters[1], (unsigned long long)(f1 - f0));
    atomicAdd((unsigned long long *)&counters[2], (unsigned long long)nf_int);
    atomicAdd((unsigned long long *)&counters[3], (unsigned long long)ne_vis);
    atomicAdd((unsigned long long *)&counters[4], (unsigned long long)ne_int);
    atomicAdd((unsigned long long *)&counters[5], (unsigned long long)nfd0);
    atomicAdd((unsigned long long *)&counters[6], (unsigned long long)nfd1);
  }
}

}  // namespace

void exact_integral(Ctx &ctx, const TessDev &t, const PartDev &p, PairsDev &P, int precision, hipStream_t s) {
  (void)precision;
  P.w = P.mem.get<double>("w", P.n_pairs);
  if (P.n_pairs == 0) return;
  int64_t *ctr = ctx.counting ? ctx.d_counters : nullptr;
  if (ctr) SPH_HIP(hipMemsetAsync(ctr, 0, 8 * sizeof(int64_t), s));
  KernelTimer kt(&ctx, "exact_integral", s);
  k_exact_fp64<<<(unsigned)div_up(P.n_pairs, 256), 256, 0, s>>>(P.n_pairs, P.pair_c, P.pair_p, p.xyz, p.h, t.gen,
                                                                 t.cell_face_off, t.face_vtx_off, t.fplane,
                                                                 t.fsphere, t.fvpos, P.w, ctr);
  SPH_LAUNCH_CHECK();
  kt.done();
}

}  // namespace sphmap
