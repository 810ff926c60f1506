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
// along the edge from the foot of P0, U = sqrt(d^2 + p^2 + tau^2) and
// H(u) = -int_u^2 (1 - Phi(s))/s^2 ds (zero for u >= 2),
//     4pi C_f = sum_e sgn(p_e) int_{phi_A}^{phi_B} |d| [H(U) - H(|d|)] dphi.
// Each edge term is evaluated with the same angles phi = atan(tau/p) in both
// of its parts, so rounding in an endpoint angle is multiplied by
// H(U) - H(|d|), which vanishes where that rounding is largest (foot point
// next to a vertex).  A face none of whose edges comes within 2h, or whose
// foot point lies outside its bounding sphere by more than 0.1 h, uses the
// exact angle sum (2pi if P0 is inside the polygon, 0 outside) in place of
// the per-edge angle terms: far from the vertices the pairing is not needed,
// and the terms' binary32 rounding would otherwise remain in a face whose
// plane passes close to the particle while its polygon lies far off.
//
// The antiderivative |d| int H(U) dphi is, per regime (U < 1, 1 <= U < 2),
//     c_phi phi + c_beta beta + c_L L + tau (c_1 + c_3 tau^2)
//                                     + tau U (c_5 + c_7 tau^2),
//     phi = atan(tau/p), beta = atan(|d| tau / (p U)), L = asinh(tau/a),
//     a^2 = d^2 + p^2,
// with coefficients that depend on (|d|, p) only, joined continuously at
// U = 1.  Two evaluation paths:
//   binary64: every step in binary64 with the math library's functions;
//   mixed: edge geometry in binary32; atan, asinh and square roots from
//     binary32 polynomial cores and seeds with binary64 range reduction and
//     assembly (atan within 4.7e-9, log within 7.3e-10 relative);
//     coefficients, angles' combination and
//     every accumulation in binary64.  A pair with an edge whose line passes
//     within 1e-2 h of the particle (d^2 + p^2 below 1e-4 h^2) or whose
//     foot point lies on the edge line (p = 0), or with a face plane through
//     the particle (|d| below 1e-20 h), goes to a second kernel that
//     recomputes such edges, and faces within 1e-4 h, from binary64
//     geometry; every pair whose cell is small against the support (R_c <
//     0.25 h) takes the binary64 path.
#include <algorithm>
#include <vector>
#include <cstdlib>
#include <type_traits>

#include "common.hpp"

namespace sphmap {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kHalfPi = 1.57079632679489661923;
constexpr double kQuarterPi = 0.78539816339744830962;
constexpr double kInv4Pi = 0.079577471545947667884;
constexpr double kLn2 = 0.69314718055994530942;

// ----------------------------------------------------------- coefficients
struct Coef {
  double phi, beta, L, t1, t3, tU, t3U;
};

// Regime 0 (U < 1) and regime 1 (1 <= U < 2) coefficients of
// |d| int H(U) dphi for one edge.
__device__ inline void edge_coefs(double ad, double p, Coef &c0, Coef &c1) {
  const double d2 = ad * ad, p2 = p * p, a2 = d2 + p2, d4 = d2 * d2;
  const double A = 2.0 * d2 * p + p2 * p;
  const double B = d4 * p + 0.5 * A * a2 - 0.125 * p * a2 * a2;
  const double T = 0.5 * A + 0.125 * p * a2;
  const double adp = ad * p;
  c0.phi = ad * (1.4 - (2.0 / 3.0) * d2 + 0.3 * d4);
  c0.beta = -1.0 - 0.1 * d4 * d2;
  c0.L = -0.1 * ad * B;
  c0.t1 = ad * (-(2.0 / 3.0) * p + 0.3 * A);
  c0.t3 = 0.1 * adp;
  c0.tU = -0.1 * ad * T;
  c0.t3U = -0.025 * adp;
  c1.phi = ad * (1.6 - (4.0 / 3.0) * d2 - 0.3 * d4);
  c1.beta = -16.0 / 15.0 + d4 + d4 * d2 * (1.0 / 30.0);
  c1.L = ad * (d2 * p + 0.5 * p * a2 + B * (1.0 / 30.0));
  c1.t1 = ad * (-(4.0 / 3.0) * p - 0.3 * A);
  c1.t3 = -0.1 * adp;
  c1.tU = ad * (0.5 * p + T * (1.0 / 30.0));
  c1.t3U = adp * (1.0 / 120.0);
}

__device__ inline double coef_eval(const Coef &c, double phi, double beta, double L, double tau, double U) {
  const double t2 = tau * tau;
  return c.phi * phi + c.beta * beta + c.L * L + tau * (c.t1 + c.t3 * t2) + tau * U * (c.tU + c.t3U * t2);
}

// |d| H(|d|)
__device__ inline double dH(double ad) {
  const double a2 = ad * ad, a3 = a2 * ad;
  if (ad < 1.0) return 1.4 * ad - 1.0 - (2.0 / 3.0) * a3 + 0.3 * a3 * a2 - 0.1 * a3 * a3;
  return 1.6 * ad - 16.0 / 15.0 - (4.0 / 3.0) * a3 + a3 * ad - 0.3 * a3 * a2 + a3 * a3 * (1.0 / 30.0);
}

// ------------------------------------------------- transcendental kernels
// binary64 with the math library
struct Math64 {
  static __device__ inline double atanq(double y, double x) { return atan2(y, x); }  // x > 0
  // angle subtended at the foot point by the edge [tA, tB] at distance p > 0
  static __device__ inline double span(double p, double tA, double tB) {
    return atan2(p * (tB - tA), fma(tA, tB, p * p));
  }
  static __device__ inline double asinh_(double z) { return asinh(z); }
  static __device__ inline double sqrt_(double v) { return sqrt(v); }
  static __device__ inline double rcp(double v) { return 1.0 / v; }
};

// binary32 seeds / polynomial cores, binary64 refinement and assembly
__device__ inline double rcp_mixed(double x) {
  const double r = (double)__builtin_amdgcn_rcpf((float)x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double sqrt_mixed(double v) {
  // binary32 seed and one Newton step for 1/sqrt: ~2e-14 relative, below
  // the 7e-10 to 5e-9 of the transcendental cores it feeds
  double y = (double)__builtin_amdgcn_rsqf((float)v);
  y = y * fma(-0.5 * v * y, y, 1.5);
  return v * y;
}
// atan(y/x) for x > 0: reduce to |s| <= tan(pi/8) with one division, then
// atan(s) = s + s^3 P(s^2), P a degree-5 polynomial: a minimax fit of the
// relative error on [0, tan^2(pi/8)] (fit_cores.py), evaluated in binary32;
// with binary32 coefficients and Horner steps the core's relative error is
// at most 4.7e-9.
__device__ inline double atan_mixed(double y, double x) {
  const double ay = fabs(y);
  const bool small = ay <= 0.41421356237309503 * x;
  const bool large = ay >= 2.414213562373095 * x;
  const double num = small ? ay : (large ? -x : ay - x);
  const double den = small ? x : (large ? ay : ay + x);
  const double base = small ? 0.0 : (large ? kHalfPi : kQuarterPi);
  // rcp_mixed is within ~1e-14 relative, far below the core's 4.7e-9: no
  // further correction of the quotient
  const double s = num * rcp_mixed(den);
  const double z = s * s;
  const float zf = (float)z;
  float P = 0.050527118146419525f;
  P = fmaf(P, zf, -0.08626646548509598f);
  P = fmaf(P, zf, 0.11071662604808807f);
  P = fmaf(P, zf, -0.14284169673919678f);
  P = fmaf(P, zf, 0.19999977946281433f);
  P = fmaf(P, zf, -0.3333333432674408f);
  const double r = base + fma(s * z, (double)P, s);
  return copysign(r, y);
}
// asinh(z) = log(|z| + sqrt(z^2 + 1)); log(2^e m) = e ln2 + 2 atanh(t),
// t = (m - 1)/(m + 1), 2 atanh(t) = 2t + t^3 Q(t^2), Q a degree-3 polynomial
// fitted on |t| <= 3 - 2 sqrt(2) (fit_cores.py), evaluated in binary32 (the
// core's relative error is at most 7.3e-10).
__device__ inline double asinh_mixed(double z) {
  const double az = fabs(z);
  const double q = sqrt_mixed(fma(az, az, 1.0));
  const double sv = az + q;
  int e = __builtin_amdgcn_frexp_exp(sv);
  double m = __builtin_amdgcn_frexp_mant(sv);  // [0.5, 1)
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const double mm1 = (e == 0) ? az + az * az * rcp_mixed(q + 1.0) : m - 1.0;
  const double t = mm1 * rcp_mixed(m + 1.0);  // ~1e-14 relative, as in atan_mixed
  const double t2 = t * t;
  const float zf = (float)t2;
  float Q = 0.23331113159656525f;
  Q = fmaf(Q, zf, 0.2855079174041748f);
  Q = fmaf(Q, zf, 0.4000012278556824f);
  Q = fmaf(Q, zf, 0.6666666865348816f);
  const double L = (double)e * kLn2 + fma(t * t2, (double)Q, 2.0 * t);
  return copysign(L, z);
}
struct MathMixed {
  static __device__ inline double atanq(double y, double x) { return atan_mixed(y, x); }
  static __device__ inline double span(double p, double tA, double tB) {
    const double y = p * (tB - tA), x = fma(tA, tB, p * p);  // y > 0
    const double r = atan_mixed(y, fabs(x));  // pi/2 for x = 0
    return x < 0.0 ? kPi - r : r;
  }
  static __device__ inline double asinh_(double z) { return asinh_mixed(z); }
  static __device__ inline double sqrt_(double v) { return sqrt_mixed(v); }
  static __device__ inline double rcp(double v) { return rcp_mixed(v); }
};

// ------------------------------------------------------------- one edge
struct EdgeCount {
  int n0 = 0, n1 = 0;
};

// sum over the fan of |d| [H(U) - H(|d|)] dphi for one edge with p > 0 and
// tA < tB.  Returns false in `integ` when no part of the edge lies within
// U < 2 (then the value is -dh * (phi_B - phi_A)).
template <class M>
__device__ double edge_term(double ad, double p, double tA, double tB, double dh, bool &integ, EdgeCount &cnt) {
  const double a2 = ad * ad + p * p;
  const double r2 = 4.0 - a2;
  integ = r2 > 0.0 && (tA < 0.0 || tA * tA < r2) && (tB > 0.0 || tB * tB < r2);
  const double phiA = M::atanq(tA, p), phiB = M::atanq(tB, p);
  if (!integ) return -dh * (phiB - phiA);
  const double t2 = M::sqrt_(r2);
  const double ca = fmin(fmax(tA, -t2), t2), cb = fmin(fmax(tB, -t2), t2);
  if (!(ca < cb)) {
    integ = false;
    return -dh * (phiB - phiA);
  }
  Coef c0, c1;
  edge_coefs(ad, p, c0, c1);
  const double a = M::sqrt_(a2);
  const double ia = M::rcp(a);
  double t1 = -1.0, D = 0.0;
  if (a2 < 1.0) {
    t1 = M::sqrt_(1.0 - a2);
    if (fabs(ca) > t1 || fabs(cb) > t1) {
      const double ph = M::atanq(t1, p), be = M::atanq(ad * t1, p), Lz = M::asinh_(t1 * ia);
      D = coef_eval(c0, ph, be, Lz, t1, 1.0) - coef_eval(c1, ph, be, Lz, t1, 1.0);
      ++cnt.n0;
      ++cnt.n1;
    }
  }
  auto F = [&](double t, double phi) -> double {
    const double at = fabs(t);
    const double U = (at == t2) ? 2.0 : M::sqrt_(a2 + t * t);
    const double be = M::atanq(ad * t, p * U), Lz = M::asinh_(t * ia);
    if (at <= t1) {
      ++cnt.n0;
      return coef_eval(c0, phi, be, Lz, t, U);
    }
    ++cnt.n1;
    return coef_eval(c1, phi, be, Lz, t, U) + copysign(D, t);
  };
  const double fa = F(ca, ca == tA ? phiA : M::atanq(ca, p));
  const double fb = F(cb, cb == tB ? phiB : M::atanq(cb, p));
  return (fb - fa) - dh * (phiB - phiA);
}

// edge_term with binary64 geometry from the mixed path: the mixed cores seed
// their square roots, reciprocals and divisions in binary32, so lengths below
// 1e-15 h (a^2 or p under 1e-30) go to the math library instead.
template <class M>
__device__ inline double edge_term_geo64(double ad, double p, double tA, double tB, double dh, bool &integ,
                                         EdgeCount &cnt) {
  if (!std::is_same<M, Math64>::value && (ad * ad + p * p < 1e-30 || p < 1e-30))
    return edge_term<Math64>(ad, p, tA, tB, dh, integ, cnt);
  return edge_term<M>(ad, p, tA, tB, dh, integ, cnt);
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

// S for a particle exactly on the boundary: signed solid angles of the faces
// it is not on, in binary64.
__device__ double boundary_S(int64_t f0, int64_t f1, const double4 *fplane, const int64_t *fvo, const double *fvpos,
                             double x0, double x1, double x2) {
  double om = 0.0;
  for (int64_t f = f0; f < f1; ++f) {
    const double4 pl = fplane[f];
    if (!(pl.w > 0.0)) continue;
    const double dist = pl.w - (pl.x * x0 + pl.y * x1 + pl.z * x2);
    if (dist == 0.0) continue;
    om += fabs(solid_angle(fvpos + 3 * fvo[f], (int)(fvo[f + 1] - fvo[f]), x0, x1, x2));
  }
  return om * kInv4Pi;
}

// One face with binary64 geometry about the generator, particle at xr; the
// edges are evaluated with M's transcendental cores (the math library for
// the binary64 path, the mixed cores where the mixed path meets a face
// within 1e-4 h of the particle).
template <class M>
__device__ double face_fp64(const double4 pl, double dist, double ih, double xr0, double xr1, double xr2,
                            const double *V, int nv, int &ne_vis, int &ne_int, EdgeCount &cnt) {
  const double d = dist * ih, ad = fabs(d);
  const double dh = dH(ad);
  const double P0x = xr0 + dist * pl.x, P0y = xr1 + dist * pl.y, P0z = xr2 + dist * pl.z;
  double sum = 0.0;
  bool allpos = true, anyzero = false, anyint = false;
  for (int q = 0; q < nv; ++q) {
    const int q1 = (q + 1 == nv) ? 0 : q + 1;
    const double Ax = V[3 * q], Ay = V[3 * q + 1], Az = V[3 * q + 2];
    const double Bx = V[3 * q1], By = V[3 * q1 + 1], Bz = V[3 * q1 + 2];
    const double abx = Bx - Ax, aby = By - Ay, abz = Bz - Az;
    const double len2 = abx * abx + aby * aby + abz * abz;
    if (len2 == 0.0) continue;
    const double il = 1.0 / sqrt(len2);
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
    const double tB = ((Bx - P0x) * ex + (By - P0y) * ey + (Bz - P0z) * ez) * ih;
    bool integ;
    const double v = edge_term_geo64<M>(ad, fabs(p), tA, tB, dh, integ, cnt);
    anyint |= integ;
    ne_int += integ;
    sum += p > 0.0 ? v : -v;
  }
  if (!anyint && !anyzero) sum = -dh * (allpos ? 2.0 * kPi : 0.0);
  const double Cf = sum * kInv4Pi;
  return d > 0.0 ? Cf : -Cf;
}

// One mapping instance as the persistent kernels see it (device-side table).
struct ExactInst {
  const int32_t *pair_c, *pair_p;
  const double *xyz, *hh, *gen;
  const float *radius;  // binary32 bounding radius R_c of each cell
  const int64_t *cfo, *fvo;
  const double4 *fplane, *fsphere;
  const float4 *fplane32, *fvpos32, *edgeA, *edgeE, *edgeM;
  const double *fvpos;
  double *w;
  int64_t P;
  // shared faces (mixed path; all null when the grid has none, and in a
  // device-counted batch): the pair lists' cell offsets; each face's code
  // (its slot among the shared faces its cell evaluates, -1 a face of this
  // cell only, -2 the twin's); per cell the number of those slots and where
  // its gifts start; the gifts, slot-major per cell (slot s of the cell's
  // pair t at gbase[c] + s n_c + t: the fixed-point total of that face for
  // that pair); each pair's state after the edge kernel
  const int64_t *cell_off;
  const int32_t *fcode, *cslots, *ftwin;
  const int64_t *gbase;
  long long *gift;
  uint8_t *wflag;  // bit 0: S (inside); bit 1: left to the redo kernel
};
constexpr uint8_t kFlagInside = 1, kFlagRedo = 2;

// v in units of 2^-46, rounded to nearest, as a two's-complement 64-bit
// integer, for |v| < 32 (every term is an angle weighted by at most 1 in
// magnitude).  With 1.5 * 2^52 added, v * 2^46 is rounded once, to an
// integer, and lies in [2^52, 2^53) where the binary64 spacing is 1, so
// subtracting the constant's bit pattern from the result's leaves that
// integer.
constexpr double kFixMagic = 0x1.8p52;
// the integer left in t = fma(x, y, kFixMagic), for |x y| < 2^51
__device__ inline unsigned long long fixed_from(double t) {
  return (unsigned long long)__double_as_longlong(t) - (unsigned long long)__double_as_longlong(kFixMagic);
}
__device__ inline unsigned long long to_fixed(double v) { return fixed_from(fma(v, 0x1p46, kFixMagic)); }

__device__ inline double from_fixed(unsigned long long a) {
  const int hi = (int)(a >> 32);
  const unsigned lo = (unsigned)a;
  return ((double)hi * 0x1p32 + (double)lo) * 0x1p-46;
}


// instance holding global chunk `chunk` (chunk0: first chunk of each
// instance, ascending, n_inst + 1 entries)
__device__ inline int inst_of(const int64_t *chunk0, int n_inst, int64_t chunk) {
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chunk0[mid] <= chunk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct Counters {
  int nf_int = 0, ne_vis = 0, ne_int = 0, n64 = 0;
  EdgeCount fd;
};

__device__ inline void flush_counters(int64_t *counters, int64_t nfaces, const Counters &k) {
  atomicAdd((unsigned long long *)&counters[1], (unsigned long long)nfaces);
  atomicAdd((unsigned long long *)&counters[2], (unsigned long long)k.nf_int);
  atomicAdd((unsigned long long *)&counters[3], (unsigned long long)k.ne_vis);
  atomicAdd((unsigned long long *)&counters[4], (unsigned long long)k.ne_int);
  atomicAdd((unsigned long long *)&counters[5], (unsigned long long)k.fd.n0);
  atomicAdd((unsigned long long *)&counters[6], (unsigned long long)k.fd.n1);
  atomicAdd((unsigned long long *)&counters[7], (unsigned long long)k.n64);
}

// Whether a face can reach the support: the particle (at xr about the
// generator, dist from the face plane) lies within 2h of the face's bounding
// disk -- the circle of the bounding sphere's radius about its centre,
// which lies in the face plane and holds the polygon.  The distance from the
// disk bounds the distance from the polygon from below, and a face farther
// than 2h adds exactly 0.  The in-plane distance is taken in binary32 and
// rounded down by 1e-6, so no face within reach is dropped.
__device__ inline bool disk_within_2h(double xr0, double xr1, double xr2, double dist, double h, const double4 &sp) {
  const double sx = xr0 - sp.x, sy = xr1 - sp.y, sz = xr2 - sp.z;
  const double rho2 = (sx * sx + sy * sy + sz * sz) - dist * dist;
  const double rho = (double)__builtin_sqrtf((float)fmax(rho2, 0.0)) * (1.0 - 1e-6);
  const double t = fmax(rho - sp.w, 0.0);
  return dist * dist + t * t < 4.0 * h * h;
}

// ------------------------------------------------------- binary64 kernel
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
  Counters K;
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
    if (fabs(dist) >= 2.0 * h) continue;
    if (!disk_within_2h(xr0, xr1, xr2, dist, h, fsphere[f])) continue;
    ++K.nf_int;
    acc += face_fp64<Math64>(pl, dist, ih, xr0, xr1, xr2, fvpos + 3 * fvo[f], (int)(fvo[f + 1] - fvo[f]), K.ne_vis,
                     K.ne_int, K.fd);
  }
  double S = inside ? 1.0 : 0.0;
  if (inside && on_boundary) S = boundary_S(f0, f1, fplane, fvo, fvpos, xr0, xr1, xr2);
  w_out[k] = S - acc;
  if (counters) flush_counters(counters, f1 - f0, K);
}

// ---------------------------------------------------------- mixed kernel
constexpr float kDegenerate = 1e-4f;  // p or |d| below this (units of h): binary64 edge
// A face plane closer than this to the particle (units of h) is taken as
// through it: the edge kernel leaves the pair to the binary64 kernel.  Any
// larger distance is resolved by the edge kernel's binary32 geometry, whose
// rounding matters only near edge lines (kEdgeNear below).
constexpr double kOnPlane = 1e-20;
// An edge whose line passes within this distance of the particle (in units
// of h: d^2 + p^2 below its square) is evaluated from binary64 geometry: the
// fan's terms there vary on the scale sqrt(d^2 + p^2), so the binary32
// rounding of the foot point and edge frame is amplified by its inverse.
constexpr float kEdgeNear = 1e-2f;
// A cell smaller than this fraction of h (R_c < 0.25 h) is evaluated as on
// the binary64 path (binary64 geometry and functions): its faces are small
// and, seen from a particle far out in the support, their terms cancel far
// below the mixed path's absolute accuracy (about 1e-8 of w), which matters
// where a heavy entry grazes a light cell (a pseudo-particle's support over
// the small cells of the particles near a source).
constexpr double kSmallCell = 0.25;

// Face f's share of sum_f sgn(d_f) C_f for the pair whose particle sits at
// xr about the generator (x in units of h, binary32), with the face's part of
// the inside and boundary tests; 0 for a face out of reach.
__device__ inline double face_mixed(int64_t f, double xr0, double xr1, double xr2, double h, double ih, float ihf,
                                    float x0, float x1, float x2, const int64_t *fvo, const double4 *fplane,
                                    const float4 *fplane32, const double4 *fsphere, const double *fvpos,
                                    const float4 *fvpos32, bool &inside, bool &on_boundary, Counters &K) {
  const double4 pl = fplane[f];
  if (!(pl.w > 0.0)) return 0.0;
  const double dist = pl.w - (pl.x * xr0 + pl.y * xr1 + pl.z * xr2);
  if (dist < 0.0) inside = false;
  if (dist == 0.0) {
    on_boundary = true;
    return 0.0;
  }
  if (fabs(dist) >= 2.0 * h) return 0.0;
  if (!disk_within_2h(xr0, xr1, xr2, dist, h, fsphere[f])) return 0.0;
  ++K.nf_int;
  const int64_t vs = fvo[f];
  const int nv = (int)(fvo[f + 1] - vs);
  const double d = dist * ih, ad = fabs(d);
  if (ad < kDegenerate) {
    // particle on the face plane to within 1e-4 h: the whole face from binary64 geometry
    K.n64 += nv;
    return face_fp64<MathMixed>(pl, dist, ih, xr0, xr1, xr2, fvpos + 3 * vs, nv, K.ne_vis, K.ne_int, K.fd);
  }
  const double dh = dH(ad);
  const float4 pf = fplane32[f];
  const float df = (float)d;
  const float P0x = x0 + df * pf.x, P0y = x1 + df * pf.y, P0z = x2 + df * pf.z;
  double sum = 0.0;
  bool allpos = true, anyzero = false, anyint = false;
  float4 A = fvpos32[vs];
  A.x *= ihf;
  A.y *= ihf;
  A.z *= ihf;
  for (int q = 0; q < nv; ++q) {
    const int q1 = (q + 1 == nv) ? 0 : q + 1;
    float4 B = fvpos32[vs + q1];
    B.x *= ihf;
    B.y *= ihf;
    B.z *= ihf;
    const float abx = B.x - A.x, aby = B.y - A.y, abz = B.z - A.z;
    const float len2 = abx * abx + aby * aby + abz * abz;
    if (len2 > 0.0f) {
      const float il = __builtin_amdgcn_rsqf(len2);
      const float ex = abx * il, ey = aby * il, ez = abz * il;
      const float mx = pf.y * ez - pf.z * ey, my = pf.z * ex - pf.x * ez, mz = pf.x * ey - pf.y * ex;
      const float p = (P0x - A.x) * mx + (P0y - A.y) * my + (P0z - A.z) * mz;
      if (p <= 0.0f) allpos = false;
      if (p == 0.0f) {
        anyzero = true;
      } else {
        ++K.ne_vis;
        bool integ;
        double v;
        if (fabsf(p) < kDegenerate || (float)(ad * ad) + p * p < kEdgeNear * kEdgeNear) {
          // foot point within 1e-4 h of the edge line, or the edge line
          // within 1e-2 h of the particle: binary64 geometry
          ++K.n64;
          const double *V = fvpos + 3 * vs;
          const double P0dx = xr0 + dist * pl.x, P0dy = xr1 + dist * pl.y, P0dz = xr2 + dist * pl.z;
          const double Ax = V[3 * q], Ay = V[3 * q + 1], Az = V[3 * q + 2];
          const double Bx = V[3 * q1], By = V[3 * q1 + 1], Bz = V[3 * q1 + 2];
          const double bx = Bx - Ax, by = By - Ay, bz = Bz - Az;
          const double il64 = 1.0 / sqrt(bx * bx + by * by + bz * bz);
          const double e0 = bx * il64, e1 = by * il64, e2 = bz * il64;
          const double m0 = pl.y * e2 - pl.z * e1, m1 = pl.z * e0 - pl.x * e2, m2 = pl.x * e1 - pl.y * e0;
          const double p64 = ((P0dx - Ax) * m0 + (P0dy - Ay) * m1 + (P0dz - Az) * m2) * ih;
          const double tA = ((Ax - P0dx) * e0 + (Ay - P0dy) * e1 + (Az - P0dz) * e2) * ih;
          const double tB = ((Bx - P0dx) * e0 + (By - P0dy) * e1 + (Bz - P0dz) * e2) * ih;
          if (p64 == 0.0) {
            v = 0.0;
            integ = false;
          } else {
            v = edge_term_geo64<MathMixed>(ad, fabs(p64), tA, tB, dh, integ, K.fd);
            if (p64 < 0.0) v = -v;
          }
        } else {
          const float tA = (A.x - P0x) * ex + (A.y - P0y) * ey + (A.z - P0z) * ez;
          const float tB = (B.x - P0x) * ex + (B.y - P0y) * ey + (B.z - P0z) * ez;
          v = edge_term<MathMixed>(ad, (double)fabsf(p), (double)tA, (double)tB, dh, integ, K.fd);
          if (p < 0.0f) v = -v;
        }
        anyint |= integ;
        K.ne_int += integ;
        sum += v;
      }
    }
    A = B;
  }
  if (!anyint && !anyzero) sum = -dh * (allpos ? 2.0 * kPi : 0.0);
  const double Cf = sum * kInv4Pi;
  return d > 0.0 ? Cf : -Cf;
}

// ------------------------------------------------------- wave helpers
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int wave_scan_excl(int v, int lane) {
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x - v;
}

// binary64 geometry of edge (e, e1) of a face about the generator, particle at xr
__device__ inline bool edge_geo64(const double4 pl, double dist, double ih, double xr0, double xr1, double xr2,
                                  const double *V, int e, int e1, double &p, double &tA, double &tB) {
  const double P0x = xr0 + dist * pl.x, P0y = xr1 + dist * pl.y, P0z = xr2 + dist * pl.z;
  const double Ax = V[3 * e], Ay = V[3 * e + 1], Az = V[3 * e + 2];
  const double Bx = V[3 * e1], By = V[3 * e1 + 1], Bz = V[3 * e1 + 2];
  const double bx = Bx - Ax, by = By - Ay, bz = Bz - Az;
  const double len2 = bx * bx + by * by + bz * bz;
  if (!(len2 > 0.0)) return false;
  const double il = 1.0 / sqrt(len2);
  const double ex = bx * il, ey = by * il, ez = bz * il;
  const double mx = pl.y * ez - pl.z * ey, my = pl.z * ex - pl.x * ez, mz = pl.x * ey - pl.y * ex;
  p = ((P0x - Ax) * mx + (P0y - Ay) * my + (P0z - Az) * mz) * ih;
  tA = ((Ax - P0x) * ex + (Ay - P0y) * ey + (Az - P0z) * ez) * ih;
  tB = ((Bx - P0x) * ex + (By - P0y) * ey + (Bz - P0z) * ez) * ih;
  return true;
}

// ------------------------------------------------- persistent kernels
constexpr int kFlatWaves = 4;  // wavefronts per workgroup

__global__ void k_zero_i32(int32_t *p, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = 0;
}

// Work counters of the persistent Exact kernel: one per XCD, each on its own
// 64-byte line, then the redo count.  Workgroups are dispatched to the eight
// XCDs in turn (workgroup b on XCD b mod 8), so XCD x first takes the x-th
// eighth of the chunks, in order: consecutive chunks (the pairs of one cell
// and its neighbours) meet in one L2 and reuse its face and edge data.  An
// XCD whose eighth runs out takes chunks from the others' in turn.
constexpr int kXcd = 8;
constexpr int kCtrStride = 16;
constexpr int kCtrInts = kXcd * kCtrStride + 1;
constexpr int kRedoCtr = kXcd * kCtrStride;

// Instance table of a batch whose pair counts are known only on the device:
// each instance's count *np[k] (0 for an overflowed list) and the first
// chunk of each instance.  One thread; the table's pointers were uploaded
// with the plan.
__global__ void k_exact_table(int n_inst, const int64_t *const *np, ExactInst *insts, int64_t *chunk0) {
  if (threadIdx.x != 0) return;
  int64_t c = 0;
  for (int k = 0; k < n_inst; ++k) {
    const int64_t P = *np[k];
    insts[k].P = P;
    chunk0[k] = c;
    c += (P + 63) / 64;
  }
  chunk0[n_inst] = c;
}

// atan2(y, x) for any x, from the binary32-core atan
__device__ inline double atan2_mixed(double y, double x) {
  const double r = atan_mixed(y, fabs(x));  // copysign(pi/2, y) for x = 0
  return x < 0.0 ? copysign(kPi, y) - r : r;
}

// log(num / den) for num, den > 0 with one division: the exponents are split
// off both, the mantissa ratio brought into [1/sqrt2, sqrt2] and
// log(m) = 2 atanh((m_n - m_d) / (m_n + m_d)) from the binary32 core.
__device__ inline double log_ratio_mixed(double num, double den) {
  int e = __builtin_amdgcn_frexp_exp(num) - __builtin_amdgcn_frexp_exp(den);
  double mn = __builtin_amdgcn_frexp_mant(num);  // [0.5, 1)
  const double md = __builtin_amdgcn_frexp_mant(den);
  if (mn < 0.70710678118654752 * md) {
    mn *= 2.0;
    e -= 1;
  } else if (mn > 1.4142135623730950 * md) {
    mn *= 0.5;
    e += 1;
  }
  const double t = (mn - md) * rcp_mixed(mn + md);  // ~1e-14 relative, as in atan_mixed
  const double t2 = t * t;
  const float zf = (float)t2;
  float Q = 0.23331113159656525f;
  Q = fmaf(Q, zf, 0.2855079174041748f);
  Q = fmaf(Q, zf, 0.4000012278556824f);
  Q = fmaf(Q, zf, 0.6666666865348816f);
  return (double)e * kLn2 + fma(t * t2, (double)Q, 2.0 * t);
}

// The functions the pieces take: binary32 cores with binary64 assembly for
// the edge kernel, the math library for the binary64-geometry kernel's
// small cells.
struct PieceMixed {
  static __device__ inline double atan2_(double y, double x) { return atan2_mixed(y, x); }
  static __device__ inline double log_ratio(double num, double den) { return log_ratio_mixed(num, den); }
  static __device__ inline double sqrt_(double v) { return sqrt_mixed(v); }
};
struct Piece64 {
  static __device__ inline double atan2_(double y, double x) { return atan2(y, x); }
  static __device__ inline double log_ratio(double num, double den) { return log(num / den); }
  static __device__ inline double sqrt_(double v) { return sqrt(v); }
};

// F(v) - F(u) over [u, v] inside one regime with coefficients c, from
// differences: phi(v) - phi(u) and beta(v) - beta(u) as one angle each
// (atan2 of the tangent-difference numerator and denominator, scaled by
// positive factors), L(v) - L(u) = log(N(v) / N(u)) with N(t) = t + U(t),
// written a^2 / (U - t) for t < 0 to avoid cancellation.
template <class Q>
__device__ inline double piece(const Coef &c, double ad, double p, double a2, double u, double Uu, double v,
                               double Uv) {
  const double dphi = Q::atan2_(p * (v - u), fma(u, v, p * p));
  const double dbeta = Q::atan2_(ad * p * (v * Uu - u * Uv), p * p * Uu * Uv + ad * ad * u * v);
  const bool un = u < 0.0, vn = v < 0.0;
  const double Nv = vn ? Uu - u : v + Uv;
  const double Nu = un ? (vn ? Uv - v : a2) : u + Uu;
  const double num = (un && !vn) ? Nv * (Uu - u) : Nv;
  const double dL = Q::log_ratio(num, Nu);
  const double u2 = u * u, v2 = v * v;
  const double poly = (v * fma(c.t3, v2, c.t1) - u * fma(c.t3, u2, c.t1)) +
                      (v * Uv * fma(c.t3U, v2, c.tU) - u * Uu * fma(c.t3U, u2, c.tU));
  return c.phi * dphi + c.beta * dbeta + c.L * dL + poly;
}

// w0 * (inner coefficients) + w1 * (outer coefficients) of one edge, formed
// directly so that only one set is live: (1, 0) inner, (0, 1) outer,
// (2, -2) twice their difference.
__device__ inline Coef coef_mix(double ad, double p, double w0, double w1) {
  const double d2 = ad * ad, p2 = p * p, a2 = d2 + p2, d4 = d2 * d2;
  const double A = 2.0 * d2 * p + p2 * p;
  const double B = d4 * p + 0.5 * A * a2 - 0.125 * p * a2 * a2;
  const double T = 0.5 * A + 0.125 * p * a2;
  const double adp = ad * p;
  const double kA = -(2.0 / 3.0) * w0 - (4.0 / 3.0) * w1;
  const double kB = 0.3 * (w0 - w1);
  const double kC = -0.1 * w0 + w1 * (1.0 / 30.0);
  Coef c;
  c.phi = ad * ((1.4 * w0 + 1.6 * w1) + kA * d2 + kB * d4);
  c.beta = (-w0 - (16.0 / 15.0) * w1) + w1 * d4 + kC * d4 * d2;
  c.L = ad * (w1 * (d2 * p + 0.5 * p * a2) + kC * B);
  c.t1 = ad * (kA * p + kB * A);
  c.t3 = 0.1 * (w0 - w1) * adp;
  c.tU = ad * (0.5 * w1 * p + kC * T);
  c.t3U = (-0.025 * w0 + w1 * (1.0 / 120.0)) * adp;
  return c;
}

// One piece of an edge within 2h (p > 0, tA < tB), its range clipped to
// U <= 2.  Mode 0: the whole clipped range, in the regime of its midpoint.
// A range that crosses t = -t1 or t = +t1 (U = 1) is evaluated as two
// items: mode 1 its first piece and mode 2 its second -- split at the
// crossing, or, across both crossings, the outer coefficients over the
// whole range (mode 1) plus 2 (F_inner - F_outer) over [0, t1] (mode 2;
// both antiderivatives are odd in t).  When rounding at the join loses the
// crossing, mode 1 takes the whole range and mode 2 adds nothing.
template <class Q>
__device__ inline double piece_of(double ad, double p, double tA, double tB, int mode, EdgeCount &cnt) {
  const double a2 = ad * ad + p * p;
  const double t2 = Q::sqrt_(4.0 - a2);
  const double ca = fmin(fmax(tA, -t2), t2), cb = fmin(fmax(tB, -t2), t2);
  const bool in = a2 < 1.0;  // an inner regime exists
  const double t1 = in ? Q::sqrt_(1.0 - a2) : 0.0;
  const bool lo = in && ca < -t1 && cb > -t1, hi = in && ca < t1 && cb > t1;
  const bool both = lo && hi, one = mode == 0 || (!lo && !hi);
  const bool m2 = mode == 2 && !one, m1 = !one && !m2;
  const double s = lo ? -t1 : t1;
  const double u = m2 ? (both ? 0.0 : s) : ca;
  const double v = one ? cb : (m2 ? (both ? t1 : cb) : (both ? cb : s));
  // U at the ends: 1 at a crossing, 2 at a clipped end, else from the root
  const bool u_split = m2 && !both, v_split = (m1 && !both) || (m2 && both);
  const double Uu = u_split ? 1.0 : (fabs(u) == t2 ? 2.0 : Q::sqrt_(fma(u, u, a2)));
  const double Uv = v_split ? 1.0 : (fabs(v) == t2 ? 2.0 : Q::sqrt_(fma(v, v, a2)));
  // regime weights: (1, 0) inner, (0, 1) outer, (2, -2) twice their difference
  const double mid = 0.5 * (ca + cb);
  const bool outer = one ? !(mid * mid < 1.0 - a2) : (m1 ? (both || lo) : (!both && !lo));
  const double w0 = (m2 && both) ? 2.0 : (outer ? 0.0 : 1.0);
  const double w1 = (m2 && both) ? -2.0 : (outer ? 1.0 : 0.0);
  const bool none = mode == 2 && one;
  cnt.n0 += !none && w0 != 0.0;
  cnt.n1 += !none && w0 == 0.0;
  const double r = piece<Q>(coef_mix(ad, p, w0, w1), ad, p, a2, u, Uu, v, Uv);
  return none ? 0.0 : r;
}

__device__ inline double item_value(const float4 it, int mode, EdgeCount &cnt) {
  const double ad = (double)fabsf(it.x), p = (double)fabsf(it.y), tA = (double)it.z, tB = (double)it.w;
  const double v = piece_of<PieceMixed>(ad, p, tA, tB, mode, cnt);
  return ((it.x < 0.0f) != (it.y < 0.0f)) ? -v : v;
}

// |d| int [H(U) - H(|d|)] dphi over the fan of one edge (p > 0, tA < tB),
// binary64 with the math library, in the difference form: the angle term
// from the span, the part within 2h as the edge kernel's pieces (two when
// the range crosses U = 1).  For cells small against the support, whose
// per-endpoint terms cancel far below the mixed cores' accuracy.
__device__ double edge_term_diff(double ad, double p, double tA, double tB, double dh, bool &integ, EdgeCount &cnt) {
  const double a2 = ad * ad + p * p;
  const double r2 = 4.0 - a2, s1 = 1.0 - a2;
  const double A2 = tA * tA, B2 = tB * tB;
  integ = (r2 > 0.0) && (tA < tB) && (tA < 0.0 || A2 < r2) && (tB > 0.0 || B2 < r2);
  double v = -dh * Math64::span(p, tA, tB);
  if (integ) {
    const bool lo = tA < 0.0 && A2 > s1 && (tB >= 0.0 || B2 < s1);
    const bool hi = (tA < 0.0 || A2 < s1) && tB > 0.0 && B2 > s1;
    if (s1 > 0.0 && (lo || hi))
      v += piece_of<Piece64>(ad, p, tA, tB, 1, cnt) + piece_of<Piece64>(ad, p, tA, tB, 2, cnt);
    else
      v += piece_of<Piece64>(ad, p, tA, tB, 0, cnt);
  }
  return v;
}

__device__ inline void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One face of a small cell's window in the binary64-geometry kernel.
struct SmallFace {
  double P0x, P0y, P0z;  // foot point of the particle on the face plane, about the generator
  double nx, ny, nz;     // unit normal
  double ad, dh;         // |d| / h and |d| H(|d|)
  const double *V;       // the face's vertices (binary64)
  int nv;                // vertex count; 0 for a face that adds nothing
  int off;               // its first edge among the window's edges
  int dpos;              // d > 0
  int flags;             // 1: an edge sees the foot point on or beyond it (p <= 0),
                         // 2: an edge through it (p = 0), 4: an edge within 2h
  double sum;            // the running sum of its edge terms, in edge order
};

// The faces [f - sub, f - sub + 16) of a cell small against the support,
// called by the 16 lanes of a group: binary64 geometry and the math
// library's functions in the difference form (the terms of a small face
// seen from afar cancel far below the binary32 geometry's and cores'
// accuracy), as face_fp64 evaluates them.  Lane sub sets up face f (the
// tests of face_mixed), the window's edges are taken 16 at a time, one per
// lane, and the first lane of each face's run in a round adds the run's
// terms to the face's running sum in edge order.  Returns face f's share
// of sum_f sgn(d_f) C_f (0 past f1 or for a face beyond the support).
// F, val and face_of are the group's LDS (16 entries each).
__device__ double small_window(int64_t f, int64_t f1, double xr0, double xr1, double xr2, double h, double ih,
                               const int64_t *fvo, const double4 *fplane, const double4 *fsphere, const double *fvpos,
                               bool &inside, bool &on_boundary, Counters &K, SmallFace *F, double *val,
                               int8_t *face_of, int sub) {
  SmallFace &me = F[sub];
  int nv = 0;
  if (f < f1) {
    const double4 pl = fplane[f];
    if (pl.w > 0.0) {
      const double dist = pl.w - (pl.x * xr0 + pl.y * xr1 + pl.z * xr2);
      if (dist < 0.0) inside = false;
      if (dist == 0.0) {
        on_boundary = true;
      } else if (fabs(dist) < 2.0 * h) {
        if (disk_within_2h(xr0, xr1, xr2, dist, h, fsphere[f])) {
          ++K.nf_int;
          const int64_t vs = fvo[f];
          nv = (int)(fvo[f + 1] - vs);
          const double d = dist * ih, ad = fabs(d);
          me.P0x = xr0 + dist * pl.x;
          me.P0y = xr1 + dist * pl.y;
          me.P0z = xr2 + dist * pl.z;
          me.nx = pl.x;
          me.ny = pl.y;
          me.nz = pl.z;
          me.ad = ad;
          me.dh = dH(ad);
          me.V = fvpos + 3 * vs;
          me.dpos = d > 0.0;
        }
      }
    }
  }
  // the faces' first edges: an inclusive scan of the edge counts over the group
  int incl = nv;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    const int y = __shfl_up(incl, o, 16);
    if (sub >= o) incl += y;
  }
  const int n_edge = __shfl(incl, 15, 16);
  me.nv = nv;
  me.off = incl - nv;
  me.flags = 0;
  me.sum = 0.0;
  wave_sync();
  for (int eb = 0; eb < n_edge; eb += 16) {
    const int e = eb + sub;
    int j = -1;
    bool has = false;
    double v = 0.0;
    if (e < n_edge) {
      // the face of edge e: the last window face starting at or before it
      // (faces without edges share their successor's start)
      int lo = 0, hi = 15;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (F[mid].off <= e) lo = mid;
        else hi = mid - 1;
      }
      j = lo;
      const SmallFace &fc = F[j];
      const int q = e - fc.off;
      const int q1 = (q + 1 == fc.nv) ? 0 : q + 1;
      const double *V = fc.V;
      const double Ax = V[3 * q], Ay = V[3 * q + 1], Az = V[3 * q + 2];
      const double Bx = V[3 * q1], By = V[3 * q1 + 1], Bz = V[3 * q1 + 2];
      const double abx = Bx - Ax, aby = By - Ay, abz = Bz - Az;
      const double len2 = abx * abx + aby * aby + abz * abz;
      int fl = 0;
      if (len2 != 0.0) {
        const double il = 1.0 / sqrt(len2);
        const double ex = abx * il, ey = aby * il, ez = abz * il;
        // in-plane normal of the edge pointing into the polygon: n x e
        const double mx = fc.ny * ez - fc.nz * ey, my = fc.nz * ex - fc.nx * ez, mz = fc.nx * ey - fc.ny * ex;
        const double p = ((fc.P0x - Ax) * mx + (fc.P0y - Ay) * my + (fc.P0z - Az) * mz) * ih;
        if (p <= 0.0) fl |= 1;
        if (p == 0.0) {
          fl |= 2;
        } else {
          ++K.ne_vis;
          const double tA = ((Ax - fc.P0x) * ex + (Ay - fc.P0y) * ey + (Az - fc.P0z) * ez) * ih;
          const double tB = ((Bx - fc.P0x) * ex + (By - fc.P0y) * ey + (Bz - fc.P0z) * ez) * ih;
          bool integ;
          const double t = edge_term_diff(fc.ad, fabs(p), tA, tB, fc.dh, integ, K.fd);
          if (integ) fl |= 4;
          K.ne_int += integ;
          v = p > 0.0 ? t : -t;
          has = true;
        }
      }
      if (fl) atomicOr(&F[j].flags, fl);
    }
    face_of[sub] = (int8_t)(j < 0 ? -1 : (has ? j : j + 16));
    val[sub] = v;
    wave_sync();
    // the first lane of each face's run in this round adds the run's terms
    auto face_at = [&](int t) { return face_of[t] < 0 ? -1 : (face_of[t] & 15); };
    if (j >= 0 && (sub == 0 || face_at(sub - 1) != j)) {
      double acc = F[j].sum;
      for (int t = sub; t < 16 && face_at(t) == j; ++t)
        if (face_of[t] < 16) acc += val[t];
      F[j].sum = acc;
    }
    wave_sync();
  }
  double r = 0.0;
  if (nv > 0) {
    double sum = me.sum;
    const int fl = me.flags;
    if (!(fl & 4) && !(fl & 2)) sum = -me.dh * ((fl & 1) ? 0.0 : 2.0 * kPi);
    const double Cf = sum * kInv4Pi;
    r = me.dpos ? Cf : -Cf;
  }
  wave_sync();  // every lane has read the window before the next one is set up
  return r;
}

// The pairs the edge-parallel kernel leaves to binary64 geometry, 16 lanes
// per pair (four pairs per wavefront).  A cell small against the support
// (every face reached, about five edges each) takes its faces 16 at a time:
// lane s sets up face s of the window, then the window's edges are dealt
// out 16 at a time, one per lane, and each face's terms are added in edge
// order by the first lane of its run; otherwise lane s takes the cell's
// faces s, s + 16, ... with all their edges.  Each round's 16 face shares
// go through LDS and the group's first lane adds them in face order, so
// either way every sum is the serial one.  Two workgroups per SIMD (at
// most 256 registers): one leaves the library's binary64 functions without
// latency hiding.
__global__ void __launch_bounds__(256, 2) k_exact_mixed_list(const int64_t *list, const int32_t *n_list,
                                                         const ExactInst *__restrict__ insts,
                                                         const int64_t *__restrict__ chunk0, int n_inst,
                                                         int64_t *counters) {
  __shared__ double share[16][16];
  __shared__ SmallFace sface[16][16];  // per group: the window's faces (small cells)
  __shared__ double sval[16][16];      // per group: this round's edge terms
  __shared__ int8_t sface_of[16][16];  // per group: the window face of each lane's edge (-1: none)
  const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int lane = threadIdx.x & 63;
  const uint64_t gmask = 0xffffull << (lane & 48);  // this group's lanes in the wave
  const int n = *n_list;
  for (int t = blockIdx.x * 16 + grp; t < n; t += gridDim.x * 16) {
    const int64_t gid = list[t];
    const int ins = inst_of(chunk0, n_inst, gid >> 6);
    const ExactInst &I = insts[ins];
    const int64_t k = gid - chunk0[ins] * 64;
    const int64_t c = I.pair_c[k];
    const int64_t i = I.pair_p[k];
    const double h = I.hh[i];
    const double ih = 1.0 / h;
    const float ihf = (float)ih;
    const double xr0 = I.xyz[3 * i] - I.gen[3 * c], xr1 = I.xyz[3 * i + 1] - I.gen[3 * c + 1],
                 xr2 = I.xyz[3 * i + 2] - I.gen[3 * c + 2];
    // particle about the generator, in units of h, binary32
    const float x0 = (float)(xr0 * ih), x1 = (float)(xr1 * ih), x2 = (float)(xr2 * ih);
    double acc = 0.0;
    bool inside = true, on_boundary = false;
    Counters K;
    const bool geo64 = (double)I.radius[c] < kSmallCell * h;
    const int64_t f0 = I.cfo[c], f1 = I.cfo[c + 1];
    for (int64_t fb = f0; fb < f1; fb += 16) {
      const int64_t f = fb + sub;
      double v = 0.0;
      if (geo64)
        v = small_window(f, f1, xr0, xr1, xr2, h, ih, I.fvo, I.fplane, I.fsphere, I.fvpos, inside, on_boundary, K,
                         sface[grp], sval[grp], sface_of[grp], sub);
      else if (f < f1)
        v = face_mixed(f, xr0, xr1, xr2, h, ih, ihf, x0, x1, x2, I.fvo, I.fplane, I.fplane32, I.fsphere, I.fvpos,
                       I.fvpos32, inside, on_boundary, K);
      share[grp][sub] = v;
      // a shared face this cell evaluates: its gift to the twin pair (same
      // particle, twin cell), replacing the edge kernel's
      if (I.gift && f < f1) {
        const int32_t sl = I.fcode[f];
        if (sl >= 0) {
          const int64_t cb = I.cell_off[c], nc = I.cell_off[c + 1] - cb;
          I.gift[I.gbase[c] + (int64_t)sl * nc + (k - cb)] = (long long)to_fixed(4.0 * kPi * v);
        }
      }
      wave_sync();
      if (sub == 0) {
        const int m = (int)min((int64_t)16, f1 - fb);
        for (int j = 0; j < m; ++j) acc += share[grp][j];
      }
      wave_sync();
    }
    // the group's inside (all faces) and boundary (any face) tests
    const bool all_in = (__ballot(!inside) & gmask) == 0ull;
    const bool any_on = (__ballot(on_boundary) & gmask) != 0ull;
    if (sub == 0) {
      double S = all_in ? 1.0 : 0.0;
      if (all_in && any_on) S = boundary_S(f0, f1, I.fplane, I.fvo, I.fvpos, xr0, xr1, xr2);
      I.w[k] = S - acc;
    }
    K.n64 = 0;  // counter 7 counts the pairs sent here, in the edge kernel
    if (counters) flush_counters(counters, sub == 0 ? f1 - f0 : 0, K);
  }
}

// Gift slots of each cell: its pairs times the shared faces it evaluates.
__global__ void k_gift_sizes(int64_t C, const int64_t *coff, const int32_t *cslots, int64_t *sz) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) sz[c] = (coff[c + 1] - coff[c]) * (int64_t)cslots[c];
}

// the number of set bits of m in the lanes below this one
__device__ inline int mbcnt64(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// A device-counted batch: gifts on while the instance's slots fit the
// capacity planned for them; else off (its faces are then evaluated from
// each side) and the plan flagged.
__global__ void k_gift_check(ExactInst *inst, const int64_t *total, int64_t cap, long long *gift, int32_t *flag) {
  if (threadIdx.x != 0) return;
  const bool fits = *total <= cap;
  inst->gift = fits ? gift : nullptr;
  if (!fits) *flag = 1;
}

// w = S - (own + received) / (4 pi) for every pair the edge kernel kept:
// its own total waits in w as a 64-bit integer until here.  One wavefront
// per cell takes its pairs kGatherW at a time (their particles in LDS).  The
// faces of the cell that a twin evaluates are listed first, with the twin's
// list and the face's gift run (both contiguous); their rows are then read
// kGatherU blocks of 64 at a time (loads in flight together), and each gift
// goes, with the opposite sign, to the pair of this cell with the same
// particle (bisection in LDS).  Integer sums: the order does not matter.
constexpr int kGatherW = 256;
constexpr int kGatherWaves = 4;
constexpr int kGatherU = 4;
__global__ void __launch_bounds__(64 * kGatherWaves) k_exact_gather(const ExactInst *__restrict__ insts, int ins,
                                                                    int64_t C) {
  __shared__ int32_t pl_[kGatherWaves][kGatherW];
  __shared__ unsigned long long ga_[kGatherWaves][kGatherW];
  __shared__ int64_t fcb_[kGatherWaves][64], fgs_[kGatherWaves][64];
  __shared__ int32_t fra_[kGatherWaves][64], frb_[kGatherWaves][64];
  const ExactInst &I = insts[ins];
  if (!I.gift) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t *const pl = pl_[wid];
  unsigned long long *const ga = ga_[wid];
  int64_t *const fcb = fcb_[wid], *const fgs = fgs_[wid];
  int32_t *const fra = fra_[wid], *const frb = frb_[wid];
  const int64_t *coff = I.cell_off;
  const int32_t *pair_p = I.pair_p;
  for (int64_t cp = (int64_t)blockIdx.x * kGatherWaves + wid; cp < C; cp += (int64_t)gridDim.x * kGatherWaves) {
    const int64_t b = coff[cp], n = coff[cp + 1] - b;
    const int64_t f0 = I.cfo[cp], nf = I.cfo[cp + 1] - f0;
    for (int64_t w0 = 0; w0 < n; w0 += kGatherW) {
      const int m = (int)min((int64_t)kGatherW, n - w0);
      for (int l = lane; l < m; l += 64) {
        pl[l] = pair_p[b + w0 + l];
        ga[l] = 0ull;
      }
      wave_sync();
      const int32_t i_lo = pl[0], i_hi = pl[m - 1];
      for (int64_t fw = 0; fw < nf; fw += 64) {
        const int64_t f = f0 + fw + lane;
        const int code = fw + lane < nf ? I.fcode[f] : 0;
        const bool inc = code <= -2;
        const uint64_t mk = __ballot(inc);
        if (inc) {
          const int pos = mbcnt64(mk);
          const int64_t tc = I.ftwin[f];
          const int64_t cb = coff[tc], nc = coff[tc + 1] - cb;
          fcb[pos] = cb;
          fgs[pos] = I.gbase[tc] + (int64_t)(-2 - code) * nc;
          // the twin's rows whose particles fall in this window's range
          // [i_lo, i_hi] (its list ascends by particle): all of them when the
          // cell takes one or two windows, else found by bisection, so that a
          // long list is not read once per window
          int32_t ra = 0, rb = (int32_t)nc;
          if (n > 2 * kGatherW) {
            int32_t lo = 0, hi = (int32_t)nc;
            while (lo < hi) {
              const int32_t mid = (lo + hi) >> 1;
              if (pair_p[cb + mid] < i_lo) lo = mid + 1;
              else hi = mid;
            }
            ra = lo;
            hi = (int32_t)nc;
            while (lo < hi) {
              const int32_t mid = (lo + hi) >> 1;
              if (pair_p[cb + mid] <= i_hi) lo = mid + 1;
              else hi = mid;
            }
            rb = lo;
          }
          fra[pos] = ra;
          frb[pos] = rb;
        }
        const int nin = __popcll(mk);
        wave_sync();
        int j = 0, r = 0;  // next block: rows fra[j] + [64 r, 64 r + 64) of face j's run
        while (j < nin) {
          int64_t gs[kGatherU], cb[kGatherU];
          bool uv[kGatherU];
#pragma unroll
          for (int u = 0; u < kGatherU; ++u) {
            const int jj = min(j, nin - 1);
            const int64_t t = fra[jj] + 64 * (int64_t)r + lane;
            uv[u] = j < nin && t < frb[jj];
            gs[u] = j < nin ? fgs[j] + t : 0;
            cb[u] = j < nin ? fcb[j] + t : 0;
            if (j < nin) {
              if (fra[j] + 64 * (r + 1) < frb[j]) {
                ++r;
              } else {
                ++j;
                r = 0;
              }
            }
          }
          long long T[kGatherU];
          int32_t ip[kGatherU];
#pragma unroll
          for (int u = 0; u < kGatherU; ++u) {
            T[u] = uv[u] ? I.gift[gs[u]] : 0;
            ip[u] = uv[u] ? pair_p[cb[u]] : 0;
          }
#pragma unroll
          for (int u = 0; u < kGatherU; ++u) {
            if (T[u] != 0 && ip[u] >= i_lo && ip[u] <= i_hi) {
              int lo = 0, hi = m;
              while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (pl[mid] < ip[u]) lo = mid + 1;
                else hi = mid;
              }
              if (lo < m && pl[lo] == ip[u]) atomicAdd(&ga[lo], (unsigned long long)(-T[u]));
            }
          }
        }
        wave_sync();
      }
      for (int l = lane; l < m; l += 64) {
        const int64_t jj = b + w0 + l;
        const uint8_t fl = I.wflag[jj];
        if (!(fl & kFlagRedo)) {
          const unsigned long long tot = (unsigned long long)__double_as_longlong(I.w[jj]) + ga[l];
          I.w[jj] = ((fl & kFlagInside) ? 1.0 : 0.0) - kInv4Pi * from_fixed(tot);
        }
      }
      wave_sync();
    }
  }
}

// ------------------------------------ edge-parallel wave kernel (mixed)
// A wavefront takes 64 consecutive pairs (one per lane) from a work counter.
//   A1 (lane = pair): the cull over the cell's faces (plane distance, and
//      the distance from the face's bounding disk in its plane against 2h),
//      kept as a bit mask; the faces within
//      reach are listed pair-major with their foot point, |d| and
//      |d| H(|d|); the chunk's edges are numbered in the same order, and a
//      bit in LDS marks where each listed face's edges begin;
//   A2 (lane = edge): the wave walks those edges 64 at a time; each lane
//      finds its face from the start bits (a population count) and forms
//      its edge's in-plane geometry from the precomputed edge frame,
//      adds the angle term -dh (phi_B - phi_A) to its pair, and queues the
//      edge in LDS when it comes within 2h (one queue for ranges crossing
//      U = 1, one for the others);
//   B  (lane = item): whenever a queue holds 64 items the wave evaluates
//      them together, so every lane runs the same closed form.
// Each pair's terms are added as 64-bit fixed-point integers (2^-46) with
// LDS atomics: integer sums do not depend on order, so a weight is a
// function of its own pair alone and repeats bit for bit.  Pairs with more
// than 64 faces, more candidate edges than a chunk slot holds, or that need
// binary64 geometry are listed for the redo kernel (16 lanes per pair).
constexpr int kMaxFaces = 64;              // faces per cell handled here
constexpr int kEntryCap = 64 * kMaxFaces;  // face entries per chunk
constexpr int kEdgeCap = 256;              // candidate edges per pair handled here
constexpr int kQueue = 192;                // items in the LDS queue (a batch adds at most 128)
constexpr int kRing = 128;                 // face records whose sums are open at once
static_assert(kEntryCap <= 4096, "an item names its record in 12 bits");

struct __align__(16) FaceRec {  // a face within reach of a pair
  float px, py, pz;  // foot point about the generator (absolute units)
  float df;          // signed |d| / h, binary32
  double dhs;        // -sign(d) |d| H(|d|) 2^46, sign(0) = -1: the angle
                     // term's factor in fixed-point units
  float ihf;         // 1/h of the pair (binary32)
  uint32_t slot;     // bits 0-23: first vertex slot - the chunk's first; 24-29: lane of the
                     // pair; 31: the foot point is far outside the face (kFarFoot)
};
constexpr int64_t kSlotSpan = 1 << 24;  // vertex slots a chunk's faces may span
constexpr uint32_t kFarBit = 1u << 31;    // record flag: the foot point is far outside the face
// A face whose foot point lies farther than this (in units of h) beyond the
// face's bounding sphere takes its exact angle part, 0: the per-edge angle
// terms of such a face sum to 0 in exact arithmetic, but each is of the size
// of |d| H(|d|) (near 1 for a plane that passes close to the particle) and
// carries the binary32 geometry's rounding, while the face's true
// contribution, from the part of the fan within 2h, may be orders smaller.
constexpr double kFarFoot = 0.1;
static_assert(sizeof(FaceRec) == 32, "records are addressed as index << 5");

struct EdgeData {  // what one lane reads for its edge: face record and edge geometry
  FaceRec fc;
  float4 ea, ee, em;
  int rec;  // index of the face record
};

struct Sphere {
  double x, y, z, r;
};

struct EdgeWave {  // per-wavefront LDS
  union {
    double4 wpl[64];  // cull and face list: window of the chunk's faces: plane
    struct {          // edge walk: each pair's gift run (start and stride)
      long long gb[64], gn[64];
    };
  };
  union {
    Sphere wsp[64];               // cull: the window's bounding spheres
    unsigned long long sb[kEdgeCap];  // edge walk: bit g set where a face's edges start (64 kEdgeCap bits)
  };
  // cull and face list: the window's first vertex slot, twin cell (-1: none)
  // and vertex count (at most 128)
  int wvs[64];
  int wtw[64];
  unsigned char wnv[64];
  unsigned long long acc[64];  // per pair: the total of its own face records
  // items: edge data, and the record (bits 0-11) and mode (bits 12-13)
  float4 q[kQueue];
  uint16_t o[kQueue];
  // open face records, slot r mod kRing: the fixed-point sum of record r's
  // terms, whether an edge of it comes within 2h, and whether an edge sees
  // its foot point on the outer side (p < 0: the foot point lies outside
  // the polygon)
  unsigned long long racc[kRing];
  unsigned char rint[kRing], rnin[kRing];
  unsigned char redo[64];  // the pair is left to the redo kernel
};

template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

// a value the whole wave holds alike, moved to scalar registers
__device__ inline int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline float4 load4(gptr<float4> p, int64_t i) {
  const gptr<float> q = (gptr<float>)(p + i);
  return make_float4(q[0], q[1], q[2], q[3]);
}

__device__ inline float4 load4(gptr<float4> p, uint32_t i) {
  const gptr<float> q = (gptr<float>)((gptr<char>)p + (i << 4));  // i < 2^28
  return make_float4(q[0], q[1], q[2], q[3]);
}

__device__ inline double4 load4(gptr<double4> p, int64_t i) {
  const gptr<double> q = (gptr<double>)(p + i);
  return make_double4(q[0], q[1], q[2], q[3]);
}

// face record rec of a wave's region (a 32-bit byte offset from its base)
__device__ inline FaceRec load_rec(gptr<FaceRec> base, int rec) {
  const gptr<float> q = (gptr<float>)((gptr<char>)base + ((uint32_t)rec << 5));
  FaceRec r;
  r.px = q[0];
  r.py = q[1];
  r.pz = q[2];
  r.df = q[3];
  r.dhs = *(gptr<double>)(q + 4);
  r.ihf = q[6];
  r.slot = *(gptr<uint32_t>)(q + 7);
  return r;
}


__device__ inline uint64_t lanes_in(int lo, int hi) {  // bits [lo, hi), 0 <= lo <= hi <= 64
  const uint64_t a = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
  const uint64_t b = lo >= 64 ? ~0ull : ((1ull << lo) - 1ull);
  return a & ~b;
}

// Evaluate the first n (<= 64) queued items and add them to their records;
// move the rest (at most kQueue - 64) to the front.  Returns the new length.
__device__ inline int drain(EdgeWave &L, int len, int n, int lane, EdgeCount &cnt) {
  if (lane < n) {
    const int o = L.o[lane];
    const double r = item_value(L.q[lane], o >> 12, cnt);
    atomicAdd(&L.racc[o & (kRing - 1)], to_fixed(r));
  }
  const int rest = len - n;
  const bool ha = lane < rest, hb = lane + 64 < rest;
  float4 a = {}, b = {};
  uint16_t oa = 0, ob = 0;
  if (ha) {
    a = L.q[n + lane];
    oa = L.o[n + lane];
  }
  if (hb) {
    b = L.q[n + 64 + lane];
    ob = L.o[n + 64 + lane];
  }
  wave_sync();  // every read before any write
  if (ha) {
    L.q[lane] = a;
    L.o[lane] = oa;
  }
  if (hb) {
    L.q[64 + lane] = b;
    L.o[64 + lane] = ob;
  }
  wave_sync();
  return rest;
}

template <bool kCount>
// Four waves per SIMD (128 VGPRs; 4 workgroups of 39 KB LDS per CU): the
// few values that spill are the chunk's and the fetch's, stored and reloaded
// outside the edge walk and the queue evaluation.
__global__ void __launch_bounds__(64 * kFlatWaves, 4) k_exact_edges(
    const ExactInst *__restrict__ insts, const int64_t *__restrict__ chunk0, int n_inst, int per_fetch,
    int64_t *counters, FaceRec *faces, int32_t *rec_slot, int32_t *next_chunk, int64_t *redo, int32_t *n_redo) {
  __shared__ EdgeWave lds[kFlatWaves];
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  EdgeWave &L = lds[wid];
  const int64_t wave = (int64_t)blockIdx.x * kFlatWaves + wid;
  FaceRec *const fr = faces + wave * kEntryCap;
  int32_t *const rtw = rec_slot + wave * kEntryCap;
  const int64_t n_chunks = chunk0[n_inst];
  Counters K;
  int64_t nfaces = 0;
  const int home = blockIdx.x % kXcd;
  int vict = 0;  // eighths tried after this XCD's own
  while (true) {
    const int x = (home + vict) % kXcd;
    const int64_t lo = n_chunks * x / kXcd, hi = n_chunks * (x + 1) / kXcd;
    int gbase = 0;
    if (lane == 0) gbase = atomicAdd(next_chunk + x * kCtrStride, per_fetch);
    gbase = __builtin_amdgcn_readfirstlane(gbase);  // uniform: chunk state in scalar registers
    if (lo + gbase >= hi) {
      if (++vict == kXcd) break;
      continue;
    }
    const int64_t gend = min(lo + gbase + per_fetch, hi);
    gbase = (int)(lo + gbase);
    for (int64_t gchunk = gbase; gchunk < gend; ++gchunk) {
    const int ins = inst_of(chunk0, n_inst, gchunk);
    const ExactInst &I = insts[ins];
    // all instance arrays through global pointers (see the edge arrays below):
    // generic loads could alias LDS and would be ordered against its stores
    const gptr<int32_t> pair_c = (gptr<int32_t>)I.pair_c, pair_p = (gptr<int32_t>)I.pair_p;
    const gptr<double> xyz = (gptr<double>)I.xyz, hh = (gptr<double>)I.hh, gen = (gptr<double>)I.gen;
    const gptr<int64_t> cfo = (gptr<int64_t>)I.cfo, fvo = (gptr<int64_t>)I.fvo;
    const gptr<double4> fplane = (gptr<double4>)I.fplane, fsphere = (gptr<double4>)I.fsphere;
    // global (not generic) address space: the loads then count only against
    // the vector-memory counter and never hold up waits on LDS traffic
    const gptr<float4> edgeA = (gptr<float4>)I.edgeA, edgeE = (gptr<float4>)I.edgeE, edgeM = (gptr<float4>)I.edgeM;
    const gptr<int32_t> fcode = (gptr<int32_t>)I.fcode;
    const bool shared = I.gift != nullptr;  // the same for the whole wave
    const int64_t P = I.P;
    const int64_t chunk = gchunk - chunk0[ins];
    const int64_t k = chunk * 64 + lane;
    const bool valid = k < P;
    // ---------------- A1: cull
    // The chunk's pairs are sorted by cell, so their faces are one range
    // [F0, F1); it is staged through LDS 64 faces at a time.
    const int64_t k_last = min(chunk * 64 + 63, P - 1);
    const int64_t F0 = uniform64(cfo[pair_c[chunk * 64]]), F1 = uniform64(cfo[pair_c[k_last] + 1]);
    // vertex slots of the chunk's faces, kept relative to the first in 24 bits
    const int64_t VB = uniform64(fvo[F0]);
    const bool wide = fvo[F1] - VB > kSlotSpan;
    uint64_t mask = 0, farmask = 0;
    int nsurv = 0, nedge = 0;
    bool inside = true, on_boundary = false, again = false;
    int64_t f0 = 0, f1 = 0, c = 0;
    double xr0 = 0.0, xr1 = 0.0, xr2 = 0.0, ih = 0.0, h = 0.0;
    if (valid) {
      if (wide) again = true;
      c = pair_c[k];
      const int64_t i = pair_p[k];
      h = hh[i];
      ih = 1.0 / h;
      xr0 = xyz[3 * i] - gen[3 * c];
      xr1 = xyz[3 * i + 1] - gen[3 * c + 1];
      xr2 = xyz[3 * i + 2] - gen[3 * c + 2];
      f0 = cfo[c];
      f1 = cfo[c + 1];
      nfaces += f1 - f0;
      if (f1 - f0 > kMaxFaces) again = true;
      if ((double)((gptr<float>)I.radius)[c] < kSmallCell * h) again = true;  // binary64 geometry
    }
    for (int64_t wb = F0; wb < F1; wb += 64) {
      {
        const int64_t f = wb + lane;
        if (f < F1) {
          L.wpl[lane] = load4(fplane, f);
          const double4 sph = load4(fsphere, f);
          L.wsp[lane] = Sphere{sph.x, sph.y, sph.z, sph.w};
          const int64_t vs = fvo[f];
          L.wvs[lane] = (int)vs;
          L.wnv[lane] = (unsigned char)(fvo[f + 1] - vs);
          L.wtw[lane] = shared ? fcode[f] : -1;
        }
      }
      wave_sync();
      if (valid && !again) {
        const int64_t ja = max(f0, wb) - wb, jb = min(f1, wb + 64) - wb;
        // branch-free over the faces: a degenerate face sets again, which
        // discards the pair's list, so the loop need not stop there
        for (int64_t j = ja; j < jb; ++j) {
          const double4 pl = L.wpl[j];
          const Sphere sp = L.wsp[j];
          const bool real = pl.w > 0.0;
          const double dist = pl.w - (pl.x * xr0 + pl.y * xr1 + pl.z * xr2);
          inside &= !(real & (dist < 0.0));
          on_boundary |= real & (dist == 0.0);
          const double sx = xr0 - sp.x, sy = xr1 - sp.y, sz = xr2 - sp.z;
          // the sphere's centre lies in the face plane, so the foot point's
          // squared distance from it is s2 - dist^2
          const double rho2 = (sx * sx + sy * sy + sz * sz) - dist * dist;
          // The face's polygon lies in the disk of the sphere's radius about
          // that centre, so the particle's distance from the disk,
          // sqrt(dist^2 + max(rho - R, 0)^2), bounds its distance from the
          // polygon from below; a face farther than 2h adds exactly 0.  rho
          // is taken in binary32 and rounded down, so that no face within
          // reach is dropped.
          const double rho = (double)__builtin_sqrtf((float)fmax(rho2, 0.0)) * (1.0 - 1e-6);
          const double t = fmax(rho - sp.r, 0.0);
          // a shared face is evaluated by the lower-numbered of its two
          // cells, for both pairs of the particle
          const bool mine = L.wtw[j] >= -1;
          const bool near = real & mine & (dist != 0.0) & (fabs(dist) < 2.0 * h) & (dist * dist + t * t < 4.0 * h * h);
          // a foot point beyond the sphere by kFarFoot h is outside the
          // polygon and clear of its vertices
          const double rf = sp.r + kFarFoot * h;
          const bool far = rho2 > rf * rf;
          const bool deg = near & (fabs(dist * ih) < kOnPlane);
          again |= deg;
          const bool keep = near & !deg & (L.wnv[j] > 0);  // a face without edges adds nothing
          mask |= (uint64_t)keep << (wb + j - f0);
          farmask |= (uint64_t)(keep & far) << (wb + j - f0);
          nsurv += keep;
          nedge += keep ? L.wnv[j] : 0;
        }
      }
      wave_sync();
    }
    if (valid) {
      again |= nedge > kEdgeCap || (inside && on_boundary);
      if (again) {
        mask = 0;
        nsurv = nedge = 0;
      }
    }
    // the pair's gift run: slot q of its cell at gbl + q gnl, each set to
    // 0 here and to the face's total when its record closes (the redo
    // kernel rewrites them for the pairs it recomputes)
    long long gbl = 0, gnl = 0;
    if (shared && valid) {
      const gptr<int64_t> coff = (gptr<int64_t>)I.cell_off;
      const int64_t cb = coff[c];
      gnl = coff[c + 1] - cb;
      gbl = ((gptr<int64_t>)I.gbase)[c] + (k - cb);
      const int ns = ((gptr<int32_t>)I.cslots)[c];
      for (int q = 0; q < ns; ++q) I.gift[gbl + (int64_t)q * gnl] = 0;
    }
    const int e_off = wave_scan_excl(nsurv, lane);
    const int x_off = wave_scan_excl(nedge, lane);
    // wave-uniform counts in scalar registers (the edge walk's loop bound)
    const int n_edge = __builtin_amdgcn_readlane(x_off + nedge, 63);
    const int n_rec = __builtin_amdgcn_readlane(e_off + nsurv, 63);
    L.acc[lane] = 0ull;
    L.redo[lane] = again ? 1 : 0;
    L.racc[lane] = 0ull;
    L.racc[lane + 64] = 0ull;
    L.rint[lane] = L.rint[lane + 64] = 0;
    L.rnin[lane] = L.rnin[lane + 64] = 0;
    if (kCount) K.nf_int += nsurv;
    // the start bits of the chunk's edges, n_edge <= 64 kEdgeCap of them
    for (int w = lane; w < (n_edge + 63) >> 6; w += 64) L.sb[w] = 0ull;
    wave_sync();
    // ---------------- A1b: the face list, pair-major, and where each face's edges start
    {
      int e = e_off, start = x_off;
      for (int64_t wb = F0; wb < F1; wb += 64) {
        if (F1 - F0 > 64) {  // a single window is still staged from the cull
          const int64_t f = wb + lane;
          if (f < F1) {
            L.wpl[lane] = load4(fplane, f);
            const int64_t vs = fvo[f];
            L.wvs[lane] = (int)vs;
            L.wnv[lane] = (unsigned char)(fvo[f + 1] - vs);
            L.wtw[lane] = shared ? fcode[f] : -1;
          }
        }
        wave_sync();
        const int64_t ja = max(f0, wb) - wb, jb = min(f1, wb + 64) - wb;
        if (mask && ja < jb) {
          uint64_t m = mask & lanes_in((int)(wb + ja - f0), (int)(wb + jb - f0));
          while (m) {
            const int bit = __builtin_ctzll(m);
            const int j = (int)(bit - (wb - f0));
            m &= m - 1;
            const double4 pl = L.wpl[j];
            const double dist = pl.w - (pl.x * xr0 + pl.y * xr1 + pl.z * xr2);
            // |d| rounded to binary32, like the rest of the face's geometry
            const float df = (float)(dist * ih);
            FaceRec rec;
            rec.px = (float)(xr0 + dist * pl.x);
            rec.py = (float)(xr1 + dist * pl.y);
            rec.pz = (float)(xr2 + dist * pl.z);
            rec.df = df;
            const double dh = dH((double)fabsf(df));
            rec.dhs = (df > 0.0f ? -dh : dh) * 0x1p46;
            rec.ihf = (float)ih;
            // a face whose foot point is far outside it: its angle part is
            // exactly 0, so its edges add no angle terms
            const uint32_t fb = (uint32_t)((farmask >> bit) & 1ull) << 31;
            rec.slot = (uint32_t)(L.wvs[j] - VB) | ((uint32_t)lane << 24) | fb;
            fr[e] = rec;
            if (shared) rtw[e] = L.wtw[j];  // the face's gift slot, or -1
            atomicOr(&L.sb[start >> 6], 1ull << (start & 63));
            ++e;
            start += L.wnv[j];
          }
        }
        wave_sync();
      }
    }
    wave_fence();
    L.gb[lane] = gbl;  // the plane window is done with
    L.gn[lane] = gnl;
    wave_sync();
    // ---------------- A2: one edge per lane; B whenever the queue fills
    int qn = 0;    // queued items
    int done = 0;  // records below this are closed
    // the rounding constant of fixed_from in scalar registers (otherwise
    // rebuilt in vector registers for every batch)
    uint32_t magic_hi;
    asm volatile("s_mov_b32 %0, 0x43380000" : "=s"(magic_hi));
    const double magic = __hiloint2double((int)magic_hi, 0);
    const gptr<FaceRec> frg = (gptr<FaceRec>)fr;
    // Close records [done, upto): each one's total -- the sum of its terms,
    // or, when no edge of it came within 2h, its exact angle sum 2 pi [foot
    // point inside] times its factor (a face clear of the support adds
    // exactly 0) -- is added to its pair and, for a shared face, written to
    // the pair's gift slot; its ring slot is cleared for reuse.
    auto retire = [&](int upto) {
      while (done < upto) {
        const int r = done + lane;
        if (r < upto) {
          const int sl = r & (kRing - 1);
          const FaceRec rc = load_rec(frg, r);
          const long long T = L.rint[sl] ? (long long)L.racc[sl]
                                         : (L.rnin[sl] ? 0ll : (long long)fixed_from(fma(rc.dhs, 2.0 * kPi, magic)));
          const int ow = (int)((rc.slot >> 24) & 63u);
          atomicAdd(&L.acc[ow], (unsigned long long)T);
          if (shared) {
            const int q = rtw[r];
            if (q >= 0) I.gift[L.gb[ow] + (int64_t)q * L.gn[ow]] = T;  // after its 0: same wave, in order
          }
          L.racc[sl] = 0ull;
          L.rint[sl] = 0;
          L.rnin[sl] = 0;
        }
        done = min(done + 64, upto);
        wave_sync();
      }
    };
    // Evaluate batch [b, b + 64) from the data d fetched for it; `walked`
    // is the first record with an edge past the batch (n_rec after the last).
    auto batch = [&](int b, const EdgeData &d, int walked) {
      const int g = b + lane;
      const bool live = g < n_edge;
      // The batch touches records [first, last]; their ring slots must not
      // hold records still open (an item of record r may wait in the queue):
      // when they would, everything queued is evaluated and the records
      // before this batch are closed first.
      {
        const int first = __builtin_amdgcn_readfirstlane(d.rec);
        const int last = __builtin_amdgcn_readlane(d.rec, 63);
        if (last >= done + kRing) {
          while (qn > 0) qn = drain(L, qn, min(qn, 64), lane, K.fd);
          retire(first);
        }
      }
      const int sl = d.rec & (kRing - 1);
      const FaceRec &fc = d.fc;
      const float4 EA = d.ea, EE = d.ee, EM = d.em;
      // Branch-free: nearly every lane has a live edge of positive length at
      // a nonzero distance, so every lane does the arithmetic (the clamped
      // loads keep it finite) and the tests only select what is kept.
      const int owner = (int)((fc.slot >> 24) & 63u);
      const bool far = (fc.slot & kFarBit) != 0u;
      const float dx = fc.px - EA.x, dy = fc.py - EA.y, dz = fc.pz - EA.z;
      const float p = (dx * EM.x + dy * EM.y + dz * EM.z) * fc.ihf;
      // an edge of positive length whose line passes within 1e-2 h of the
      // particle (d^2 + p^2), or whose foot point lies on its line (p = 0),
      // needs binary64 geometry: the pair goes to the redo kernel
      const bool act = live & (EA.w > 0.0f);
      const bool degen = act & ((p == 0.0f) | (fmaf(fc.df, fc.df, p * p) < kEdgeNear * kEdgeNear));
      if (degen) L.redo[owner] = 1;
      const bool ok = act & !degen;
      // the foot point is outside the record's polygon if any edge sees it
      // on its outer side
      if (ok & (p < 0.0f)) L.rnin[sl] = 1;
      const float tA = -(dx * EE.x + dy * EE.y + dz * EE.z) * fc.ihf;
      const float tB = fmaf(EA.w, fc.ihf, tA);
      const double ap = (double)fabsf(p), dA = (double)tA, dB = (double)tB;
      const double ad = (double)fabsf(fc.df);
      // the angle term -dh (phi_B - phi_A), negated when the edge and the
      // face are oriented oppositely (p and d of unequal signs): the record's
      // factor takes the sign bit of p (p != 0 here) and feeds one fma
      const double f = __hiloint2double(__double2hiint(fc.dhs) ^ (int)(__float_as_uint(p) & 0x80000000u),
                                        __double2loint(fc.dhs));
      if (ok & !far) atomicAdd(&L.racc[sl], fixed_from(fma(MathMixed::span(ap, dA, dB), f, magic)));
      // within 2h somewhere on [tA, tB], and crossing U = 1 (squares, no
      // roots; bitwise logic, so that no test becomes a branch)
      const double a2 = ad * ad + ap * ap;
      const double r2 = 4.0 - a2, s1 = 1.0 - a2;
      const double A2 = dA * dA, B2 = dB * dB;
      const bool integ = ok & (r2 > 0.0) & (dA < dB) & ((dA < 0.0) | (A2 < r2)) & ((dB > 0.0) | (B2 < r2));
      const bool lo = (dA < 0.0) & (A2 > s1) & ((dB >= 0.0) | (B2 < s1));
      const bool hi = ((dA < 0.0) | (A2 < s1)) & (dB > 0.0) & (B2 > s1);
      const bool cross = (s1 > 0.0) & (lo | hi);
      if (kCount) {
        K.ne_vis += ok;
        K.ne_int += integ;
      }
      // one item per edge within 2h, two for a range crossing U = 1
      const float4 it = make_float4(fc.df, p, tA, tB);
      const uint64_t m1 = __ballot(integ), m2 = __ballot(integ && cross);
      if (integ) {
        L.rint[sl] = 1;
        // set bits of the scalar masks below this lane, counted in hardware
        const int pos = qn + mbcnt64(m1) + mbcnt64(m2);
        L.q[pos] = it;
        L.o[pos] = (uint16_t)(d.rec | (cross ? 1 << 12 : 0));
        if (cross) {
          L.q[pos + 1] = it;
          L.o[pos + 1] = (uint16_t)(d.rec | (2 << 12));
        }
      }
      qn += __popcll(m1) + __popcll(m2);
      wave_sync();
      while (qn >= 64) qn = drain(L, qn, 64, lane, K.fd);
      // records before both the next batch and the oldest queued item are
      // complete: close them a full round at a time
      int front = walked;
      if (qn > 0) front = min(front, (int)__builtin_amdgcn_readfirstlane(L.o[0] & 0xfff));
      if (front - done >= 64) retire(done + ((front - done) & ~63));
    };
    // Edge g of the chunk belongs to the last face record starting at or
    // before g: batch [bb, bb + 64) reads one word of start bits, and a lane
    // counts the starts at or below it.  cnt (records starting before bb)
    // and qc (the offset of edge bb within its record) carry over.  Lanes
    // past n_edge take the last record's first edge, so every load stays in
    // bounds.
    int cnt = 0, qc = 0;
    auto locate = [&](int bb, int &rec, int &vq) {
      // the same word in every lane; past n_edge (look-ahead) its bits are unused
      const unsigned long long w = L.sb[min(bb >> 6, kEdgeCap - 1)];
      const unsigned long long S = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(w >> 32)) << 32) |
                                   (unsigned)__builtin_amdgcn_readfirstlane((unsigned)w);
      const unsigned long long upto = S & lanes_in(0, lane + 1);
      const bool in = bb + lane < n_edge;
      // the last start at or below this lane, or -qc when the edge's face began in an earlier batch
      const int hb = 63 - __builtin_clzll(upto | 1ull), none = upto == 0ull;
      const int last = hb - none * (hb + qc);  // arithmetic select: no branch
      rec = in ? cnt + __popcll(upto) - 1 : n_rec - 1;
      vq = in ? lane - last : 0;
      cnt += __popcll(S);
      qc = S ? __builtin_clzll(S) + 1 : qc + 64;
    };
    // Two-stage pipeline: while batch b is evaluated, the records and edge
    // data of batch b + 1 and the packed vertex slots of batch b + 2 are in
    // flight.  The loads are unconditional (lanes past n_edge fetch valid
    // but unused data), so no loaded register is merged or copied before the
    // loop's next turn; a copy would wait for its load.
    // the chunk's edge frames and the wave's face records from scalar bases
    // and 32-bit offsets (a chunk spans fewer than 2^24 slots, a wave holds
    // 4096 records)
    const gptr<float4> cA = edgeA + VB, cE = edgeE + VB, cM = edgeM + VB;
    auto fetch = [&](int rec, int vq, uint32_t slot, EdgeData &d) {
      d.rec = rec;
      d.fc = load_rec(frg, rec);
      const uint32_t v = (slot & 0xffffffu) + (uint32_t)vq;
      d.ea = load4(cA, v);
      d.ee = load4(cE, v);
      d.em = load4(cM, v);
    };
    auto slot_of = [&](int rec) { return *(gptr<uint32_t>)((gptr<char>)frg + ((uint32_t)rec << 5) + 28); };
    // one turn: evaluate batch b from `cur` while batch b + 64 is fetched
    // into `nxt` (record and slot in r, q, sl) and the record and slot of
    // batch b + 128 are found (into rn, qn, sn).  The loop below alternates
    // the roles of the two sets, so no loaded register is copied.
    auto turn = [&](int b, const EdgeData &cur, EdgeData &nxt, int r, int q, uint32_t sl, int &rn, int &qn_,
                    uint32_t &sn) {
      locate(b + 128, rn, qn_);
      sn = slot_of(rn);
      fetch(r, q, sl, nxt);
      batch(b, cur, b + 64 < n_edge ? __builtin_amdgcn_readfirstlane(r) : n_rec);
    };
    EdgeData dX{}, dY{};
    int rX = 0, qX = 0, rY = 0, qY = 0;
    uint32_t sX = 0, sY = 0;
    if (n_edge > 0) {
      int r0, q0;
      locate(0, r0, q0);
      fetch(r0, q0, slot_of(r0), dX);
      locate(64, rX, qX);
      sX = slot_of(rX);
    }
    for (int b = 0; b < n_edge; b += 128) {
      turn(b, dX, dY, rX, qX, sX, rY, qY, sY);
      if (b + 64 >= n_edge) break;
      turn(b + 64, dY, dX, rY, qY, sY, rX, qX, sX);
    }
    while (qn > 0) qn = drain(L, qn, min(qn, 64), lane, K.fd);
    retire(n_rec);
    wave_sync();
    if (valid && !again && L.redo[lane] == 0) {
      if (shared) {
        // the own total until k_exact_gather adds what the twins gave
        I.w[k] = __longlong_as_double((long long)L.acc[lane]);
        I.wflag[k] = inside ? kFlagInside : 0;
      } else {
        I.w[k] = (inside ? 1.0 : 0.0) - kInv4Pi * from_fixed(L.acc[lane]);
      }
    } else if (valid) {
      if (kCount) ++K.n64;  // a pair left to the binary64 kernel
      if (shared) I.wflag[k] = kFlagRedo;
      redo[atomicAdd(n_redo, 1)] = gchunk * 64 + lane;
    }
    wave_fence();
    }  // chunks of this fetch
  }
  if (kCount) flush_counters(counters, nfaces, K);
}

}  // namespace

struct GiftPlan {
  int64_t *gbase = nullptr, *gsize = nullptr;
  long long *gift = nullptr;
  uint8_t *wflag = nullptr;
  std::vector<int64_t> gb_off, gift_off, flag_off, cap;  // per instance (-1: no gifts)
  bool any = false;
};

// Where the gifts of shared faces go (mixed path): per instance, the start
// of its cell offsets, gift slots and flags in one buffer each.  Instances
// whose grid has no shared face take none.  The slot counts are read back
// (the host knows the pair counts here); `headroom` > 0 plans capacity for
// a device-counted batch (its counts change from step to step).
static GiftPlan gift_plan(Ctx &ctx, Arena &mem, const std::vector<ExactJob> &jobs, bool use_cap, double headroom,
                          hipStream_t s) {
  GiftPlan G;
  const int n = (int)jobs.size();
  G.gb_off.assign(n, -1);
  G.gift_off.assign(n, -1);
  G.flag_off.assign(n, -1);
  G.cap.assign(n, 0);
  int64_t nb = 0, nf = 0;
  for (int k = 0; k < n; ++k) {
    const int64_t np = use_cap ? jobs[k].P->cap : jobs[k].P->n_pairs;
    if (jobs[k].t->face_code && np > 0) {
      G.gb_off[k] = nb;
      G.flag_off[k] = nf;
      nb += jobs[k].t->n_cells + 1;
      nf += np;
      G.any = true;
    }
  }
  if (!G.any) return G;
  G.gbase = mem.get<int64_t>("gift_base", nb);
  G.gsize = mem.get<int64_t>("gift_size", nb);
  G.wflag = mem.get<uint8_t>("gift_flag", nf);
  std::vector<int64_t> tot(n, 0);
  for (int k = 0; k < n; ++k) {
    if (G.gb_off[k] < 0) continue;
    const TessDev &t = *jobs[k].t;
    k_gift_sizes<<<(unsigned)div_up(t.n_cells, 256), 256, 0, s>>>(t.n_cells, jobs[k].P->cell_off, t.cell_slots,
                                                                  G.gsize + G.gb_off[k]);
    SPH_LAUNCH_CHECK();
    scan_exclusive_i64(ctx.arena, G.gsize + G.gb_off[k], G.gbase + G.gb_off[k], t.n_cells, true, s);
    SPH_HIP(hipMemcpyAsync(&tot[k], G.gbase + G.gb_off[k] + t.n_cells, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  }
  SPH_HIP(hipStreamSynchronize(s));
  int64_t ng = 0;
  for (int k = 0; k < n; ++k)
    if (G.gb_off[k] >= 0) {
      G.gift_off[k] = ng;
      G.cap[k] = tot[k] + (headroom > 0.0 ? std::max<int64_t>((int64_t)((double)tot[k] * headroom), 1 << 16) : 0);
      ng += G.cap[k];
    }
  G.gift = mem.get<long long>("gift", std::max<int64_t>(ng, 1));
  return G;
}

// one instance's table entry (G: null, or the gifts of its shared faces)
static ExactInst inst_of_job(const ExactJob &j, const GiftPlan *G, int k) {
  const TessDev &t = *j.t;
  const PartDev &p = *j.p;
  const PairsDev &P = *j.P;
  const bool sh = G && G->gb_off[k] >= 0;
  return ExactInst{P.pair_c, P.pair_p, p.xyz, p.h, t.gen, t.radius, t.cell_face_off, t.face_vtx_off, t.fplane,
                   t.fsphere, t.fplane32, t.fvpos32, t.edgeA, t.edgeE, t.edgeM, t.fvpos, P.w, P.n_pairs,
                   P.cell_off, sh ? t.face_code : nullptr, sh ? t.cell_slots : nullptr, sh ? t.face_twin : nullptr,
                   sh ? G->gbase + G->gb_off[k] : nullptr, sh ? G->gift + G->gift_off[k] : nullptr,
                   sh ? G->wflag + G->flag_off[k] : nullptr};
}

// the gather pass of every instance with gifts (device table d_inst)
static void launch_gather(Ctx &ctx, const std::vector<ExactJob> &jobs, const GiftPlan &G, const ExactInst *d_inst,
                          hipStream_t s) {
  for (int k = 0; k < (int)jobs.size(); ++k) {
    if (G.gb_off[k] < 0) continue;
    const int64_t C = jobs[k].t->n_cells;
    const int64_t blocks = std::min<int64_t>(div_up(C, kGatherWaves), (int64_t)ctx.n_cu * 8);
    k_exact_gather<<<(unsigned)blocks, 64 * kGatherWaves, 0, s>>>(d_inst, k, C);
    SPH_LAUNCH_CHECK();
  }
}

// Compute units and resident Exact workgroups per CU, queried once per
// context (contexts may live on different threads).
static void exact_occupancy(Ctx &ctx) {
  if (ctx.n_cu != 0) return;
  SPH_HIP(hipDeviceGetAttribute(&ctx.n_cu, hipDeviceAttributeMultiprocessorCount, ctx.device));
  SPH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&ctx.exact_per_cu, k_exact_edges<false>, 64 * kFlatWaves, 0));
  ctx.exact_per_cu = std::max(ctx.exact_per_cu, 1);
}

void exact_integral_batch(Ctx &ctx, const std::vector<ExactJob> &jobs, int precision, hipStream_t s,
                          const ExactTable *tab) {
  int64_t total = 0;
  for (const auto &j : jobs) {
    j.P->w = j.P->mem.get<double>("w", j.P->n_pairs);
    total += j.P->n_pairs;
  }
  if (tab) {
    // pair counts on the device (capacity mode): the table of pointers is
    // already uploaded; one kernel fills in the counts and chunk offsets,
    // and the persistent grid takes its full size
    SPH_REQUIRE(precision == SPHMAP_PREC_MIXED, SPHMAP_EINVAL, "a device-counted batch runs the mixed path");
    const int n_inst = (int)jobs.size();
    k_exact_table<<<1, 64, 0, s>>>(n_inst, tab->np, (ExactInst *)tab->insts, tab->chunk0);
    SPH_LAUNCH_CHECK();
    exact_occupancy(ctx);
    int bpc = ctx.exact_per_cu, pf = 1;
    const int bucket = 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(total, 1));
    auto it = ctx.tuned.find(bucket);
    if (it != ctx.tuned.end()) {
      bpc = it->second.blocks_per_cu;
      pf = it->second.per_fetch;
    }
    const int64_t grid = (int64_t)ctx.n_cu * std::min(bpc, ctx.exact_per_cu);
    const int64_t waves = grid * kFlatWaves;
    FaceRec *faces = ctx.arena.get<FaceRec>("flat_faces", waves * kEntryCap);
    const GiftPlan &G = *(const GiftPlan *)tab->gifts;
    int32_t *rtw = G.any ? ctx.arena.get<int32_t>("flat_rslot", waves * kEntryCap) : nullptr;
    int32_t *next = ctx.arena.get<int32_t>("flat_next", 2);
    int64_t *redo = ctx.arena.get<int64_t>("flat_redo", std::max<int64_t>(total, 1));
    ExactInst *d_inst = (ExactInst *)tab->insts;
    // gift slots from this step's pair counts, within the planned capacity
    for (int k = 0; k < n_inst; ++k) {
      if (G.gb_off[k] < 0) continue;
      const TessDev &t = *jobs[k].t;
      k_gift_sizes<<<(unsigned)div_up(t.n_cells, 256), 256, 0, s>>>(t.n_cells, jobs[k].P->cell_off, t.cell_slots,
                                                                    G.gsize + G.gb_off[k]);
      SPH_LAUNCH_CHECK();
      scan_exclusive_i64(ctx.arena, G.gsize + G.gb_off[k], G.gbase + G.gb_off[k], t.n_cells, true, s);
      k_gift_check<<<1, 64, 0, s>>>(d_inst + k, G.gbase + G.gb_off[k] + t.n_cells, G.cap[k], G.gift + G.gift_off[k],
                                    tab->flag);
      SPH_LAUNCH_CHECK();
    }
    k_zero_i32<<<1, 64, 0, s>>>(next, kCtrInts);
    SPH_LAUNCH_CHECK();
    k_exact_edges<false><<<(unsigned)grid, 64 * kFlatWaves, 0, s>>>(d_inst, tab->chunk0, n_inst, pf, nullptr, faces,
                                                                   rtw, next, redo, next + kRedoCtr);
    SPH_LAUNCH_CHECK();
    k_exact_mixed_list<<<(unsigned)(ctx.n_cu * 4), 256, 0, s>>>(redo, next + kRedoCtr, d_inst, tab->chunk0, n_inst,
                                                                nullptr);
    SPH_LAUNCH_CHECK();
    launch_gather(ctx, jobs, G, d_inst, s);
    return;
  }
  int64_t *ctr = ctx.counting ? ctx.d_counters : nullptr;
  if (ctr) SPH_HIP(hipMemsetAsync(ctr, 0, 8 * sizeof(int64_t), s));
  if (total == 0) return;
  if (precision == SPHMAP_PREC_FP64) {
    KernelTimer kt(&ctx, "exact_integral", s);
    for (const auto &j : jobs) {
      const TessDev &t = *j.t;
      const PartDev &p = *j.p;
      PairsDev &P = *j.P;
      if (P.n_pairs == 0) continue;
      k_exact_fp64<<<(unsigned)div_up(P.n_pairs, 256), 256, 0, s>>>(P.n_pairs, P.pair_c, P.pair_p, p.xyz, p.h, t.gen,
                                                                    t.cell_face_off, t.face_vtx_off, t.fplane,
                                                                    t.fsphere, t.fvpos, P.w, ctr);
      SPH_LAUNCH_CHECK();
    }
    kt.done();
    return;
  }
  // instance table: each instance's pairs start at a fresh 64-pair chunk
  const int n_inst = (int)jobs.size();
  char *stage = (char *)ctx.pinned_get(n_inst * sizeof(ExactInst) + (n_inst + 1) * sizeof(int64_t) + 64);
  ExactInst *host = (ExactInst *)stage;
  int64_t *c0 = (int64_t *)(stage + ((n_inst * sizeof(ExactInst) + 63) & ~(size_t)63));
  c0[0] = 0;
  const GiftPlan G = gift_plan(ctx, ctx.arena, jobs, false, 0.0, s);
  const bool shared = G.any;
  for (int k = 0; k < n_inst; ++k) {
    host[k] = inst_of_job(jobs[k], &G, k);
    c0[k + 1] = c0[k] + div_up(jobs[k].P->n_pairs, 64);
  }
  ExactInst *d_inst = ctx.arena.get<ExactInst>("flat_insts", n_inst);
  int64_t *d_c0 = ctx.arena.get<int64_t>("flat_chunk0", n_inst + 1);
  SPH_HIP(hipMemcpyAsync(d_inst, host, n_inst * sizeof(ExactInst), hipMemcpyHostToDevice, s));
  SPH_HIP(hipMemcpyAsync(d_c0, c0, (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  // persistent kernel: as many workgroups as stay resident at once
  exact_occupancy(ctx);
  const int n_cu = ctx.n_cu, per_cu = ctx.exact_per_cu;
  const int64_t n_chunks = c0[n_inst];
  int32_t *next = ctx.arena.get<int32_t>("flat_next", kCtrInts);  // work counters, redo count
  int64_t *redo = ctx.arena.get<int64_t>("flat_redo", total);
  auto launch = [&](int blocks_per_cu, int per_fetch) {
    const int64_t grid = std::min<int64_t>((int64_t)n_cu * std::min(blocks_per_cu, per_cu), div_up(n_chunks, kFlatWaves));
    const int64_t waves = grid * kFlatWaves;
    FaceRec *faces = ctx.arena.get<FaceRec>("flat_faces", waves * kEntryCap);
    int32_t *rtw = shared ? ctx.arena.get<int32_t>("flat_rslot", waves * kEntryCap) : nullptr;
    KernelTimer kz(&ctx, "flat_reset", s);
    k_zero_i32<<<1, 64, 0, s>>>(next, kCtrInts);
    SPH_LAUNCH_CHECK();
    kz.done();
    KernelTimer kt(&ctx, "exact_integral", s);
    (ctr ? k_exact_edges<true> : k_exact_edges<false>)<<<(unsigned)grid, 64 * kFlatWaves, 0, s>>>(
        d_inst, d_c0, n_inst, per_fetch, ctr, faces, rtw, next, redo, next + kRedoCtr);
    SPH_LAUNCH_CHECK();
    kt.done();
  };
  // Launch shape: workgroups per CU and 64-pair chunks per work fetch.  With
  // autotuning on, the first call in a size class (power of two of the pair
  // count) times every candidate -- each computes the same weights -- and
  // keeps the fastest for later calls of that class.
  const int bucket = 63 - __builtin_clzll((unsigned long long)total);
  auto it = ctx.tuned.find(bucket);
  if (it != ctx.tuned.end()) {
    launch(it->second.blocks_per_cu, it->second.per_fetch);
  } else if (ctx.autotune && !ctr) {
    TuneChoice best{per_cu, 1, 0.0};
    hipEvent_t a, b;
    SPH_HIP(hipEventCreate(&a));
    SPH_HIP(hipEventCreate(&b));
    for (int bpc = per_cu; bpc >= 1; --bpc)
      for (int pf : {1, 2, 4}) {
        SPH_HIP(hipEventRecord(a, s));
        launch(bpc, pf);
        SPH_HIP(hipEventRecord(b, s));
        SPH_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        SPH_HIP(hipEventElapsedTime(&ms, a, b));
        if (best.ms == 0.0 || ms < best.ms) best = TuneChoice{bpc, pf, (double)ms};
      }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    ctx.tuned[bucket] = best;
  } else {
    launch(per_cu, 1);
  }
  KernelTimer kr(&ctx, "exact_redo", s);
  k_exact_mixed_list<<<(unsigned)(n_cu * 4), 256, 0, s>>>(redo, next + kRedoCtr, d_inst, d_c0, n_inst, ctr);
  SPH_LAUNCH_CHECK();
  kr.done();
  if (shared) {
    KernelTimer kg(&ctx, "exact_gather", s);
    launch_gather(ctx, jobs, G, d_inst, s);
    kg.done();
  }
}

// Upload the pointer table of a device-counted batch (before capture).
void exact_table_upload(Ctx &ctx, const std::vector<ExactJob> &jobs, ExactTable &tab, Arena &mem, double headroom,
                        hipStream_t s) {
  const int n_inst = (int)jobs.size();
  std::vector<ExactInst> host(n_inst);
  std::vector<const int64_t *> np(n_inst);
  // gift slots planned from the planning pass's counts, with headroom; the
  // step recounts them on the device and switches an instance's gifts off
  // when they do not fit (k_gift_check)
  if (!tab.gifts) tab.gifts = new GiftPlan();
  GiftPlan &G = *(GiftPlan *)tab.gifts;
  G = gift_plan(ctx, mem, jobs, true, std::max(headroom, 0.05), s);
  for (int k = 0; k < n_inst; ++k) {
    host[k] = inst_of_job(jobs[k], &G, k);
    host[k].P = 0;
    np[k] = jobs[k].P->d_np;
  }
  SPH_HIP(hipMemcpyAsync(tab.insts, host.data(), n_inst * sizeof(ExactInst), hipMemcpyHostToDevice, s));
  SPH_HIP(hipMemcpyAsync((void *)tab.np, np.data(), n_inst * sizeof(int64_t *), hipMemcpyHostToDevice, s));
  SPH_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
}

void exact_table_free(ExactTable &tab) {
  delete (GiftPlan *)tab.gifts;
  tab.gifts = nullptr;
}

size_t exact_inst_bytes() { return sizeof(ExactInst); }

constexpr int64_t kGiftBound = 16;

size_t exact_workspace_bytes(Ctx &ctx, int64_t n_pairs) {
  exact_occupancy(ctx);
  const int64_t grid = std::min<int64_t>((int64_t)ctx.n_cu * ctx.exact_per_cu, div_up(div_up(n_pairs, 64), kFlatWaves));
  const int64_t waves = std::max<int64_t>(grid, 1) * kFlatWaves;
  // face records, their totals and gift slots per resident wave; per pair
  // the redo list, the flags and its gifts (at most kGiftBound slots a pair
  // on average: a cell evaluates about half its faces' shares)
  return (size_t)(waves * kEntryCap * (sizeof(FaceRec) + sizeof(long long) + sizeof(int32_t)) +
                  n_pairs * (sizeof(int64_t) + sizeof(uint8_t) + kGiftBound * sizeof(long long)));
}

void exact_integral(Ctx &ctx, const TessDev &t, const PartDev &p, PairsDev &P, int precision, hipStream_t s) {
  exact_integral_batch(ctx, {ExactJob{&t, &p, &P}}, precision, s);
}

}  // namespace sphmap
