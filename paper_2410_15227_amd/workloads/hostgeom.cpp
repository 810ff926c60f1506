// Host-side input tools for the synthetic workloads.
//
// These build the INPUTS of the mapping: smoothing lengths of the SPH
// particles and a box-clipped Voronoi tessellation of the generation sites.
// In the scheme the SPH code has already solved the particle smoothing
// lengths before the radiation step runs (Sec. 2.3), and the grid code builds
// the Voronoi grid from the generation sites (Sec. 1, Sec. 2.3); neither is
// part of the mapping itself.  Nothing here is used by the device library or
// by the CPU oracle beyond providing their common inputs.
//
// Build: g++ -O2 -fopenmp -shared -fPIC hostgeom.cpp -o libsphinput.so

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <queue>
#include <vector>
#include <omp.h>

namespace {

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 mul(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// ---------------------------------------------------------------- k-d tree
struct KDNode {
  double lo[3], hi[3];
  int32_t start, end;   // range in perm
  int32_t left, right;  // children (-1 for a leaf)
};

struct KDTree {
  const double *X;  // [n][3]
  int64_t n;
  std::vector<int32_t> perm;
  std::vector<KDNode> nodes;
  std::vector<double> P;  // points in perm order [n][3]

  void build(const double *pts, int64_t npts, int leaf = 8) {
    X = pts;
    n = npts;
    perm.resize(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    nodes.clear();
    nodes.reserve(2 * (n / leaf + 1) + 8);
    build_rec(0, (int32_t)n, leaf);
    P.resize(3 * n);
    for (int64_t t = 0; t < n; ++t)
      for (int k = 0; k < 3; ++k) P[3 * t + k] = X[3 * (int64_t)perm[t] + k];
  }
  int build_rec(int32_t s, int32_t e, int leaf) {
    KDNode nd;
    for (int k = 0; k < 3; ++k) {
      nd.lo[k] = 1e300;
      nd.hi[k] = -1e300;
    }
    for (int32_t t = s; t < e; ++t) {
      const double *p = X + 3 * (int64_t)perm[t];
      for (int k = 0; k < 3; ++k) {
        nd.lo[k] = std::min(nd.lo[k], p[k]);
        nd.hi[k] = std::max(nd.hi[k], p[k]);
      }
    }
    nd.start = s;
    nd.end = e;
    nd.left = nd.right = -1;
    int id = (int)nodes.size();
    nodes.push_back(nd);
    if (e - s > leaf) {
      int ax = 0;
      double ext = nd.hi[0] - nd.lo[0];
      for (int k = 1; k < 3; ++k)
        if (nd.hi[k] - nd.lo[k] > ext) {
          ext = nd.hi[k] - nd.lo[k];
          ax = k;
        }
      int32_t mid = s + (e - s) / 2;
      std::nth_element(perm.begin() + s, perm.begin() + mid, perm.begin() + e,
                       [&](int32_t a, int32_t b) {
                         double va = X[3 * (int64_t)a + ax], vb = X[3 * (int64_t)b + ax];
                         return va < vb || (va == vb && a < b);
                       });
      int l = build_rec(s, mid, leaf);
      int r = build_rec(mid, e, leaf);
      nodes[id].left = l;
      nodes[id].right = r;
    }
    return id;
  }
  double box_d2(const KDNode &nd, const double *q) const {
    double d2 = 0;
    for (int k = 0; k < 3; ++k) {
      double t = 0;
      if (q[k] < nd.lo[k]) t = nd.lo[k] - q[k];
      else if (q[k] > nd.hi[k]) t = q[k] - nd.hi[k];
      d2 += t * t;
    }
    return d2;
  }
  // all points within radius r of q (squared distance < r2)
  void range(const double *q, double r2, std::vector<int32_t> &out) const {
    out.clear();
    int stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp) {
      const KDNode &nd = nodes[stack[--sp]];
      if (box_d2(nd, q) >= r2) continue;
      if (nd.left < 0) {
        for (int32_t t = nd.start; t < nd.end; ++t) {
          const double *p = P.data() + 3 * (int64_t)t;
          double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
          if (dx * dx + dy * dy + dz * dz < r2) out.push_back(perm[t]);
        }
      } else {
        stack[sp++] = nd.left;
        stack[sp++] = nd.right;
      }
    }
  }
};

// Incremental nearest-neighbour iterator (best-first over the k-d tree).
struct NNIter {
  struct Item {
    double d2;
    int32_t id;  // >=0: point index; <0: -(node+1)
    bool operator<(const Item &o) const { return d2 > o.d2 || (d2 == o.d2 && id > o.id); }
  };
  const KDTree *T;
  double q[3];
  std::priority_queue<Item> pq;
  void start(const KDTree *t, const double *qq) {
    T = t;
    q[0] = qq[0];
    q[1] = qq[1];
    q[2] = qq[2];
    pq = std::priority_queue<Item>();
    pq.push({T->box_d2(T->nodes[0], q), -1});
  }
  // returns false when exhausted
  bool next(int32_t &j, double &d2) {
    while (!pq.empty()) {
      Item it = pq.top();
      pq.pop();
      if (it.id >= 0) {
        j = it.id;
        d2 = it.d2;
        return true;
      }
      const KDNode &nd = T->nodes[-it.id - 1];
      if (nd.left < 0) {
        for (int32_t t = nd.start; t < nd.end; ++t) {
          const double *x = T->P.data() + 3 * (int64_t)t;
          double dx = x[0] - q[0], dy = x[1] - q[1], dz = x[2] - q[2];
          pq.push({dx * dx + dy * dy + dz * dz, T->perm[t]});
        }
      } else {
        pq.push({T->box_d2(T->nodes[nd.left], q), -(nd.left + 1)});
        pq.push({T->box_d2(T->nodes[nd.right], q), -(nd.right + 1)});
      }
    }
    return false;
  }
};

// ------------------------------------------------------- M4 kernel (inputs)
// Cubic-spline shape w(q) with W = w/(pi h^3), support 2h; used here only to
// solve the INPUT particles' SPH smoothing lengths.
inline double m4_w(double q) {
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) {
    double t = 2.0 - q;
    return 0.25 * t * t * t;
  }
  return 0.0;
}
inline double m4_dw(double q) {
  if (q < 1.0) return -3.0 * q + 2.25 * q * q;
  if (q < 2.0) {
    double t = 2.0 - q;
    return -0.75 * t * t;
  }
  return 0.0;
}

// ------------------------------------------------------ Voronoi clipping
struct Poly {
  std::vector<V3> v;
  std::vector<std::vector<int>> f;  // CCW seen from outside
  std::vector<int> nbr;             // neighbour id, -1 for a wall
};

void make_box(Poly &P, const double *lo, const double *hi) {
  P.v.clear();
  P.f.clear();
  P.nbr.clear();
  for (int k = 0; k < 8; ++k)
    P.v.push_back({(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]});
  // faces CCW seen from outside
  P.f.push_back({0, 4, 6, 2});  // x = lo
  P.f.push_back({1, 3, 7, 5});  // x = hi
  P.f.push_back({0, 1, 5, 4});  // y = lo
  P.f.push_back({2, 6, 7, 3});  // y = hi
  P.f.push_back({0, 2, 3, 1});  // z = lo
  P.f.push_back({4, 5, 7, 6});  // z = hi
  for (int k = 0; k < 6; ++k) P.nbr.push_back(-1);
}

// Clip P by the half-space {x : n.x <= c}; new face gets neighbour id `nb`.
// Returns 0 if unchanged, 1 if clipped, -1 on a topological failure.
int clip(Poly &P, V3 n, double c, int nb, double tol) {
  const size_t nv = P.v.size();
  std::vector<double> s(nv);
  std::vector<int8_t> st(nv);  // +1 out, 0 on, -1 in
  bool any_out = false;
  double nn = std::sqrt(dot(n, n));
  for (size_t i = 0; i < nv; ++i) {
    s[i] = dot(n, P.v[i]) - c;
    double sd = s[i] / nn;
    st[i] = sd > tol ? 1 : (sd < -tol ? -1 : 0);
    if (st[i] > 0) any_out = true;
  }
  if (!any_out) return 0;
  std::vector<std::pair<uint64_t, int>> cuts;  // edge key -> vertex id
  auto cut_vertex = [&](int a, int b) -> int {
    int lo = std::min(a, b), hi = std::max(a, b);
    uint64_t key = ((uint64_t)lo << 32) | (uint32_t)hi;
    for (auto &kv : cuts)
      if (kv.first == key) return kv.second;
    // parametrise from the lower-index end so both faces get the same point
    double t = s[lo] / (s[lo] - s[hi]);
    V3 p = add(P.v[lo], mul(sub(P.v[hi], P.v[lo]), t));
    int id = (int)P.v.size();
    P.v.push_back(p);
    cuts.push_back({key, id});
    return id;
  };
  std::vector<std::vector<int>> nf;
  std::vector<int> nnbr;
  std::vector<std::pair<int, int>> seg;  // (entry, exit) of each clipped face
  for (size_t fi = 0; fi < P.f.size(); ++fi) {
    const std::vector<int> &F = P.f[fi];
    const int m = (int)F.size();
    bool has_out = false, has_keep = false;
    for (int k = 0; k < m; ++k) {
      if (st[F[k]] > 0) has_out = true;
      else has_keep = true;
    }
    if (!has_out) {
      nf.push_back(F);
      nnbr.push_back(P.nbr[fi]);
      continue;
    }
    if (!has_keep) continue;  // whole face removed
    std::vector<int> out;
    int exitv = -1, entryv = -1;
    for (int k = 0; k < m; ++k) {
      int a = F[k], b = F[(k + 1) % m];
      if (st[a] <= 0) out.push_back(a);
      if (st[a] <= 0 && st[b] > 0) {  // leaving
        if (st[a] == 0) exitv = a;
        else {
          exitv = cut_vertex(a, b);
          out.push_back(exitv);
        }
      } else if (st[a] > 0 && st[b] <= 0) {  // entering
        if (st[b] == 0) entryv = b;
        else {
          entryv = cut_vertex(a, b);
          out.push_back(entryv);
        }
      }
    }
    if (exitv < 0 || entryv < 0) return -1;
    if (out.size() >= 3) {
      nf.push_back(out);
      nnbr.push_back(P.nbr[fi]);
    }
    if (exitv != entryv) seg.push_back({entryv, exitv});
  }
  // chain the new face: next[entry] = exit
  if (seg.size() >= 3) {
    std::vector<int> face;
    int startv = seg[0].first;
    int cur = startv;
    for (size_t it = 0; it <= seg.size(); ++it) {
      face.push_back(cur);
      int nxt = -1;
      for (auto &sg : seg)
        if (sg.first == cur) {
          nxt = sg.second;
          break;
        }
      if (nxt < 0) return -1;
      cur = nxt;
      if (cur == startv) break;
    }
    if (cur != startv || face.size() != seg.size()) return -1;
    nf.push_back(face);
    nnbr.push_back(nb);
  }
  P.f.swap(nf);
  P.nbr.swap(nnbr);
  return 1;
}

struct CellOut {
  std::vector<V3> v;
  std::vector<int32_t> fsize, fvtx, fnbr;
  int status = 0;
};

void compact(const Poly &P, CellOut &o) {
  std::vector<int> remap(P.v.size(), -1);
  o.v.clear();
  o.fsize.clear();
  o.fvtx.clear();
  o.fnbr.clear();
  for (size_t fi = 0; fi < P.f.size(); ++fi) {
    o.fsize.push_back((int32_t)P.f[fi].size());
    o.fnbr.push_back(P.nbr[fi]);
    for (int vid : P.f[fi]) {
      if (remap[vid] < 0) {
        remap[vid] = (int)o.v.size();
        o.v.push_back(P.v[vid]);
      }
      o.fvtx.push_back(remap[vid]);
    }
  }
}

}  // namespace

extern "C" {

// SPH smoothing lengths of the input particles: rho_i = sum_j m_j W(r_ij, h_i)
// (self term included) and h_i = hfact (m_i/rho_i)^(1/3), solved by Newton's
// method on rho_sum(h) - m (hfact/h)^3 to |dh|/h < tol, kept inside a
// bracket by bisection.
// Returns the number of bisection steps taken.
int64_t sph_smoothing_lengths(int64_t n, const double *xyz, const double *m, double hfact,
                              double tol, double *h_out, double *rho_out) {
  KDTree T;
  T.build(xyz, n, 8);
  int64_t nbis = 0;
  const int k_guess = (int)std::min<int64_t>(n - 1, 58);
#pragma omp parallel reduction(+ : nbis)
  {
    std::vector<int32_t> cand;
    std::vector<std::pair<double, double>> buf;
    NNIter it;
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      const double *q = xyz + 3 * i;
      // initial guess: half the distance to the ~58th neighbour
      it.start(&T, q);
      int32_t j;
      double d2 = 0, dk2 = 0;
      int cnt = 0;
      while (cnt <= k_guess && it.next(j, d2)) {
        dk2 = d2;
        ++cnt;
      }
      double h = 0.5 * std::sqrt(dk2);
      if (!(h > 0)) h = 1e-3;
      double rq = 0;  // current query radius
      auto eval = [&](double hh, double &f, double &fp) {
        if (2.0 * hh > rq || 4.0 * hh < rq) {
          rq = 2.0 * hh * 1.25;
          T.range(q, rq * rq, cand);
          buf.clear();
          for (int32_t jj : cand) {
            const double *p = xyz + 3 * (int64_t)jj;
            double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
            buf.push_back({dx * dx + dy * dy + dz * dz, m[jj]});
          }
        }
        double rs = 0, drs = 0, ih = 1.0 / hh, r2max = 4.0 * hh * hh;
        for (const auto &b : buf) {
          if (b.first >= r2max) continue;
          double qq = std::sqrt(b.first) * ih;
          double wq = m4_w(qq);
          rs += b.second * wq;
          drs -= b.second * (3.0 * wq + qq * m4_dw(qq));
        }
        double ih3 = ih * ih * ih / M_PI;
        rs *= ih3;
        drs *= ih3 * ih;
        double rh = m[i] * std::pow(hfact / hh, 3);
        f = rs - rh;
        fp = drs + 3.0 * rh / hh;
      };
      // safeguarded Newton: keep a bracket lo < root < hi (f < 0 below the
      // root since the self term alone is below m (hfact/h)^3), bisect when
      // the Newton step leaves it.
      double lo = 0.0, hi = HUGE_VAL;
      bool ok = false;
      for (int itn = 0; itn < 200; ++itn) {
        double f, fp;
        eval(h, f, fp);
        if (f < 0) lo = h;
        else hi = h;
        double hn = h - f / fp;
        if (!(fp > 0) || !(hn > lo) || !(hn < hi)) {
          if (hi == HUGE_VAL) hn = 2.0 * h;
          else if (lo == 0.0) hn = 0.5 * h;
          else hn = 0.5 * (lo + hi);
          if (itn > 0 && lo > 0 && hi < HUGE_VAL) ++nbis;
        }
        double rel = std::fabs(hn - h) / h;
        h = hn;
        if (rel < tol) {
          ok = true;
          break;
        }
      }
      (void)ok;
      h_out[i] = h;
      double f, fp;
      eval(h, f, fp);
      rho_out[i] = f + m[i] * std::pow(hfact / h, 3);
    }
  }
  return nbis;
}

// Box-clipped Voronoi tessellation of n generators inside [lo, hi].
// Pass 1 (out arrays NULL) builds every cell and returns the sizes through
// sizes[0..2] = (n_vertices, n_faces, n_face_vertices); pass 2 fills:
//   vertices[V][3]     per-cell vertex blocks (cell_vtx_off)
//   cell_face_off[n+1] faces grouped by cell
//   face_vtx_off[F+1], face_vtx[FV] global vertex ids, CCW seen from outside
//   face_nbr[F]        neighbouring generator, -1 for a box wall
// The cells are kept between the two calls in an opaque handle.
struct VoroHandle {
  std::vector<CellOut> cells;
};

void *voronoi_build(int64_t n, const double *gen, const double *lo, const double *hi,
                    int64_t *sizes, int64_t *n_failed) {
  VoroHandle *H = new VoroHandle;
  H->cells.resize(n);
  KDTree T;
  T.build(gen, n, 8);
  double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                          (hi[2] - lo[2]) * (hi[2] - lo[2]));
  double tol = 1e-13 * diag;
  int64_t failed = 0;
#pragma omp parallel reduction(+ : failed)
  {
    Poly P;
    NNIter it;
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      const double *q = gen + 3 * i;
      V3 xi{q[0], q[1], q[2]};
      make_box(P, lo, hi);
      auto rmax2 = [&]() {
        double r = 0;
        for (auto &f : P.f)
          for (int vid : f) {
            V3 dv = sub(P.v[vid], xi);
            r = std::max(r, dot(dv, dv));
          }
        return r;
      };
      double r2 = rmax2();
      it.start(&T, q);
      int32_t j;
      double d2;
      int st = 0;
      while (it.next(j, d2)) {
        if (j == i) continue;
        if (d2 > 4.0 * r2) break;
        const double *pj = gen + 3 * (int64_t)j;
        V3 xj{pj[0], pj[1], pj[2]};
        V3 nrm = sub(xj, xi);
        double c = dot(nrm, mul(add(xi, xj), 0.5));
        int rc = clip(P, nrm, c, (int)j, tol);
        if (rc < 0) {
          st = 1;
          break;
        }
        if (rc > 0) r2 = rmax2();
      }
      CellOut &o = H->cells[i];
      compact(P, o);
      o.status = st;
      if (st) ++failed;
    }
  }
  int64_t V = 0, F = 0, FV = 0;
  for (auto &c : H->cells) {
    V += (int64_t)c.v.size();
    F += (int64_t)c.fsize.size();
    FV += (int64_t)c.fvtx.size();
  }
  sizes[0] = V;
  sizes[1] = F;
  sizes[2] = FV;
  *n_failed = failed;
  return H;
}

void voronoi_fill(void *h, double *vertices, int64_t *cell_vtx_off, int64_t *cell_face_off,
                  int64_t *face_vtx_off, int32_t *face_vtx, int32_t *face_nbr) {
  VoroHandle *H = (VoroHandle *)h;
  const int64_t n = (int64_t)H->cells.size();
  int64_t V = 0, F = 0, FV = 0;
  cell_vtx_off[0] = 0;
  cell_face_off[0] = 0;
  face_vtx_off[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const CellOut &c = H->cells[i];
    for (auto &p : c.v) {
      vertices[3 * V + 0] = p.x;
      vertices[3 * V + 1] = p.y;
      vertices[3 * V + 2] = p.z;
      ++V;
    }
    int64_t base = cell_vtx_off[i];
    size_t k = 0;
    for (size_t fi = 0; fi < c.fsize.size(); ++fi) {
      for (int32_t t = 0; t < c.fsize[fi]; ++t) face_vtx[FV++] = (int32_t)(base + c.fvtx[k++]);
      face_nbr[F] = c.fnbr[fi];
      ++F;
      face_vtx_off[F] = FV;
    }
    cell_vtx_off[i + 1] = V;
    cell_face_off[i + 1] = F;
  }
}

void voronoi_free(void *h) { delete (VoroHandle *)h; }

// Geometry checks of a tessellation: per-cell volume (divergence theorem),
// closure |sum of face area vectors|, and the worst non-planarity of a face.
// Writes vol[n]; returns max closure defect; stats[0] = max non-planarity,
// stats[1] = number of faces whose orientation points towards the generator.
double tess_check(int64_t n, const double *gen, const double *vert, const int64_t *cell_face_off,
                  const int64_t *face_vtx_off, const int32_t *face_vtx, double *vol,
                  double *stats) {
  double worst = 0, nonplanar = 0, inward = 0;
#pragma omp parallel for reduction(max : worst, nonplanar) reduction(+ : inward) schedule(dynamic, 256)
  for (int64_t c = 0; c < n; ++c) {
    V3 g{gen[3 * c], gen[3 * c + 1], gen[3 * c + 2]};
    V3 asum{0, 0, 0};
    double V = 0;
    for (int64_t f = cell_face_off[c]; f < cell_face_off[c + 1]; ++f) {
      int64_t s = face_vtx_off[f], e = face_vtx_off[f + 1];
      const int m = (int)(e - s);
      V3 cen{0, 0, 0};
      for (int64_t k = s; k < e; ++k) {
        const double *p = vert + 3 * (int64_t)face_vtx[k];
        cen = add(cen, V3{p[0], p[1], p[2]});
      }
      cen = mul(cen, 1.0 / m);
      V3 a{0, 0, 0};
      for (int k = 0; k < m; ++k) {
        const double *p = vert + 3 * (int64_t)face_vtx[s + k];
        const double *q = vert + 3 * (int64_t)face_vtx[s + (k + 1) % m];
        a = add(a, mul(cross(sub(V3{p[0], p[1], p[2]}, cen), sub(V3{q[0], q[1], q[2]}, cen)), 0.5));
      }
      asum = add(asum, a);
      V += dot(sub(cen, g), a) / 3.0;
      double an = std::sqrt(dot(a, a));
      if (an > 0) {
        V3 nh = mul(a, 1.0 / an);
        for (int64_t k = s; k < e; ++k) {
          const double *p = vert + 3 * (int64_t)face_vtx[k];
          nonplanar = std::max(nonplanar, std::fabs(dot(sub(V3{p[0], p[1], p[2]}, cen), nh)));
        }
        if (dot(sub(cen, g), nh) < 0) inward += 1;
      }
    }
    vol[c] = V;
    worst = std::max(worst, std::sqrt(dot(asum, asum)));
  }
  stats[0] = nonplanar;
  stats[1] = inward;
  return worst;
}

}  // extern "C"
