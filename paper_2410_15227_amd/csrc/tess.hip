// Tessellation preprocessing (once per uploaded tessellation) and particle
// staging.
//
// Per face: the Newell area vector gives the plane; the face is oriented so
// that its normal points away from the cell's generation site (the site is
// strictly inside its Voronoi cell), its vertices are rewritten about the
// site in that orientation (counter-clockwise seen from outside), and a
// bounding sphere about the vertex centroid is kept for culling.  Per cell:
// the volume (sum of pyramids from the site) and the canonical binary32
// bounding radius used by the candidate-pair test.
#include "common.hpp"

namespace sphmap {
namespace {

__global__ void k_face_cell(const int64_t *cfo, int64_t C, int32_t *face_cell) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  for (int64_t f = cfo[c]; f < cfo[c + 1]; ++f) face_cell[f] = (int32_t)c;
}

__global__ void k_face_prep(int64_t F, const int32_t *face_cell, const double *gen, const double *vert,
                            const int64_t *fvo, const int32_t *fv, double4 *fplane, double4 *fsphere,
                            double *fvpos, float4 *fvpos32, float4 *fplane32, float4 *edgeA, float4 *edgeE,
                            float4 *edgeM, int *bad) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const int64_t c = face_cell[f];
  const double gx = gen[3 * c], gy = gen[3 * c + 1], gz = gen[3 * c + 2];
  const int64_t s = fvo[f], e = fvo[f + 1];
  const int nv = (int)(e - s);
  double cx = 0, cy = 0, cz = 0;
  for (int64_t k = s; k < e; ++k) {
    const double *v = vert + 3 * (int64_t)fv[k];
    cx += v[0] - gx;
    cy += v[1] - gy;
    cz += v[2] - gz;
  }
  if (nv > 0) {
    cx /= nv;
    cy /= nv;
    cz /= nv;
  }
  double ax = 0, ay = 0, az = 0, rad2 = 0;
  for (int k = 0; k < nv; ++k) {
    const double *v = vert + 3 * (int64_t)fv[s + k];
    const double *w = vert + 3 * (int64_t)fv[s + (k + 1) % nv];
    double px = v[0] - gx - cx, py = v[1] - gy - cy, pz = v[2] - gz - cz;
    double qx = w[0] - gx - cx, qy = w[1] - gy - cy, qz = w[2] - gz - cz;
    ax += 0.5 * (py * qz - pz * qy);
    ay += 0.5 * (pz * qx - px * qz);
    az += 0.5 * (px * qy - py * qx);
    rad2 = fmax(rad2, px * px + py * py + pz * pz);
  }
  double an = sqrt(ax * ax + ay * ay + az * az);
  double nx = 0, ny = 0, nz = 0, off = -1.0;
  bool rev = false;
  if (nv >= 3 && an > 0.0) {
    nx = ax / an;
    ny = ay / an;
    nz = az / an;
    off = nx * cx + ny * cy + nz * cz;
    if (off < 0.0) {
      rev = true;
      nx = -nx;
      ny = -ny;
      nz = -nz;
      off = -off;
    }
    if (!(off > 0.0)) {
      atomicAdd(bad, 1);  // generation site on the face plane: not a valid cell
      off = -1.0;
    }
  }
  fplane[f] = make_double4(nx, ny, nz, off);
  fplane32[f] = make_float4((float)nx, (float)ny, (float)nz, (float)off);
  fsphere[f] = make_double4(cx, cy, cz, sqrt(rad2));
  for (int k = 0; k < nv; ++k) {
    int src = rev ? (nv - 1 - k) : k;
    const double *v = vert + 3 * (int64_t)fv[s + src];
    double px = v[0] - gx, py = v[1] - gy, pz = v[2] - gz;
    fvpos[3 * (s + k) + 0] = px;
    fvpos[3 * (s + k) + 1] = py;
    fvpos[3 * (s + k) + 2] = pz;
    fvpos32[s + k] = make_float4((float)px, (float)py, (float)pz, 0.0f);
  }
  // edges of the oriented polygon, from binary64 vertices
  for (int k = 0; k < nv; ++k) {
    const double *A = fvpos + 3 * (s + k);
    const double *B = fvpos + 3 * (s + (k + 1 == nv ? 0 : k + 1));
    const double bx = B[0] - A[0], by = B[1] - A[1], bz = B[2] - A[2];
    const double len = sqrt(bx * bx + by * by + bz * bz);
    double ex = 0.0, ey = 0.0, ez = 0.0;
    if (len > 0.0) {
      ex = bx / len;
      ey = by / len;
      ez = bz / len;
    }
    const double mx = ny * ez - nz * ey, my = nz * ex - nx * ez, mz = nx * ey - ny * ex;
    edgeA[s + k] = make_float4((float)A[0], (float)A[1], (float)A[2], (float)len);
    edgeE[s + k] = make_float4((float)ex, (float)ey, (float)ez, 0.0f);
    edgeM[s + k] = make_float4((float)mx, (float)my, (float)mz, 0.0f);
  }
}

// Canonical radius: smallest binary32 R with R*R >= max_v |v - g|^2 where
// the squared distance is (dx*dx + dy*dy) + dz*dz in binary64 without
// contraction.
__device__ float canonical_radius(double r2) {
  float R = (float)sqrt(r2);
  while ((double)R * (double)R < r2) R = nextafterf(R, INFINITY);
  while (R > 0.0f) {
    float Rm = nextafterf(R, 0.0f);
    if ((double)Rm * (double)Rm >= r2) R = Rm;
    else break;
  }
  return R;
}

__global__ void k_cell_prep(int64_t C, const double *gen, const double *vert, const int64_t *cfo, const int64_t *fvo,
                            const int32_t *fv, const double4 *fplane, const double4 *fsphere, double *volume,
                            float *radius, float4 *gen32) {
#pragma clang fp contract(off)
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const double gx = gen[3 * c], gy = gen[3 * c + 1], gz = gen[3 * c + 2];
  double r2 = 0.0, vol = 0.0;
  for (int64_t f = cfo[c]; f < cfo[c + 1]; ++f) {
    for (int64_t k = fvo[f]; k < fvo[f + 1]; ++k) {
      const double *v = vert + 3 * (int64_t)fv[k];
      double dx = v[0] - gx, dy = v[1] - gy, dz = v[2] - gz;
      double s = (dx * dx + dy * dy) + dz * dz;
      if (s > r2) r2 = s;
    }
  }
  // volume: pyramids from the site, height = plane offset, base = face area
  for (int64_t f = cfo[c]; f < cfo[c + 1]; ++f) {
    double4 pl = fplane[f];
    if (!(pl.w > 0.0)) continue;
    const int64_t s = fvo[f], e = fvo[f + 1];
    const int nv = (int)(e - s);
    double4 sp = fsphere[f];
    double ax = 0, ay = 0, az = 0;
    for (int k = 0; k < nv; ++k) {
      const double *v = vert + 3 * (int64_t)fv[s + k];
      const double *w = vert + 3 * (int64_t)fv[s + (k + 1) % nv];
      double px = v[0] - gx - sp.x, py = v[1] - gy - sp.y, pz = v[2] - gz - sp.z;
      double qx = w[0] - gx - sp.x, qy = w[1] - gy - sp.y, qz = w[2] - gz - sp.z;
      ax += 0.5 * (py * qz - pz * qy);
      ay += 0.5 * (pz * qx - px * qz);
      az += 0.5 * (px * qy - py * qx);
    }
    vol += pl.w * sqrt(ax * ax + ay * ay + az * az) / 3.0;
  }
  volume[c] = vol;
  float R = canonical_radius(r2);
  radius[c] = R;
  gen32[c] = make_float4((float)gx, (float)gy, (float)gz, R);
}

// Twin of each face: a face is shared when the cell it names has a face
// naming it back, both planes are valid, the two bounding spheres agree
// (centres in absolute coordinates and radii, to 1e-9 of the larger radius)
// and the normals are opposite.  Such a face is one polygon seen from two
// cells: its share of the Exact sum is the same magnitude from both sides
// with opposite sign (Sec. 3 of the closed form: C_f depends only on the
// polygon and the particle, the sign on the side).  twin[f] is the other
// cell, or -1 (a wall, no declaration, or no match); twin_face[f] the
// matching face of that cell.
__global__ void k_face_twin(int64_t F, int64_t C, const int32_t *face_cell, const int64_t *cfo, const int32_t *nbr,
                            const double *gen, const double4 *fplane, const double4 *fsphere, int32_t *twin,
                            int32_t *twin_face, unsigned long long *n_shared) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  int32_t tw = -1, tf = -1;
  const int64_t c = face_cell[f], n = nbr[f];
  const double4 pa = fplane[f];
  if (n >= 0 && n < C && n != c && pa.w > 0.0) {
    const double4 sa = fsphere[f];
    const double ax = gen[3 * c] + sa.x, ay = gen[3 * c + 1] + sa.y, az = gen[3 * c + 2] + sa.z;
    for (int64_t g = cfo[n]; g < cfo[n + 1]; ++g) {
      if (nbr[g] != c) continue;
      const double4 pb = fplane[g], sb = fsphere[g];
      const double bx = gen[3 * n] + sb.x, by = gen[3 * n + 1] + sb.y, bz = gen[3 * n + 2] + sb.z;
      const double tol = 1e-9 * fmax(sa.w, sb.w);
      const double dx = ax - bx, dy = ay - by, dz = az - bz;
      if (pb.w > 0.0 && dx * dx + dy * dy + dz * dz <= tol * tol && fabs(sa.w - sb.w) <= tol &&
          pa.x * pb.x + pa.y * pb.y + pa.z * pb.z < -1.0 + 1e-9) {
        tw = (int32_t)n;
        tf = (int32_t)g;
      }
      break;
    }
  }
  twin[f] = tw;
  twin_face[f] = tf;
  if (tw >= 0) atomicAdd(n_shared, 1ull);
}

// Per cell: its faces' roles in the mixed path -- code[f] = the face's slot
// among the cell's shared faces it evaluates (twin cell above it), -1 for a
// face evaluated for this cell only (wall or unshared) -- and the number of
// such slots.  A second pass gives each shared face the twin evaluates the
// code -2 - (its twin's slot).
__global__ void k_face_slots(int64_t C, const int64_t *cfo, const int32_t *twin, int32_t *code, int32_t *n_slots) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  int32_t n = 0;
  for (int64_t f = cfo[c]; f < cfo[c + 1]; ++f) {
    const int32_t tw = twin[f];
    code[f] = tw < 0 ? -1 : (tw > c ? n++ : -2);
  }
  n_slots[c] = n;
}

__global__ void k_face_slots_in(int64_t F, const int32_t *twin_face, int32_t *code) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F || code[f] != -2) return;
  code[f] = -2 - code[twin_face[f]];  // the twin's code is a slot (>= 0)
}

__global__ void k_particles_prep(int64_t n, const double *xyz, const double *h, float4 *x32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x32[i] = make_float4((float)xyz[3 * i], (float)xyz[3 * i + 1], (float)xyz[3 * i + 2], (float)h[i]);
}

}  // namespace

void tess_prepare(Ctx &ctx, TessDev &t, hipStream_t s) {
  const int64_t C = t.n_cells, F = t.n_faces, FV = t.n_fv;
  t.face_cell = t.mem.get<int32_t>("face_cell", F);
  t.fplane = t.mem.get<double4>("fplane", F);
  t.fsphere = t.mem.get<double4>("fsphere", F);
  t.fplane32 = t.mem.get<float4>("fplane32", F);
  t.fvpos = t.mem.get<double>("fvpos", 3 * FV);
  t.fvpos32 = t.mem.get<float4>("fvpos32", FV);
  t.edgeA = t.mem.get<float4>("edgeA", FV);
  t.edgeE = t.mem.get<float4>("edgeE", FV);
  t.edgeM = t.mem.get<float4>("edgeM", FV);
  t.volume = t.mem.get<double>("volume", C);
  t.radius = t.mem.get<float>("radius", C);
  t.gen32 = t.mem.get<float4>("gen32", C);
  t.cell_order = t.mem.get<int32_t>("cell_order", C);
  int *bad = t.mem.get<int>("bad", 1);
  SPH_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  k_face_cell<<<(unsigned)div_up(C, 256), 256, 0, s>>>(t.cell_face_off, C, t.face_cell);
  SPH_LAUNCH_CHECK();
  if (F > 0) {
    k_face_prep<<<(unsigned)div_up(F, 256), 256, 0, s>>>(F, t.face_cell, t.gen, t.vert, t.face_vtx_off, t.face_vtx,
                                                         t.fplane, t.fsphere, t.fvpos, t.fvpos32, t.fplane32,
                                                         t.edgeA, t.edgeE, t.edgeM, bad);
    SPH_LAUNCH_CHECK();
  }
  k_cell_prep<<<(unsigned)div_up(C, 256), 256, 0, s>>>(C, t.gen, t.vert, t.cell_face_off, t.face_vtx_off,
                                                       t.face_vtx, t.fplane, t.fsphere, t.volume, t.radius, t.gen32);
  SPH_LAUNCH_CHECK();
  // cells in Morton order of their sites (locality of the pair search)
  uint64_t *keys = t.mem.get<uint64_t>("cell_keys", C);
  morton_keys(t.gen, 3, C, t.box_lo[0], t.box_lo[1], t.box_lo[2], t.box_size, keys, t.cell_order, s);
  radix_sort_u64(ctx.arena, keys, t.cell_order, C, 63, s);
  int bad_h = 0;
  SPH_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  SPH_REQUIRE(bad_h == 0, SPHMAP_EGEOM,
              std::to_string(bad_h) + " face(s) have the generation site on their plane (site not strictly inside)");
  // a grid built here records the neighbour of every face
  if (t.face_nbr) tess_set_twins(ctx, t, t.face_nbr, s);
}

int64_t tess_set_twins(Ctx &ctx, TessDev &t, const int32_t *d_nbr, hipStream_t s) {
  (void)ctx;
  if (!d_nbr || t.n_faces == 0) {
    t.face_twin = t.twin_face = t.face_code = t.cell_slots = nullptr;
    return 0;
  }
  int32_t *tw = t.mem.get<int32_t>("ftwin", t.n_faces);
  int32_t *tf = t.mem.get<int32_t>("ftwinf", t.n_faces);
  int32_t *code = t.mem.get<int32_t>("fcode", t.n_faces);
  int32_t *ns = t.mem.get<int32_t>("cslots", t.n_cells);
  unsigned long long *cnt = t.mem.get<unsigned long long>("ftwin_n", 1);
  SPH_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
  k_face_twin<<<(unsigned)div_up(t.n_faces, 256), 256, 0, s>>>(t.n_faces, t.n_cells, t.face_cell, t.cell_face_off,
                                                               d_nbr, t.gen, t.fplane, t.fsphere, tw, tf, cnt);
  SPH_LAUNCH_CHECK();
  k_face_slots<<<(unsigned)div_up(t.n_cells, 256), 256, 0, s>>>(t.n_cells, t.cell_face_off, tw, code, ns);
  SPH_LAUNCH_CHECK();
  k_face_slots_in<<<(unsigned)div_up(t.n_faces, 256), 256, 0, s>>>(t.n_faces, tf, code);
  SPH_LAUNCH_CHECK();
  unsigned long long n = 0;
  SPH_HIP(hipMemcpyAsync(&n, cnt, sizeof(n), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  if (n) {
    t.face_twin = tw;
    t.twin_face = tf;
    t.face_code = code;
    t.cell_slots = ns;
  } else {
    t.face_twin = t.twin_face = t.face_code = t.cell_slots = nullptr;
  }
  return (int64_t)n;
}

void particles_prepare(Ctx &ctx, PartDev &p, hipStream_t s) {
  (void)ctx;
  k_particles_prep<<<(unsigned)div_up(p.n, 256), 256, 0, s>>>(p.n, p.xyz, p.h, p.x32);
  SPH_LAUNCH_CHECK();
}

}  // namespace sphmap
