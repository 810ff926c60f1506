/*
 * sphmap: Exact SPH-particle <-> Voronoi-cell mapping and tree-node
 * pseudo-particles on AMD Instinct MI355X (gfx950).
 *
 * The mapping transfers the SPH density field onto a Voronoi grid whose
 * generation sites need not coincide with the particles, by integrating each
 * particle's M4 cubic-spline kernel (truncated at 2h) analytically over every
 * cell it overlaps (Sec. 1; Sec. 2.3, forward mapping; kernel in Sec. 2.4.2):
 *     w_ic  = integral over cell c of W(|r - x_i|, h_i) dV
 *     M_c   = sum_i m_i w_ic,      rho_c = M_c / V_c
 * and transfers cell quantities back onto the particles (Sec. 2.3, inverse
 * mapping):
 *     q_i   = sum_c w_ic q_c / c_i,   c_i = sum_c w_ic  (q_i = 0 if c_i = 0).
 * The pseudo-particle builder collapses gravity-tree nodes far from the
 * ionising sources into pseudo-particles and solves their smoothing lengths
 * (Sec. 2.4.1 eq. opening_angle; Sec. 2.4.2 eqs. h_node .. hnode_estval).
 *
 * Conventions for every entry point:
 *  - Pointers prefixed d_ are DEVICE pointers (memory of the context's
 *    device); pointers prefixed h_ are HOST pointers.  The caller owns every
 *    buffer it passes in and out; the library never frees caller memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it; device outputs are valid once the stream has reached that point.
 *    Calls that must size an output (pair lists, pseudo-particle counts)
 *    synchronise the stream once internally.
 *  - Return value: 0 on success or a negative SPHMAP_E* code.  Arguments and
 *    shapes are validated before anything is enqueued.  sphmap_last_error()
 *    gives a message for the last failing call on that context.
 *  - Contexts are independent; a context must not be used by two host
 *    threads at once.
 */
#ifndef SPHMAP_H
#define SPHMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPHMAP_OK 0
#define SPHMAP_EINVAL (-1) /* bad argument, size or layout                  */
#define SPHMAP_ENOMEM (-2) /* device allocation failed, or the context's
                              workspace limit is too small (the bytes the
                              call needs: sphmap_workspace_info)            */
#define SPHMAP_EGEOM (-3)  /* tessellation fails validation                 */
#define SPHMAP_EHIP (-4)   /* HIP runtime error                             */
#define SPHMAP_ERANGE (-5) /* output capacity too small                     */

/* Bits of the device status word (sphmap_sync_status). */
#define SPHMAP_STATUS_NONFINITE_MASS 1  /* a cell mass M_c was not finite      */
#define SPHMAP_STATUS_ZERO_COVERAGE 2   /* inverse map: a particle with c_i = 0
                                           (no cell overlaps it) got q_i = 0  */
#define SPHMAP_STATUS_NONFINITE_VALUE 4 /* inverse map or interpolation wrote a
                                           value that was not finite          */

#define SPHMAP_PREC_FP64 0  /* every step of the integral in binary64        */
#define SPHMAP_PREC_MIXED 1 /* binary32 closed form, binary64 for degenerate
                               pieces and for every accumulation            */

typedef struct sphmap_ctx sphmap_ctx;     /* device, workspace, timers       */
typedef struct sphmap_tess sphmap_tess;   /* device-resident tessellation     */
typedef struct sphmap_pairs sphmap_pairs; /* retained pair list and weights   */

/* Library version (major*10000 + minor*100 + patch). */
int sphmap_version(void);

/* Create a context on HIP device `device`.  *out receives the handle.
   workspace_bytes caps the device memory of the context's scratch (pair
   search, Exact-integral work lists, transpose, and the pair lists of calls
   that keep none); 0 = no cap, the scratch grows on demand.  The scratch is
   kept between calls.  A call whose scratch would pass the cap fails with
   SPHMAP_ENOMEM before it allocates; sphmap_workspace_info then reports an
   upper bound of the workspace it needs (sphmap_estimate_footprint gives the
   same bound beforehand).  Retained pair lists (pairs_out) and uploaded
   grids are not part of the workspace. */
int sphmap_create(int32_t device, size_t workspace_bytes, sphmap_ctx **out);
/* Change the workspace cap (0 = none).  Lowering it below what the scratch
   holds frees the scratch (after waiting for the device). */
int sphmap_set_workspace_limit(sphmap_ctx *ctx, size_t bytes);
/* Device bytes the scratch holds now, the cap, and the largest workspace a
   call refused with SPHMAP_ENOMEM since the cap was last set (0 if none);
   any pointer may be NULL. */
int sphmap_workspace_info(sphmap_ctx *ctx, size_t *held, size_t *limit, size_t *required);
/* Release a context and everything it still owns (tessellations and pair
   lists created from it must be freed first or become invalid). */
int sphmap_destroy(sphmap_ctx *ctx);
/* Message of the last failing call on ctx ("" if none); valid until the
   next call on ctx. */
const char *sphmap_last_error(const sphmap_ctx *ctx);

/* Device-side anomalies do not stop a call: the kernels that meet them set
   bits (SPHMAP_STATUS_*) in a status word of the context.  This waits for
   `stream`, stores the word in *status (host) and, if clear != 0, resets it
   to 0.  The word collects every call on ctx since it was last cleared. */
int sphmap_sync_status(sphmap_ctx *ctx, void *stream, int32_t clear, int32_t *status);

/* Device memory a mapping needs, by owner (upper bounds, in bytes):
     workspace     the context's scratch for one forward mapping of
                   n_particles on the grid followed by an inverse mapping
                   (pair search, Exact integral work queues, transpose);
                   the context keeps it between calls
     pairs         the retained pair list with its weights and particle-major
                   copy (freed with sphmap_pairs_free)
     tessellation  the uploaded grid (freed with sphmap_tess_free)
   n_pairs: the candidate-pair count when known (an earlier step on the same
   grid), else 0 for an estimate of 200 per particle.  Each named device
   buffer is counted as at least one 2 MiB allocation granule.  Caller
   buffers are not included.  Errors: EINVAL for negative sizes. */
typedef struct {
  size_t workspace;
  size_t pairs;
  size_t tessellation;
} sphmap_footprint;
int sphmap_estimate_footprint(sphmap_ctx *ctx, int64_t n_particles, int64_t n_pairs, int64_t n_cells,
                              int64_t n_faces, int64_t n_face_vertices, int64_t n_vertices, sphmap_footprint *out);

/* ------------------------------------------------------------------------
 * Tessellation upload (Sec. 2.3: the grid code receives the generation sites
 * and builds the Voronoi grid; here the grid is given).  Cells are convex
 * polyhedra given as faces grouped by cell:
 *   h_generators  [n_cells][3]      generation site of each cell (strictly
 *                                   inside its cell)
 *   h_vertices    [n_vertices][3]
 *   h_cell_face_off [n_cells+1]     faces of cell c: cell_face_off[c] ..
 *                                   cell_face_off[c+1]-1 (non-decreasing,
 *                                   cell_face_off[0] = 0)
 *   h_face_vtx_off  [n_faces+1]     vertex list of face f: face_vtx[
 *                                   face_vtx_off[f] .. face_vtx_off[f+1]-1]
 *   h_face_vtx    [face_vtx_off[n_faces]]  vertex indices, each face a
 *                                   cyclic convex polygon in EITHER
 *                                   orientation (oriented internally so its
 *                                   normal points away from the generator)
 * Faces of zero area are accepted and contribute nothing; a face may have at
 * most 128 vertices.  All arrays are
 * copied; the host memory may be reused after return.  The preprocessing
 * (face planes, volumes, bounding radii) is enqueued on `stream`.
 * Errors: EINVAL for inconsistent offsets or out-of-range indices.
 * ---------------------------------------------------------------------- */
int sphmap_tess_upload(sphmap_ctx *ctx, int64_t n_cells, int64_t n_faces, int64_t n_vertices,
                       const double *h_generators, const double *h_vertices, const int64_t *h_cell_face_off,
                       const int64_t *h_face_vtx_off, const int32_t *h_face_vtx, void *stream,
                       sphmap_tess **out);
int sphmap_tess_free(sphmap_ctx *ctx, sphmap_tess *tess);
/* Cell volumes V_c (divergence theorem) and the binary32 bounding radius R_c
   of each cell about its generator (the smallest binary32 R with R*R >= the
   binary64 max_v |v - g_c|^2).  Either output may be NULL. */
int sphmap_tess_cell_info(sphmap_ctx *ctx, const sphmap_tess *tess, double *d_volume, float *d_radius,
                          void *stream);

/* Declare, for an uploaded grid, the cell on the other side of each face:
   h_face_nbr [n_faces] (host), a cell index or any negative value for a wall
   or an unknown neighbour.  A face is treated as shared when the cell it
   names declares a face back to it with the same bounding sphere (centre and
   radius, to 1e-9 of the radius) and the opposite normal -- one polygon seen
   from two cells.  Its term of the Exact sum w = S - sum_f sgn(d_f) C_f
   (Sec. 1, the analytic volume integral; C_f depends on the polygon and the
   particle only) is then evaluated once per particle, by the lower-numbered
   cell, and given to the other with the opposite sign (mixed precision
   only; the binary64 path evaluates every face from its own side).  Other
   faces are evaluated from their own side.  The caller vouches that the two
   faces of a declared pair are the same polygon (true of any Voronoi grid).
   NULL clears the declaration.  *n_shared (nullable) receives the number of
   shared faces.  Grids built by sphmap_tess_build_voronoi have their
   neighbours already.  Errors: EINVAL (a neighbour >= n_cells).
   The neighbours are also what sphmap_tess_export returns in d_face_nbr. */
int sphmap_tess_set_face_neighbours(sphmap_ctx *ctx, sphmap_tess *tess, const int32_t *h_face_nbr, void *stream,
                                    int64_t *n_shared);

/* ------------------------------------------------------------------------
 * Voronoi grid built on the device (Sec. 2.3: the grid of the generation
 * sites, regularised by Lloyd iterations before the forward mapping).
 *   d_generators [n][3] (device): the sites, inside [h_box_lo, h_box_hi]
 *     (host [3] each).  Cell c is the part of the box at least as close to
 *     site c as to any other.
 *   n_lloyd: Lloyd iterations first (each moves every site to the centroid
 *     of its cell; the paper uses 5).
 *   d_generators_out [n][3] (device, nullable): the sites of the final grid.
 *   *out: the grid, resident as if uploaded by sphmap_tess_upload; each cell
 *     owns its faces and vertices; faces record the neighbour they face.
 * Cuts within 1e-13 of the box size of a vertex leave it in place.
 * Errors: EINVAL (n < 1, n >= 2^31, a site outside the box, two equal
 * sites, an empty box), EGEOM (a cell with more than 58 cutting neighbours or
 * 128 vertices).  Nothing is returned on an error.
 * ---------------------------------------------------------------------- */
int sphmap_tess_build_voronoi(sphmap_ctx *ctx, int64_t n, const double *d_generators, const double *h_box_lo,
                              const double *h_box_hi, int32_t n_lloyd, double *d_generators_out, void *stream,
                              sphmap_tess **out);

/* Sizes of a resident grid (any pointer may be NULL). */
int sphmap_tess_counts(const sphmap_tess *tess, int64_t *n_cells, int64_t *n_faces, int64_t *n_face_vertices,
                       int64_t *n_vertices);

/* Copy a resident grid into caller device buffers (any may be NULL), in the
   layout of sphmap_tess_upload: d_generators [C][3], d_vertices [V][3],
   d_cell_face_off [C+1], d_face_vtx_off [F+1], d_face_vtx [FV];
   d_face_nbr [F]: the neighbouring site of each face, -1..-6 for the box
   planes x-, x+, y-, y+, z-, z+ (grids built by sphmap_tess_build_voronoi),
   or the declared neighbours of an uploaded grid (EINVAL when none were
   declared). */
int sphmap_tess_export(sphmap_ctx *ctx, const sphmap_tess *tess, double *d_generators, double *d_vertices,
                       int64_t *d_cell_face_off, int64_t *d_face_vtx_off, int32_t *d_face_vtx, int32_t *d_face_nbr,
                       void *stream);

/* ------------------------------------------------------------------------
 * Forward mapping (Sec. 1; Sec. 2.3 "forward mapping"; kernel Sec. 2.4.2).
 *   d_xyz [n][3], d_h [n], d_m [n]   particle positions, smoothing lengths,
 *                                    masses (binary64, device)
 *   precision                        SPHMAP_PREC_FP64 or SPHMAP_PREC_MIXED
 *   normalize                        0: raw integrals (kernel mass beyond a
 *                                    non-periodic wall is lost);
 *                                    1: masses rescaled by 1/c_i so that
 *                                    sum_c M_c = sum_i m_i
 *   d_cell_mass [n_cells]            M_c
 *   d_cell_density [n_cells]         M_c / V_c (nullable)
 *   d_coverage [n]                   c_i = sum_c w_ic (nullable unless
 *                                    normalize = 1)
 *   pairs_out                        nullable; receives a retained pair list
 *                                    (free with sphmap_pairs_free)
 * Candidate pairs (c,i) are those with d2 < s*s evaluated in binary32,
 * round to nearest, without contraction: dx = fl(x_i) - fl(g_x) (same for y,
 * z), d2 = (dx*dx + dy*dy) + dz*dz, s = R_c + 2 fl(h_i).  Every pair whose
 * kernel support overlaps the cell is a candidate; a candidate whose support
 * stays clear of every face gets w = 0 exactly (1 exactly for a support
 * inside the cell).  Cells take their pairs in ascending particle index.
 * M_c is summed in a fixed order that does not depend on the launch: with
 * the cell's pairs numbered k = 0, 1, ... in that index order, partial sum
 * l (l = 0..63) adds m_i w_ic over k = l, l + 64, l + 128, ... in turn
 * (each product rounded, then added), and the 64 partials are combined
 * pairwise, partial l with partial l + 32, then l + 16, l + 8, l + 4, l + 2,
 * l + 1 (a butterfly), so results repeat bit for bit.
 * Errors: EINVAL (n < 1, n >= 2^31, null required pointer, bad precision).
 * ---------------------------------------------------------------------- */
int map_particles_to_cells(sphmap_ctx *ctx, const sphmap_tess *tess, int64_t n, const double *d_xyz,
                           const double *d_h, const double *d_m, int32_t precision, int32_t normalize,
                           double *d_cell_mass, double *d_cell_density, double *d_coverage, void *stream,
                           sphmap_pairs **pairs_out);

/* ------------------------------------------------------------------------
 * Batched forward mapping: n_inst independent instances (the forward map
 * above, each with its own tessellation and particles) in one call.  The
 * candidate pairs are found per instance; the Exact integral of all
 * instances runs as one persistent launch, each 64-pair chunk of work
 * belonging to one instance; the reductions run per instance.  A weight
 * depends on its own pair only, so every instance's results equal those of
 * map_particles_to_cells on that instance alone, bit for bit.
 *   tess[k], n[k], d_xyz[k], d_h[k], d_m[k], d_cell_mass[k]: as in the
 *   single call (host arrays of n_inst entries holding device pointers);
 *   d_cell_density, d_coverage: NULL, or host arrays whose entries may be
 *   NULL; pairs_out: NULL, or a host array receiving n_inst retained lists.
 * Errors: as the single call, per instance; EINVAL for n_inst < 1.  On an
 * error no list is returned.
 * ---------------------------------------------------------------------- */
int map_particles_to_cells_batch(sphmap_ctx *ctx, int32_t n_inst, const sphmap_tess *const *tess, const int64_t *n,
                                 const double *const *d_xyz, const double *const *d_h, const double *const *d_m,
                                 int32_t precision, int32_t normalize, double *const *d_cell_mass,
                                 double *const *d_cell_density, double *const *d_coverage, void *stream,
                                 sphmap_pairs **pairs_out);

/* ------------------------------------------------------------------------
 * The same batched forward mapping as one captured HIP graph, for repeated
 * steps over fixed buffers (the mapping is called on every timestep, Sec.
 * 2.3).  sphmap_batch_create takes the arguments of
 * map_particles_to_cells_batch (mixed precision; no retained lists), runs
 * the step once to size each instance's pair lists (its pair count plus
 * headroom times that count, at least 4096 more), runs it again in that
 * capacity mode and captures the whole step -- pair search, Exact integral
 * of every instance in one persistent launch, transpose, coverage and cell
 * sums, instances dealt to four parallel branches -- into one HIP graph on
 * `stream`.  The pointers and sizes are fixed by the plan; the particle
 * arrays may hold new values at every step.
 * sphmap_batch_run launches the graph once on `stream` (asynchronous; the
 * outputs are those of map_particles_to_cells_batch on the arrays' current
 * values, bit for bit).  An instance whose pair count passes its capacity is
 * left empty (masses 0) and sets the plan's overflow flag;
 * sphmap_batch_check waits for `stream`, copies each instance's pair count
 * of the last step to h_pairs [n_inst] (host, nullable), returns the flag
 * in *overflow (1: at least one step since the last check overflowed;
 * make a new plan) and clears it.
 * Errors: as map_particles_to_cells_batch; EINVAL for headroom outside
 * [0, 16]; EHIP when the capture fails.  Free with sphmap_batch_free before
 * the context and the tessellations. */
typedef struct sphmap_batch sphmap_batch;
int sphmap_batch_create(sphmap_ctx *ctx, int32_t n_inst, const sphmap_tess *const *tess, const int64_t *n,
                        const double *const *d_xyz, const double *const *d_h, const double *const *d_m,
                        int32_t normalize, double *const *d_cell_mass, double *const *d_cell_density,
                        double *const *d_coverage, double headroom, void *stream, sphmap_batch **out);
int sphmap_batch_run(sphmap_ctx *ctx, sphmap_batch *batch, void *stream);
int sphmap_batch_check(sphmap_ctx *ctx, sphmap_batch *batch, void *stream, int64_t *h_pairs, int32_t *overflow);
int sphmap_batch_free(sphmap_ctx *ctx, sphmap_batch *batch);

/* Number of candidate pairs, cells and particles of a retained pair list. */
int sphmap_pairs_info(const sphmap_pairs *pairs, int64_t *n_pairs, int64_t *n_cells, int64_t *n_particles);
/* Copy the retained list into caller device buffers (any may be NULL):
   d_cell_off [n_cells+1] (int64), d_particle [n_pairs] (int32, ascending
   within each cell), d_w [n_pairs] (binary64 weights w_ic). */
int sphmap_pairs_export(sphmap_ctx *ctx, const sphmap_pairs *pairs, int64_t *d_cell_off, int32_t *d_particle,
                        double *d_w, void *stream);
/* Release a retained list (waits for the device first).  Its device blocks
   go to the context's pool, from which later retained lists allocate: a
   block of B bytes serves a request of more than B/2 and at most B bytes,
   so repeated steps make no device allocation.  The pool keeps at most
   one eighth of the device's memory by default (sphmap_set_pool_limit);
   blocks beyond the limit are freed, and all of them are freed before a
   device allocation that fails is retried, and by sphmap_destroy.  Free
   every retained list before destroying its context. */
int sphmap_pairs_free(sphmap_ctx *ctx, sphmap_pairs *pairs);
/* Largest total of device memory, in bytes, that the context's pool of
   freed pair-list blocks may keep (0: keep none).  Blocks held beyond a
   lowered limit are freed at once, after waiting for the device.  For
   callers that run several contexts on one device under a memory budget. */
int sphmap_set_pool_limit(sphmap_ctx *ctx, uint64_t bytes);

/* ------------------------------------------------------------------------
 * Inverse mapping (Sec. 2.3, the ionic fractions returned onto the
 * (pseudo-)particles): q_i = sum_c w_ic q_c / c_i, c_i = sum_c w_ic, q_i = 0
 * where c_i = 0.
 *   pairs (nullable): a retained pair list of the forward mapping; its
 *     weights are used and tess, d_xyz, d_h and precision are ignored (n
 *     must be 0 or the list's particle count).  NULL: the weights are
 *     recomputed from the particles d_xyz [n][3], d_h [n] (device, binary64)
 *     and the grid tess, as the forward mapping at `precision` would give
 *     them (pair search, Exact integral), in the context's workspace.
 *   d_cell_values [n_cells][n_components]      (row-major, binary64)
 *   d_particle_values [n][n_components]
 * Each particle's sums take its cells in ascending cell index, 16 partial
 * sums per particle: with the particle's pairs numbered j = 0, 1, ... in
 * that order, partial l (l = 0..15) adds w_ic q_c over j = l, l + 16, ...
 * in turn, and the partials are combined pairwise, l with l + 8, then l + 4,
 * l + 2, l + 1; the sum is then divided by c_i.  Results repeat bit for bit.
 * Errors: EINVAL (null pointers, n_components < 1, without a list: n out of
 * [1, 2^31), bad precision), ENOMEM (workspace). */
int map_cells_to_particles(sphmap_ctx *ctx, const sphmap_tess *tess, int64_t n, const double *d_xyz,
                           const double *d_h, int32_t precision, const sphmap_pairs *pairs,
                           const double *d_cell_values, int32_t n_components, double *d_particle_values,
                           void *stream);

/* ------------------------------------------------------------------------
 * Pseudo-particles (Sec. 2.4).  The particles (positions in [0,1)^3) are
 * grouped by an octree of the unit cube (cubic subdivision, at most
 * leaf_max particles per leaf, at most max_depth levels).  Node position =
 * centre of mass, node size s = distance from the centre of mass to the
 * furthest member (Sec. 2.2.1); node sums are formed bottom-up, leaves over
 * their members in ascending index, internal nodes over their children in
 * octant order.  Walking depth first from the root, a node is accepted when
 * for every source r - s > r_part and not (theta^2 r^2 < s^2)
 * (eq. opening_angle, r = distance from the source to the centre of mass);
 * a rejected leaf is opened and its particles are emitted with their own h.
 * An accepted node with one member is emitted as that particle.
 * Each pseudo-particle's smoothing length solves eq. hnode_func with
 * n_node = sum_b W(|r_a - r_b|, h) over every emitted unit b (accepted nodes
 * and opened leaves, the latter standing in for their particles, Sec.
 * 2.4.2 last paragraph), self term included: Newton from h0 = h_fact 2 s
 * (eq. hnode_estval) until |h_new - h|/h0 < eps_h; Newton fails after 30
 * steps, when an iterate leaves [1e-2 h0, 1e2 h0] or when |f'| < 1e-12; then
 * bisection on [1e-2 h0, 1e2 h0] if f changes sign there, else h = h0; with
 * more than bypass_threshold pseudo-particles every h = h0.
 * ---------------------------------------------------------------------- */
typedef struct {
  double r_part;             /* radius around sources kept at particle level   */
  double theta;              /* opening angle                                  */
  double h_fact;             /* h = h_fact n^(-1/3)                           */
  double eps_h;              /* Newton tolerance relative to h0               */
  int32_t leaf_max;          /* particles per leaf (at most)                  */
  int32_t max_depth;         /* octree levels below the root (<= 21)          */
  int64_t bypass_threshold;  /* use h0 for all above this many pseudo-particles */
} sphmap_pseudo_opts;

typedef struct {
  int64_t n_nodes;           /* octree nodes                                  */
  int64_t n_units;           /* emitted units (accepted nodes + opened leaves) */
  int64_t n_pseudo;          /* pseudo-particles                               */
  int64_t n_real;            /* particles emitted as themselves                */
  int64_t branch_count[4];   /* h-solve branch: Newton, bisection, h0, bypass  */
  double s_root;             /* size of the root node (Sec. 2.4.1, eq. resol_param) */
} sphmap_pseudo_stats;

/* Inputs d_xyz [n][3], d_h [n], d_m [n] (device); h_sources [n_src][3] (host).
   Outputs (device, capacity entries each, emission order = depth-first, an
   opened leaf's particles in ascending index):
     d_out_xyz [cap][3], d_out_h, d_out_m, d_out_s (node size, 0 for real)
     d_out_kind (0 real particle, 1 pseudo-particle)
     d_out_first (lowest member particle index), d_out_count (members)
     d_out_branch (h-solve branch 0..3, -1 for real particles)
   Any output except d_out_xyz, d_out_h, d_out_m may be NULL.
   *n_out (host) receives the number of entries; ERANGE if it exceeds
   capacity (nothing written then).  stats (host) may be NULL. */
int build_pseudo_particles(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const double *d_h, const double *d_m,
                           int32_t n_src, const double *h_sources, const sphmap_pseudo_opts *opts,
                           int64_t capacity, double *d_out_xyz, double *d_out_h, double *d_out_m, double *d_out_s,
                           int32_t *d_out_kind, int64_t *d_out_first, int64_t *d_out_count,
                           int32_t *d_out_branch, int64_t *n_out, sphmap_pseudo_stats *stats, void *stream);

/* The same with the nodes to open named (Sec. 2.4.1: nodes that failed the
 * resolution check of an earlier walk are opened in the next one).
 *   d_open_labels [n_open] (device, any order; NULL when n_open = 0): node
 *     labels; a labelled node is opened whatever the walk criterion says
 *     (an opened leaf emits its particles with their own h).  Labels that
 *     name no node are ignored.
 *   d_out_label [capacity] (device, may be NULL): the label of each entry's
 *     unit (the accepted node, or the opened leaf holding the particle).
 *   d_out_owner [n] (device, may be NULL): for every input particle, the
 *     index of the entry that holds it (itself when emitted as a real
 *     particle, else its pseudo-particle).
 * A node label is a 1 followed by the node's octant digits (x + 2y + 4z,
 * 3 bits per level) from the root down; the root is 1. */
int build_pseudo_particles_open(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const double *d_h,
                                const double *d_m, int32_t n_src, const double *h_sources,
                                const sphmap_pseudo_opts *opts, int64_t n_open, const uint64_t *d_open_labels,
                                int64_t capacity, double *d_out_xyz, double *d_out_h, double *d_out_m,
                                double *d_out_s, int32_t *d_out_kind, int64_t *d_out_first, int64_t *d_out_count,
                                int32_t *d_out_branch, uint64_t *d_out_label, int64_t *d_out_owner,
                                int64_t *n_out, sphmap_pseudo_stats *stats, void *stream);

/* Pseudo-particles from the paper's own binary k-d tree (Sec. 2.2.1, 2.4).
 * Tree: recursive coordinate bisection of the unit cube, each node's domain
 * split through the centre of mass of its particles along the domain's
 * longest axis (first such axis on a tie; particles below the split go
 * left), until a node holds fewer than leaf_split particles, reaches
 * max_depth (<= 62) or a split would leave one side empty.  Centres of mass
 * are exact sums of m and m x rounded to fixed point 2^-K (K = 62 - the
 * binary exponent of n * max m), so the tree does not depend on summation
 * order.  Labels: root 1, children of n: 2n (left), 2n + 1 (right).
 * Walk (Sec. 2.4.1): per source, with r = |com - source| and s the node
 * size, a node reaches r_part when r - s <= r_part, r_leaf when
 * r - s <= r_leaf, and fails the opening angle when theta^2 r^2 < s^2;
 * accepted when none holds for any source and it is not in d_open_labels.
 * Emitted: accepted nodes (one particle: as itself), and leaves not
 * accepted: their particles (own h) when reaching r_part, named or single,
 * else the leaf as a pseudo-particle (the r_leaf annulus).
 * Node h: as build_pseudo_particles, over all units, or with more than
 * nf_threshold units over the trial neighbours of the k_mid neighbour-find
 * (Sec. 2.4.3): k_mid one level above the highest unit; r_cut = sqrt(3)
 * s(ancestor on k_mid), or 4 h_fact s(ancestor up_levels above) when that is
 * below 4 h_fact s (eq. compact_support_radius); trial neighbours: the units
 * whose k_mid ancestor's centre of mass lies within r_cut.
 * Arguments and outputs as build_pseudo_particles_open (opts->leaf_max is
 * unused), plus d_out_level [capacity] (nullable, each entry's node level)
 * and *k_mid (nullable: the level used, -1 when all units were summed).
 * Errors: EINVAL also for non-positive or non-finite masses. */
typedef struct {
  double r_leaf;          /* >= r_part for the annulus (= r_part: none)      */
  int32_t leaf_split;     /* split nodes holding at least this many (10)      */
  int32_t up_levels;      /* ancestor levels for the r_2h fallback (1)        */
  int64_t nf_threshold;   /* neighbour-find above this many units (10^4)      */
} sphmap_kd_opts;
int build_pseudo_particles_kd(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const double *d_h, const double *d_m,
                              int32_t n_src, const double *h_sources, const sphmap_pseudo_opts *opts,
                              const sphmap_kd_opts *kd, int64_t n_open, const uint64_t *d_open_labels,
                              int64_t capacity, double *d_out_xyz, double *d_out_h, double *d_out_m, double *d_out_s,
                              int32_t *d_out_kind, int64_t *d_out_first, int64_t *d_out_count, int32_t *d_out_branch,
                              uint64_t *d_out_label, int32_t *d_out_level, int64_t *d_out_owner, int64_t *n_out,
                              sphmap_pseudo_stats *stats, int32_t *k_mid, void *stream);

/* Resolution check of the adaptive walk (eq. resol_param, Sec. 2.4.1): a
 * pseudo-particle (kind 1) of size s whose neutral fraction f is below
 * f_neu,limit = (1/K) (K - 1 / (s / s_root)) is under-resolved.  Inputs are
 * the builder's outputs for n entries (device) and the neutral fraction of
 * each entry d_fneu [n] (device, e.g. from map_cells_to_particles of a cell
 * field).  Writes the labels of the under-resolved entries, in entry order,
 * to d_out_labels [n] (device) and their number to *n_found (host).
 * Errors: EINVAL (null pointers, s_root <= 0, K <= 1). */
int select_underresolved(sphmap_ctx *ctx, int64_t n, const int32_t *d_kind, const uint64_t *d_label,
                         const double *d_s, const double *d_fneu, double s_root, double K, uint64_t *d_out_labels,
                         int64_t *n_found, void *stream);

/* Per-particle values from the mixed set (Sec. 3.3: the refinement the paper
 * proposes over giving every member of a pseudo-particle its node's value).
 * A particle whose owner is a real entry (kind 0) takes that entry's values;
 * any other particle i takes the Shepard-normalised SPH interpolant
 *   q_i = sum_j w(r_ij / h_j) q_j / sum_j w(r_ij / h_j)
 * over all entries j with r_ij = |x_i - x_j| < 2 h_j (each entry weighted by
 * its volume (h_j / h_fact)^3 of eq. h_node times W(r_ij, h_j), which leaves
 * the dimensionless M4 kernel w), or its owner's values when no entry
 * reaches it.
 *   d_xyz [n][3]: particle positions; d_owner [n]: entry holding each particle
 *     (build_pseudo_particles_open's d_out_owner).
 *   d_entry_xyz [n_entries][3], d_entry_h, d_entry_kind: the mixed set.
 *   d_values [n_entries][ncomp]: entry values (e.g. the inverse map of the
 *     cell ionic fractions); d_out [n][ncomp].
 * All arrays device-resident, owned by the caller.  Positions must lie in
 * [0,1)^3 and owners in [0, n_entries): EINVAL otherwise, nothing written.
 * Each value is summed by one thread in a fixed order: results repeat bit
 * for bit. */
int interpolate_to_particles(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const int64_t *d_owner,
                             int64_t n_entries, const double *d_entry_xyz, const double *d_entry_h,
                             const int32_t *d_entry_kind, const double *d_values, int32_t ncomp, double *d_out,
                             void *stream);

/* interpolate_to_particles for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments, results and errors, but every buffer of
 * the call is carved from a fixed 64 MiB region of device memory that the
 * library holds on each device for the life of the process; the call makes
 * no device allocation.  n particles and n_entries entries need up to
 *   102 n_entries + 16 n bytes (+ about 100 KiB),
 * e.g. 1,048,576 particles with 167,000 entries take about 34 MB; a call
 * that needs more than 64 MiB fails with SPHMAP_EINVAL before anything is
 * enqueued.  All calls on one device share the region: calls that overlap
 * in time on one device (two streams, two contexts or two host threads)
 * race and must be serialised by the caller. */
int interpolate_to_particles_noalloc(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const int64_t *d_owner,
                                     int64_t n_entries, const double *d_entry_xyz, const double *d_entry_h,
                                     const int32_t *d_entry_kind, const double *d_values, int32_t ncomp,
                                     double *d_out, void *stream);

/* ------------------------------------------------------------------------
 * Kernel timing: when enabled, HIP events are recorded on the launch stream
 * around each launch of the named kernels ("exact_integral", "exact_redo",
 * "pair_fill", "pair_count", "cell_reduce", "reverse", "transpose",
 * "node_hsolve", "kd_build", "interp", "voronoi_lloyd", "voronoi_count",
 * "voronoi_faces").
 * sphmap_kernel_time synchronises on the recorded events and returns the
 * summed milliseconds and the number of launches since the last reset.
 * ---------------------------------------------------------------------- */
int sphmap_set_timing(sphmap_ctx *ctx, int32_t enabled);
int sphmap_kernel_time(sphmap_ctx *ctx, const char *name, double *total_ms, int64_t *launches);
int sphmap_reset_timing(sphmap_ctx *ctx);

/* Work counters of the last forward mapping (host, 8 values): [0] pairs,
   [1] faces tested, [2] faces integrated (within 2h), [3] edges visited,
   [4] edges integrated (edge line within 2h).  [5] and [6]: closed-form
   evaluations -- binary64 path: antiderivative evaluations in the inner
   (U < 1) and outer (1 <= U < 2) regime; mixed path: single-regime pieces
   (one per integrated edge, two when its range crosses U = 1) with inner /
   outer coefficients (a piece with twice their difference counts as
   inner).  [7] mixed path: pairs recomputed by the second, binary64-geometry
   kernel (16 lanes per pair): an edge line within 1e-2 h of the particle, a
   foot point on an edge line, a face plane through the particle, a cell
   smaller than h/4, more than 64 faces or 256 candidate edges, a particle
   on the boundary; binary64 path: 0.  Counting costs time; it is only done
   when enabled (sphmap_set_counting). */
int sphmap_set_counting(sphmap_ctx *ctx, int32_t enabled);

/* Launch-shape autotuning of the mixed-path Exact integral (the persistent
   kernel's workgroups per compute unit and 64-pair chunks taken per work
   fetch).  When enabled, the first forward call whose pair total falls in
   a new power-of-two class times every candidate shape -- all compute the
   same weights -- and keeps the fastest for later calls of that class
   (enabled or not).  Counting calls are never tuned.
   sphmap_tuned_shape reports the shape kept for the class of n_pairs:
   blocks_per_cu = 0 when none is kept (the default shape is then used). */
int sphmap_set_autotune(sphmap_ctx *ctx, int32_t enabled);
int sphmap_tuned_shape(sphmap_ctx *ctx, int64_t n_pairs, int32_t *blocks_per_cu, int32_t *chunks_per_fetch,
                       double *ms);
int sphmap_work_counters(sphmap_ctx *ctx, int64_t *out8);

#ifdef __cplusplus
}
#endif
#endif /* SPHMAP_H */
