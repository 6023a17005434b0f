/*
 * rc.h -- C ABI of the MI355X forest-of-octrees raycasting library (librc.so).
 *
 * The library implements the per-view hot path of Burstedde's distributed
 * forest-of-octrees raycaster for one process's share of the forest:
 *   visibility (Sec. 3.1), ray segments per leaf (Sec. 2.3, 2.7, 3.2),
 *   sort-free compositing by octree coarsening (Sec. 2.4, 3.3, 3.4) and the
 *   adjoint of the rendered image with respect to the per-leaf coefficients.
 *
 * Conventions (every entry point):
 *  - Pointers marked [device] are HIP device pointers owned by the caller;
 *    [host] pointers are ordinary host memory.  The library never allocates
 *    persistent device memory, never frees caller memory and keeps no pointer
 *    after a call returns.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    Every call only enqueues work on `stream` and returns without waiting,
 *    except rc_forest_index and rc_camera_prepare, which are set-up calls and
 *    block until their work is done.
 *  - Return value: RC_OK (0) or a negative rc_status; rc_strerror names it.
 *    On an error return nothing has been enqueued.  Capacity overflows that
 *    can only be detected on the device are reported through the device
 *    status word counts[3] of the rc_vforest (see rc_prune_visible).
 *  - Results are deterministic: no floating-point atomics are used, so
 *    repeated calls on identical inputs give bitwise identical outputs.
 *
 * Geometry and ordering (Sec. 2.1, 3): a forest is a set of trees; each tree
 * is the unit reference cube subdivided into leaves.  Leaves are given in
 * space-filling-curve order: tree-major, then by the Morton key of the anchor
 * (x bit least significant).  A leaf at level l with integer anchor (x, y, z)
 * covers [x, x + 2^(19-l)) * 2^-19 per axis.  Child and corner ids are
 * c = bx + 2 by + 4 bz.
 *
 * Camera (Sec. 2.2, eq. ray): 20 doubles
 *   o[3] position, v[3] view vector (n = |v| is the projection-plane
 *   distance), t[3] right, u[3] up (t, u, v/n orthonormal, t x u = -v/n),
 *   ell pixel edge length on the projection plane, zfar far distance (> n),
 *   w, h pixel counts, ortho flag (0 = perspective, 1 = orthographic along
 *   v/n with the ray of pixel (i, j) starting at
 *   o + ell((i-(w-1)/2) t + (j-(h-1)/2) u)), background intensity I_b, 0, 0.
 *   The ray of pixel (i, j) is o + alpha r, r = v + ell((i-(w-1)/2) t +
 *   (j-(h-1)/2) u), clipped to depths [n, zfar] (alpha in [1, zfar/n]).
 *   Images are row-major [j][i] with j = 0 the bottom row.
 */
#ifndef RC_H
#define RC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rc_status;

#define RC_OK 0
#define RC_EINVAL (-1)        /* bad argument: null pointer, bad size, bad camera */
#define RC_EUNSUPPORTED (-2)  /* unsupported geometry / field / integrator combination */
#define RC_EWORKSPACE (-3)    /* workspace smaller than rc_workspace_bytes() */
#define RC_ECAPACITY (-4)     /* a caller buffer is too small (host-detectable case) */
#define RC_EFOREST (-5)       /* leaves not in SFC order or overlapping */
#define RC_EHIP (-6)          /* a HIP runtime call failed */

#define RC_QMAXLEVEL 19
#define RC_CAMERA_DOUBLES 20
#define RC_ABSENT (-1)        /* child slot without a node in this share */

#define RC_MAXTREES 64
#define RC_MAXCH 3          /* channels per call (RGB) */
#define RC_MAXLISTS 16     /* shares rc_merge_lists takes at once */

enum {
    RC_GEOM_UNIT_CUBE = 0,
    RC_GEOM_SHELL6 = 1,
    RC_GEOM_SURFACE = 2,
    RC_GEOM_SURFACE2 = 3,
    RC_GEOM_SURFACE3 = 4,
    RC_GEOM_VOLUME2 = 5,
    RC_GEOM_VOLUME3 = 6
};
enum { RC_FIELD_CONST = 0, RC_FIELD_TRILINEAR = 1, RC_FIELD_CONST_EQ = 2, RC_FIELD_SURFACE = 3 };
enum { RC_INT_ANALYTIC = 0, RC_INT_RK4 = 1, RC_INT_GAUSS2 = 2, RC_INT_SIMPSON = 3 };
#define RC_ADAPT_MAXDEPTH 16  /* deepest halving of the adaptive recursion */

/* One process's share of a forest (Sec. 2.1): leaves in SFC order.
 *
 * RC_GEOM_UNIT_CUBE: one tree, the identity map of the unit cube.
 * RC_GEOM_SHELL6: six trees, the equiangular cubed-sphere shell (eq.
 *   geometrytrafo with a smooth map per tree): tree k has axis m = k / 2, sign
 *   sg = +1 for even k and -1 for odd k, frame e1 = unit(m+1), e2 = unit(m+2),
 *   e3 = sg unit(m), and maps t in [0,1]^3 to
 *   x = r (a e1 + b e2 + e3) / sqrt(1 + a^2 + b^2) with a = tan(pi/4 (2 t1 - 1)),
 *   b = tan(pi/4 (2 t2 - 1)), r = r0 + (r1 - r0) t3.  geom_table holds
 *   [r0, r1, L, tan(pi/4 (2 i / 2^L - 1)) for i = 0 .. 2^L] (entries 0, 2^(L-1),
 *   2^L exactly -1, 0, 1); leaves may not be finer than level L.
 * RC_GEOM_SURFACE: 1 .. 6 quadtrees, each placed in space by a bilinear map
 *   J(t1, t2) = P00 (1-t1)(1-t2) + P10 t1 (1-t2) + P01 (1-t1) t2 + P11 t1 t2
 *   (a surface, Sec. 2.8; the bilinear case of App. A.1).  Leaves have z = 0
 *   and (x, y) anchors in the tree's parameter square.  geom_table holds 12
 *   doubles per tree: P00, P10, P01, P11.
 * RC_GEOM_SURFACE2, RC_GEOM_SURFACE3: as RC_GEOM_SURFACE with each tree's map
 *   the tensor product of degree-R Lagrange polynomials (R = 2, 3) on the
 *   Gauss-Lobatto nodes of [0, 1] (eq. nodal, eq. tensorgeom): geom_table
 *   holds (R+1)^2 control points z_{m1, m2} of 3 doubles per tree, m1 fastest
 *   (the map's values at the node pairs).
 * RC_GEOM_VOLUME2, RC_GEOM_VOLUME3: 1 .. 6 octrees, each mapping its reference
 *   cube by the tensor product of degree-R Lagrange polynomials (R = 2, 3) on
 *   the Gauss-Lobatto nodes (eq. nodal, eq. tensorgeom; curved elements,
 *   Sec. 2.1): geom_table holds (R+1)^3 control points z_{m1, m2, m3} of 3
 *   doubles per tree, m1 fastest, then m2 (the map's values at the node
 *   triples).  Fields are per leaf in its reference coordinates, as on the
 *   unit cube. */
typedef struct rc_forest {
    int32_t ntrees;             /* trees in the share: 1 (unit cube), 6 (shell), 1 .. 6 (surfaces, volumes) */
    int32_t geom;               /* RC_GEOM_* */
    int64_t nleaves;            /* N >= 1 */
    const int64_t *tree_begin;  /* [host] ntrees + 1 leaf offsets per tree */
    const uint8_t *level;       /* [device] N leaf levels, 0 .. RC_QMAXLEVEL */
    const uint32_t *x, *y, *z;  /* [device] N anchors in units of 2^-19 */
    const double *geom_table;   /* [device] geometry table (RC_GEOM_SHELL6, RC_GEOM_SURFACE), else NULL */
} rc_forest;

/* Per-leaf coefficient data (Sec. 2.3): absorption kappa (beta in the paper)
 * and emission eps (gamma), leaf-major [leaf][corner] in SFC order: one value
 * per leaf for per-leaf constants, eight consecutive corner values (corner
 * c = bx + 2 by + 4 bz, 32-byte aligned rows) for trilinear data interpolated
 * in leaf reference coordinates.  nch channels (1 .. RC_MAXCH, e.g. RGB, each
 * converted to its own (A, B) as in Sec. 4.1) follow one another:
 * kappa[ch][leaf][corner].  RC_FIELD_SURFACE (surface forests only,
 * analytic method): kappa holds the surface's transparency A_s
 * and eps its intensity I_s at the leaf's four corners (corner c = bx + 2 by),
 * interpolated bilinearly at the hit; the hit contributes A = A_s^(1/cos phi),
 * phi the angle between the ray and the patch normal, and B = I_s (1 - A)
 * (eq. ABphi, eq. BIrelation; A_s = 0 is an opaque surface). */
typedef struct rc_fields {
    int32_t kind;               /* RC_FIELD_CONST, RC_FIELD_TRILINEAR, RC_FIELD_CONST_EQ (constant
                                   kappa and equilibrium intensity I = eps / kappa in place of eps,
                                   eq. BIrelation: B = I (1 - A); analytic integration only) or
                                   RC_FIELD_SURFACE */
    int32_t nch;                /* channels, 1 .. RC_MAXCH */
    const float *kappa;         /* [device] nch * N * ncorner, 16-byte aligned */
    const float *eps;           /* [device] nch * N * ncorner, 16-byte aligned */
} rc_fields;

/* Segment integrator (Sec. 2.3, 2.7):
 *  RC_INT_ANALYTIC  closed form for constant coefficients (eq. ABconstant);
 *  RC_INT_RK4       classical RK4 steps of eq. RKresultAB;
 *  RC_INT_GAUSS2    implicit Gauss, two stages at 1/2 -+ sqrt(3)/6 (eq. gaussAB);
 *  RC_INT_SIMPSON   Simpson quadrature of the closed form (eq. simpson).
 * A segment is split into `substeps` equal pieces combined with the group
 * operation, nearest first.  c_rk > 0 adds the recursion of Alg. adaptiverk: a
 * piece whose stage points give dx kappa(xi_i) > c_rk is replaced by its two
 * halves, down to RC_ADAPT_MAXDEPTH halvings.  The pieces are the dyadic
 * fractions [k, k+1] / 2^d of the segment counted from its near end, their
 * stage points at ray parameter s_in + ((k + 1 - c_i) / 2^d) (s_out - s_in)
 * in FP64, and the split test uses FP64 trilinear values, so that the
 * decisions are reproducible.  Gauss, Simpson and c_rk > 0 need a power of
 * two `substeps`. */
typedef struct rc_integrator {
    int32_t method;             /* RC_INT_* (analytic needs constant fields) */
    int32_t substeps;           /* pieces per segment, 1 .. 64 */
    double c_rk;                /* stability parameter of the recursion; 0 = off */
} rc_integrator;

/* Launch shapes of the grid-stride kernels, in 256-thread workgroups; 0 (or a
 * NULL rc_tuning pointer) selects the default.  Forward results do not depend
 * on these values; adjoint sums are deterministic for a given value. */
#define RC_MAX_FOLD_RUN 2
typedef struct rc_tuning {
    int32_t seg_blocks;   /* rc_segments (default 8192; 16384 for the shell and the
                             integrator variants, 1024 for degree-R surfaces) */
    int32_t fold_blocks;  /* level passes: rc_composite's default 8192; the adjoint's, the fused channels'
                             and the shell's 4096 */
    int32_t root_blocks;  /* root passes over the image pixels (default 4096) */
    int32_t adj_blocks;   /* rc_segments_backward leaf adjoint (default 2048) */
    uint32_t fold_skip;   /* rc_composite and rc_render on the unit cube, one channel: bit l set (1 <= l <
                             maxlevel) leaves level l's node records unwritten; the pass of the nearest
                             written level above (or the root pass) folds the skipped levels itself, in the
                             same association, so images are bit for bit the same.  At most
                             RC_MAX_FOLD_RUN consecutive levels may be skipped (RC_EINVAL otherwise); bits
                             outside 1 .. maxlevel - 1 are ignored, and rc_render keeps the levels whose
                             walk would reach a leaf.  Default 0.  The node records of a call with
                             fold_skip != 0 are NOT valid input to rc_segments_backward. */
} rc_tuning;

/* Static node table of a forest share: the internal nodes above the leaves,
 * level-major and in SFC order within a level.  Built by rc_forest_index.
 * A child slot holds an internal node index (>= 0), RC_ABSENT, or a leaf
 * l encoded as -2 - l. */
typedef struct rc_index {
    int32_t maxlevel;                       /* [out] deepest leaf level */
    int32_t leaf_levels;                    /* [out] bit l set when some leaf has level l */
    int64_t ninternal;                      /* [out] internal nodes (required capacity on RC_ECAPACITY) */
    int64_t cap_internal;                   /* [in] capacity of the arrays below */
    int64_t level_begin[RC_QMAXLEVEL + 2];  /* [out] internal nodes of level l: [level_begin[l], level_begin[l+1]) */
    int32_t root;                           /* [out] root node of tree 0 (same encoding as a child slot) */
    int32_t ntrees;                         /* [out] trees */
    int32_t roots[RC_MAXTREES];             /* [out] root node of every tree (same encoding) */
    int32_t *child;                         /* [device] cap_internal * 8 */
    uint8_t *level;                         /* [device] cap_internal */
    uint32_t *x, *y, *z;                    /* [device] cap_internal anchors */
    uint8_t *tree;                          /* [device] cap_internal: tree of each internal node */
} rc_index;

/* The visible forest ("vforest", Sec. 3.1) of a set of cameras, written by
 * rc_prune_visible and read by the other calls.  Capacities are inputs. */
typedef struct rc_vforest {
    int64_t cap_vis;       /* capacity of the visible (camera, leaf) list; at most 2^31 - 2, else every
                              call that takes the vforest returns RC_EUNSUPPORTED */
    int64_t cap_cand;      /* capacity of leaf candidate records (camera, leaf, pixel) */
    int64_t cap_rec;       /* capacity of internal-node records (camera, node, pixel) */
    int32_t *vis_leaf;     /* [device] cap_vis: leaf of visible pair v (camera-major, SFC order) */
    int16_t *vis_cam;      /* [device] cap_vis: camera of pair v */
    int16_t *vis_rect;     /* [device] cap_vis * 4: pixel rectangle i0, i1, j0, j1 (inclusive) */
    int64_t *cand_offset;  /* [device] cap_vis + 1: first candidate of pair v; [nvis] = ncand */
    int32_t *leaf_vis;     /* [device] ncams * N: pair index of (camera, leaf), -1 if invisible */
    int16_t *node_rect;    /* [device] rc_node_slots() * 4: rectangle per (level >= 1, camera, node) */
    int64_t *node_offset;  /* [device] rc_node_slots() + 1: first record per slot */
    int64_t *counts;       /* [device] 4: nvis, ncand, nrec, status (nonzero = capacity exceeded) */
    int32_t *cand_chunk;   /* [device] cap_cand / 64 + 2: visible pair holding candidate 64 w */
    int32_t *rec_chunk;    /* [device] cap_rec / 64 + 2: slot holding internal-node record 64 w */
    void *child_desc;      /* [device] ncams * ninternal * 8 * 16 bytes: children of every internal node in
                              view order, each with its rectangle and record offset */
} rc_vforest;

/* Name of a status code. */
const char *rc_strerror(rc_status s);

/* Bytes of device workspace the calls need for this forest, index, camera
 * count and (for rc_segments_backward) vforest capacities; index and vf may be
 * NULL before they exist (rc_forest_index needs neither). */
size_t rc_workspace_bytes(const rc_forest *forest, const rc_index *index, int32_t ncams, const rc_vforest *vf);

/* Bytes of the device camera block for ncams cameras. */
size_t rc_camera_bytes(int32_t ncams);

/* Number of (level >= 1, camera, internal node) slots: sizes node_rect/node_offset. */
int64_t rc_node_slots(const rc_index *index, int32_t ncams);

/*
 * Validate cams[ncams][20] [host] (Sec. 2.2: orthonormal left-handed frame,
 * n > 0, zfar > n, ell > 0, w, h in 1 .. 32767) and upload them to dcams
 * [device, rc_camera_bytes(ncams)] with the derived quantities (n, v/n, image
 * offsets: camera k's pixels start at the sum of the earlier w*h).  Blocks.
 * Returns RC_EINVAL on a bad camera.  *total_pixels receives the image size.
 */
rc_status rc_camera_prepare(const double *cams, int32_t ncams, void *dcams, int64_t *total_pixels,
                            void *stream);

/*
 * Build the static node table of a forest share (the trees above the leaves,
 * Sec. 2.1).  Validates that the leaves are in strict SFC order without
 * overlap (RC_EFOREST otherwise).  If index->cap_internal is too small,
 * returns RC_ECAPACITY with index->ninternal set to the required capacity.
 * Blocks until done.
 */
rc_status rc_forest_index(const rc_forest *forest, rc_index *index, void *ws, size_t ws_bytes, void *stream);

/*
 * Visibility and work partition (Sec. 3.1, Sec. 2.2 "our (2D) AABB"): for
 * every (camera, leaf) and (camera, internal node) compute the pixel
 * rectangle of the node's camera-aligned bounding box, clipped to [n, zfar]
 * and projected to the image; a node is visible iff the rectangle holds a
 * pixel centre.  Writes the compacted visible list in SFC order per camera
 * (vis_*), the exclusive scan of rectangle areas (cand_offset, the visible
 * pixel weight of the paper's repartition), leaf_vis, the internal-node
 * rectangles and record offsets, and counts = {nvis, ncand, nrec, status}.
 * If a count exceeds its capacity, status becomes nonzero and the later
 * calls do nothing; the caller reads counts and retries with more room.
 * RC_GEOM_SHELL6: node rectangles are unions of the children's (curved
 * elements' boxes do not nest), so nrec is exact only once cap_vis and
 * cap_cand suffice; a retry may then ask for more record room once more.
 */
rc_status rc_prune_visible(const rc_forest *forest, const rc_index *index, const void *dcams, int32_t ncams,
                           rc_vforest *vf, void *ws, size_t ws_bytes, void *stream);

/*
 * rc_prune_visible without a workspace argument and without allocating, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, hosts that forbid hipMalloc).  The workspace is a file-scope
 * device array of RC_STATIC_SCRATCH_BYTES per device, held from the library's
 * load until the process ends; its address is looked up once per device, on
 * the first call with that device current (make that first call outside
 * stream capture).  Outputs are bitwise those of rc_prune_visible.  Returns
 * RC_EWORKSPACE when the call would need more than RC_STATIC_SCRATCH_BYTES,
 * i.e. when rc_workspace_bytes(forest, index, ncams, NULL) exceeds it (about
 * 8 M (camera, leaf) and (camera, internal node) items), and the errors of
 * rc_prune_visible otherwise.  Calls on one device share the array: calls
 * that overlap in time on one device (two streams, two host threads) race and
 * must be ordered by the caller.
 */
#define RC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
rc_status rc_prune_visible_static(const rc_forest *forest, const rc_index *index, const void *dcams, int32_t ncams,
                                  rc_vforest *vf, void *stream);

/*
 * Ray segments of every candidate (Sec. 3.2): for each visible pair and each
 * pixel of its rectangle, intersect the pixel's ray with the leaf (a slab test
 * whose shared faces give bitwise equal crossing depths) and integrate
 * I' = eps - kappa I over the hit interval from the far end toward the camera
 * (eq. ABconstant, or RK4 per eq. RKresultAB over equal substeps combined by
 * eq. aggregate).  rec_leaf[device, nch * cap_cand * 2] receives (A, B) per
 * candidate and channel (channel-major blocks of cap_cand records), the
 * identity (1, 0) on a miss.  With several channels the pairing runs once and
 * every channel is integrated on the same segments (the unit cube's closed
 * form and fixed-step RK4; the other paths take one channel at a time).
 * Optional debug outputs (NULL to skip): hit[device, cap_cand] 1/0 and
 * sio[device, cap_cand * 2] the hit interval in the ray parameter (alpha for
 * perspective, depth for orthographic), zeros on a miss.
 *
 * RC_GEOM_SHELL6 forests: a ray meets a curved element in up to two
 * intervals (bounded by two planes through the centre per tangent axis and
 * two spheres), so each candidate holds two records of four floats
 * (s_in, s_out, A, B), nearer first, an unused one (1, 0, 1, 0) (s_in > s_out):
 * rec_leaf[device, cap_cand * 8], hit[] the number of intervals (0..2) and
 * sio[device, cap_cand * 4] both intervals in FP64.  Field values at the RK4
 * points use the reference coordinates obtained by inverting the tree map
 * with Newton's method in FP64.
 *
 * RC_GEOM_SURFACE forests: the ray is intersected with the leaf's whole tree
 * patch (App. A.1: projected onto two directions normal to the ray, the
 * bilinear system leaves a quadratic in t2), and each hit inside the clip
 * range belongs to the leaf whose half-open parameter square holds it, so a
 * ray crossing shared leaf edges is counted once.  A candidate holds up to two
 * zero-length records (s, s, A, B) in the layout of the shell, an unused one
 * (1, 0, 1, 0); hit[] counts them and sio[] holds (s, s) per hit.
 *
 * RC_GEOM_SURFACE2 / 3 forests (App. A.1, higher degree): the two planes
 * through the pixel's ray, applied to the control points moved to camera
 * space (eq. camerapoints), give two polynomials whose Bernstein coefficients
 * over the leaf square bound them.  The leaf square is searched depth first:
 * sub-squares where either keeps one sign (beyond a relative 1e-10) are
 * dropped; on the others Krawczyk's test (the square widened by a relative
 * 1e-9) decides no root, exactly one root (Newton's method from the centre) or
 * undecided (split into four, at most 16 levels below the leaf, then Newton).
 * A converged root is polished canonically on the tree's polynomials (snapped
 * to a 2^-40 grid, two Newton steps) so that it counts once, in the leaf whose
 * half-open square holds it.  The search visits at most 2048 sub-squares per
 * candidate (a ray lying in the surface decides none).  A candidate keeps its
 * two nearest hits; hit[] counts all.  Leaf
 * rectangles come from the camera-aligned box of the leaf's Bernstein
 * coefficients (App. A.2).
 *
 * RC_GEOM_VOLUME2 / 3 forests (curved elements, Sec. 2.1; App. A.1): the ray
 * crosses the leaf's six faces, each a degree-R patch searched as the
 * degree-R surfaces above (crossings polished canonically on the tree's face
 * polynomial, so that leaves sharing a face find the same depth); the
 * crossings cut the clip range into pieces, a piece whose midpoint maps back
 * into the leaf's cube (Newton's method on the tree map, FP64) is inside, and
 * adjacent inside pieces join.  Each interval is integrated with RK4 over 1,
 * 2, 4 or 8 equal substeps with field points mapped back the same way, or in
 * closed form for constant fields (analytic).  Records, hit[] and sio[] as
 * for the shell: the two nearest intervals, hit[] counting all.  Other
 * integrators: RC_EUNSUPPORTED.  Leaf rectangles come from the camera-aligned
 * box of the Bernstein coefficients of the map over the leaf's cube.
 */
rc_status rc_segments(const rc_forest *forest, const rc_fields *fields, const void *dcams, int32_t ncams,
                      const rc_vforest *vf, const rc_integrator *integ, float *rec_leaf, uint8_t *hit,
                      double *sio, const rc_tuning *tune, void *stream);

/*
 * Sort-free compositing (Sec. 2.4, 3.3): coarsen the octree level by level;
 * the record of an internal node at a pixel is the group product of its
 * children's records taken in the camera's view order (the Morton child id
 * with every bit flipped where the camera lies on the high side of the
 * node's midplane), absent or invisible children acting as the identity.
 * The roots are folded straight into the images: A, B and I = A I_b + B
 * [device, total_pixels floats each; total_pixels as returned by
 * rc_camera_prepare].  One channel per call: for channel ch pass that
 * channel's blocks of rec_leaf and rec_node and its images.  rec_node
 * [device, cap_rec * 2] holds the internal-node records (kept for the
 * adjoint).  vf->cap_cand must be at least 1: rec_leaf always holds at least
 * one record.
 *
 * RC_GEOM_SHELL6 forests: records hold two intervals as in rc_segments
 * (rec_node [device, cap_rec * 8]); a node's intervals are its children's
 * merged by depth, touching ones combined, and the six roots' intervals are
 * folded in depth order.  Surface forests: the same with the hits as
 * zero-length intervals (a bilinear tree's patch meets a ray at most twice; a
 * node of a degree-R tree keeps two runs of hits, joining the closest runs
 * beyond that).
 */
rc_status rc_composite(const rc_forest *forest, const rc_index *index, const void *dcams, int32_t ncams,
                       const rc_vforest *vf, const float *rec_leaf, float *rec_node, int64_t total_pixels,
                       float *A, float *B, float *I, const rc_tuning *tune, void *stream);

/*
 * The forward after rc_prune_visible in one call: rc_segments followed by
 * rc_composite, with the intra-tile fold where it applies (unit-cube forests
 * deeper than one leaf, one channel, the closed form or RK4 over fixed
 * substeps).  There the coarsening's pass of each level computes the segments
 * of its nodes' leaf children at every pixel of the nodes' rectangles (Sec. 3.2)
 * and folds them with the internal children's records in the camera's view
 * order (Sec. 3.3 aggregation of child segments, Sec. 2.4 eq. aggregate),
 * keeping them in registers and LDS: no leaf record is written, and rec_leaf
 * may be NULL.  A, B, I and rec_node are bitwise those of rc_segments followed
 * by rc_composite.  Elsewhere (curved geometry, several channels, the other
 * integrators, a forest of one leaf) the call runs rc_segments and
 * rc_composite (rc_composite_channels for nch > 1) into rec_leaf, which must
 * then be given.  rc_segments_backward needs rec_leaf: after rc_render, run
 * rc_segments before the adjoint.  Arguments, layouts and errors as for
 * rc_segments and rc_composite; all of them are checked before anything is
 * enqueued.
 */
rc_status rc_render(const rc_forest *forest, const rc_index *index, const rc_fields *fields, const void *dcams,
                    int32_t ncams, const rc_vforest *vf, const rc_integrator *integ, float *rec_leaf, float *rec_node,
                    int64_t total_pixels, float *A, float *B, float *I, const rc_tuning *tune, void *stream);

/*
 * rc_composite for nch channels (1 .. RC_MAXCH, Sec. 4.1: each channel its own
 * (A, B)) in one call, on channel-major blocks: rec_leaf [device, nch *
 * cap_cand * 2], rec_node [device, nch * cap_rec * 2] and A, B, I [device,
 * nch * total_pixels floats each], channel ch's block at ch times the block
 * size.  On the unit cube one pass locates each record's node and pixel and
 * folds every channel there; each channel's images and records are bitwise
 * those of rc_composite on that channel's blocks.  Other geometries (records
 * of cap_cand * 8 and cap_rec * 8 floats per channel) run rc_composite per
 * channel.  RC_EINVAL for nch outside 1 .. RC_MAXCH.
 */
rc_status rc_composite_channels(const rc_forest *forest, const rc_index *index, const void *dcams, int32_t ncams,
                                const rc_vforest *vf, int32_t nch, const float *rec_leaf, float *rec_node,
                                int64_t total_pixels, float *A, float *B, float *I, const rc_tuning *tune,
                                void *stream);

/*
 * One share's image as per-pixel lists (Sec. 3.3 coarsening stopped at the
 * share's maximal complete subtrees, Sec. 3.5 per-pixel segment lists).  The
 * forest is a share: a contiguous curve-order range of a larger forest's
 * leaves that tile the curve interval from the first leaf's anchor to the end
 * of the last leaf, indexed on its own (missing children are RC_ABSENT).  A
 * node is complete when its curve interval lies inside the share's; the units
 * are the leaves and complete nodes under an incomplete parent, and the root
 * when it is complete.  For every pixel whose ray crosses a unit's box, one
 * entry (s_in, s_out, A, B) [4 floats]: the canonical slab interval of the
 * box (FP64, stored as float) and the unit's record there (its children
 * folded in view order, as rc_composite does).  Every pixel's entries are
 * sorted by (s_in, s_out, A, B).  Call after rc_prune_visible and
 * rc_segments of the share; rec_node as for rc_composite (rewritten here).
 * list_offset [device, total_pixels + 1 int64]: pixel p's entries are
 * [list_offset[p], list_offset[p + 1]) of entries [device, cap_entries * 4
 * floats]; *n_entries [device] receives the total.  Entries are written only
 * when the total fits cap_entries (cap_entries = 0 asks for the count only);
 * the caller reads n_entries and calls again with more room otherwise.
 * ws [device, rc_lists_workspace_bytes()].  RC_GEOM_SHELL6 and surface
 * forests: RC_EUNSUPPORTED.
 */
size_t rc_lists_workspace_bytes(const rc_index *index, int32_t ncams, int64_t total_pixels);
rc_status rc_composite_lists(const rc_forest *forest, const rc_index *index, const void *dcams, int32_t ncams,
                             const rc_vforest *vf, const float *rec_leaf, float *rec_node, int64_t total_pixels,
                             int64_t *list_offset, float *entries, int64_t cap_entries, int64_t *n_entries,
                             void *ws, size_t ws_bytes, const rc_tuning *tune, void *stream);

/*
 * Merge the lists of nlists (1 .. RC_MAXLISTS) shares into images (Sec. 3.5,
 * Sec. 2.5).  Per pixel, the depths where entries start or end cut the ray
 * into elementary intervals; over each, every entry covering it contributes
 * the piece of its length fraction (eq. segsplit, the ratio (1 - A^f) / (1 - A)
 * evaluated through expm1), several covering entries are averaged (geometric
 * mean of the A, arithmetic mean of the B: eq. segaverage over all of them),
 * and the intervals are folded nearest first (eq. aggregate).  A zero-length
 * entry is folded whole at its depth.  list_offsets, entries [host arrays of
 * nlists device pointers] in the layout rc_composite_lists writes, for the
 * same cameras: within one list, a pixel's entries are sorted and disjoint
 * (they may touch); a pixel whose list breaks this gets NaN.  A, B and
 * I = A I_b + B [device, total_pixels floats each].  overlaps [device, one
 * int64, or NULL] is incremented by the number of entries that start inside
 * an entry of another list.  Shares of one forest meet at shared faces with
 * bitwise equal depths, so their lists touch and never overlap.
 */
rc_status rc_merge_lists(const void *dcams, int32_t ncams, int64_t total_pixels, int32_t nlists,
                         const int64_t *const *list_offsets, const float *const *entries, float *A, float *B,
                         float *I, int64_t *overlaps, void *stream);

/*
 * Adjoint of the images with respect to the coefficients.  The operation
 * differentiated is the forward path above: the image of a pixel is the group
 * product of its segments (Sec. 2.4, eq. aggregate), so with I = A_front (A_k
 * J + B_k) + B_front for every segment k the derivative of I with respect to
 * segment k's pair is (T J, T), T the product of the A in front of it and J the
 * intensity entering it from behind.  The group inverse (Sec. 2.4,
 * eq. identityinverse) and the reversal of a segment (Sec. 2.6, eq. swapxy,
 * eq. substbetagamma) would recover J from the whole pixel by dividing by
 * T A_k; this call instead passes both factors top-down.  Given
 * dL_dI [device, total_pixels], pass (g T_front, J_behind) down the same
 * hierarchy (T_front: transmittance in front of a node, J_behind: intensity
 * entering it from behind; no division), so that a segment receives
 * dL/dA = g T J and dL/dB = g T; then differentiate each segment's
 * evaluation (recomputed from the coefficients) and reduce per leaf in a
 * fixed order.  Several channels: rec_leaf, rec_node, dL_dI and the
 * gradients hold channel-major blocks as in rc_segments and rc_composite.
 * dL_dkappa, dL_deps [device, layout of rc_fields] are overwritten, or added
 * to when accumulate != 0.  adj_leaf [device, cap_cand * 2] and adj_node
 * [device, cap_rec * 2] are scratch.  Differentiated: the closed form (for
 * RC_FIELD_CONST_EQ with respect to kappa and I); RK4, Gauss and Simpson over
 * 1, 2, 4 or 8 equal pieces; and the recursion (c_rk > 0) of the three, its
 * split decisions held fixed.  RC_EUNSUPPORTED for other piece counts without
 * the recursion, and for RC_GEOM_SHELL6 and surface forests.
 */
rc_status rc_segments_backward(const rc_forest *forest, const rc_index *index, const rc_fields *fields,
                               const void *dcams, int32_t ncams, const rc_vforest *vf,
                               const rc_integrator *integ, const float *rec_leaf, const float *rec_node,
                               int64_t total_pixels, const float *dL_dI, float *adj_leaf, float *adj_node,
                               float *dL_dkappa, float *dL_deps, int32_t accumulate, void *ws, size_t ws_bytes,
                               const rc_tuning *tune, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RC_H */
