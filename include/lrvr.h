/*
 * lrvr.h -- C ABI of the MI355X (gfx950) library for direct volume rendering
 * of trivariate LR-spline volumes (Fuchs, Barrowclough, Hjelmervik, Dahl:
 * "Direct interactive visualization of locally refined spline volumes for
 * scalar and vector fields").
 *
 * The calls follow the paper's problem statement: an LR-spline volume (Eq. 2,
 * Sec. 3.1) gets an element look-up structure built on the host (Sec. 3.2.1),
 * is converted to per-element Bezier blocks (Sec. 3.2.3), and is rendered by
 * emission-absorption ray casting (Sec. 4, Eq. 3, Alg. 2) with the adaptive
 * sampling distance of Eq. 4.  lr_render_backward adds the adjoint of the
 * render with respect to the Bezier coefficients and the transfer function.
 *
 * Conventions shared by every call
 *  - Parameter domain [0,1]^3.  An element is a box [lo, hi) per axis, closed
 *    at hi = 1; elements partition the domain, so every point lies in exactly
 *    one element.  Boxes are 6 numbers: lo x, lo y, lo z, hi x, hi y, hi z.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary process memory owned by the caller.  The library
 *    never frees caller memory and never keeps a pointer after a call returns.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  Device
 *    work is enqueued asynchronously on it; the caller synchronises.
 *  - Every call returns an lr_status.  Nothing aborts or throws.  On error
 *    nothing has been enqueued unless the error is LR_EHIP (a launch failed),
 *    and lr_last_error() returns a text for the calling thread.
 *  - Only this library's kernels compute; no call falls back to the host for
 *    device work.
 */
#ifndef LRVR_H
#define LRVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lr_status;
#define LR_OK 0
#define LR_EINVAL (-1)      /* bad argument: NULL pointer, size, degree, mode */
#define LR_ENOTPOW2 (-2)    /* forest block count not a power of two in [1,512] */
#define LR_EKNOT (-3)       /* a box coordinate is not exactly representable in FP32 */
#define LR_ECAPACITY (-4)   /* an output buffer is too small (needed size is reported) */
#define LR_EHIP (-5)        /* HIP runtime or launch failure */
#define LR_EPARTITION (-6)  /* elements overlap, leave gaps or leave [0,1]^3 */

#define LR_F32 0
#define LR_F16 1
#define LR_F64 2

#define LR_STEP_FIXED 0     /* n_fixed_steps equal segments, sampled at midpoints */
#define LR_STEP_ADAPTIVE 1  /* Eq. 4: ds = 2^-d * min side of the sample's element */

#define LR_COLOR_LUT 0      /* scalar field: RGBA from the table */
#define LR_COLOR_HUE 1      /* 3-vector field: opacity from the table at |v|,
                               RGB = hsv(atan2(v_y, v_x)/2pi, 1, 1) */

#define LR_PERSP 0
#define LR_ORTHO 1

#define LR_LOOKUP_FOREST 0  /* k-d forest (Sec. 3.2.1, Alg. 1); also the O(1) table when
                               every block holds one element */
#define LR_LOOKUP_OCTREE 1  /* element octree of a dyadic mesh (Sec. 3.2, Sec. 3.2.2) */

/* Gradient-based local illumination (Sec. 4.1): C_src is multiplied by
 * I = max(0.4, |l . n|), n the unit gradient of the scalar field (of |f| for
 * 3-vectors, i.e. sum_q f_q grad f_q normalised), evaluated from the same
 * Bezier block as the value; I = 0.4 where the gradient is zero. */
#define LR_SHADE_NONE 0
#define LR_SHADE_DIRECTIONAL 1  /* l = light (normalised), the same for every sample */
#define LR_SHADE_HEADLIGHT 2    /* l = the ray direction (light at the eye, far away) */

#define LR_LEAF 0x80000000u /* head / child reference: element id in the low 31 bits */
#define LR_MAX_VIEWS_PER_LAUNCH 16

/* Text of the last non-OK status returned on the calling thread. */
const char* lr_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int32_t lr_version(void);

/* ------------------------------------------------------------------ k-d forest
 * Sec. 3.2.1, Alg. 1: the domain is divided into I x J x K regular blocks;
 * each block holds a k-d tree over the elements that intersect it (with
 * positive volume).  A block met by one element stores that element directly.
 * Trees are depth-balanced: at each node, for every axis the candidate split is
 * the element face strictly inside the node region that is nearest the mean of
 * those faces (ties: the smaller); the axis chosen minimises
 * max(#elements with lo < s, #elements with hi > s) (ties: the larger region
 * extent, then x < y < z).  An element straddling a split is in both subtrees.
 *
 * Device layout used by lr_render / lr_lookup:
 *   heads  uint32 [bz][by][bx]: LR_LEAF | element id, or the root node index
 *   nodes  lr_kdnode [n_nodes]
 * Descent for a point p in block b = min(floor(p * blocks), blocks - 1):
 *   r = heads[b]; while !(r & LR_LEAF): n = nodes[r];
 *   r = p[n.axis] < n.split ? n.lo : n.hi;  element = r & ~LR_LEAF.
 */
typedef struct {
    uint32_t lo;    /* child for p[axis] <  split: node index or LR_LEAF|element */
    uint32_t hi;    /* child for p[axis] >= split */
    float split;
    uint32_t axis;  /* 0, 1, 2 */
} lr_kdnode;

typedef struct {
    int64_t n_heads;        /* bx*by*bz */
    int64_t n_nodes;
    int64_t n_direct;       /* blocks whose head is an element */
    int32_t min_depth;      /* depth of a block's tree = deepest leaf; 0 if direct */
    int32_t max_depth;
    double mean_depth;
    double var_depth;       /* population variance over all blocks */
} lr_forest_stats;

typedef struct lr_forest_host lr_forest_host;   /* opaque host-side forest */

/* Builds the forest on the host (the paper precomputes it on the CPU).
 * elem_box  host double [n_elem][6]; every value in [0,1] and exact in FP32
 *           (else LR_EKNOT); lo < hi; the boxes must tile [0,1]^3
 *           (checked per block by volume, else LR_EPARTITION).
 * blocks    host int32[3], each a power of two in [1, 512] (else LR_ENOTPOW2).
 * out       receives a forest handle to free with lr_forest_free.
 * stats     optional (NULL allowed): sizes and the depth statistics. */
lr_status lr_build_forest(const double* elem_box, int64_t n_elem, const int32_t blocks[3],
                          lr_forest_host** out, lr_forest_stats* stats);

/* Copies a built forest into host buffers heads [n_heads] and nodes [n_nodes]
 * (sizes from lr_forest_stats); either pointer may be NULL to skip it. */
lr_status lr_forest_export(const lr_forest_host* f, uint32_t* heads, lr_kdnode* nodes);

void lr_forest_free(lr_forest_host* f);

/* The same build written into caller device buffers, in two phases.
 * elem_box  host float [n_elem][6] (values in [0,1]; the same checks as above)
 * blocks    host int32[3], each a power of two in [1, 512]
 * Phase 1: d_heads = d_nodes = NULL: builds and returns the sizes
 *          (*n_nodes_out; stats_out->n_heads = bx*by*bz and the depth
 *          statistics), writes nothing else.
 * Phase 2: d_heads device uint32 [bx*by*bz], d_nodes device lr_kdnode
 *          [nodes_cap] (may be NULL when the forest has no nodes, with
 *          nodes_cap 0): builds again, fails with LR_ECAPACITY if nodes_cap is
 *          below the node count, copies heads and nodes on `stream` and
 *          returns once the copies have completed (the host arrays are freed
 *          then).  The device layout is the one lr_lookup and lr_render read. */
lr_status lr_build_forest_device(const float* elem_box, int64_t n_elem, const int32_t blocks[3], uint32_t* d_heads,
                                 lr_kdnode* d_nodes, int64_t nodes_cap, int64_t* n_nodes_out,
                                 lr_forest_stats* stats_out, void* stream);

/* SHA-1 (hex) of the library sources and compile flags this binary was built
 * from ("unknown" if the build did not define it): lets a binding refuse, or
 * rebuild, a binary older than its sources. */
const char* lr_build_id(void);

/* Element ids of n points (device float [n][3], each coordinate in [0,1])
 * by Alg. 1 over a forest uploaded to the device; elem_out device int32 [n]. */
lr_status lr_lookup(const uint32_t* heads, const lr_kdnode* nodes, int64_t n_nodes,
                    const int32_t blocks[3], int64_t n_elem, const float* points, int64_t n,
                    int32_t* elem_out, void* stream);

/* --------------------------------------------------------------------- octree
 * Sec. 3.2 lists an octree as the O(log N) look-up for meshes whose knots are
 * dyadic; Sec. 3.2.2 stores it on the GPU as one buffer whose entries are
 * either a node or, marked by the high bit, an element.  Here a cell met by
 * one element (positive volume) is a leaf; any other cell is split into its
 * eight children.  Device layout:
 *   root   uint32: LR_LEAF | element (a one-element mesh) or node 0
 *   nodes  uint32 [n_nodes][8]: child k (x bit 0, y bit 1, z bit 2 of k; bit
 *          set = upper half) as a node index or LR_LEAF | element
 * Descent for p in [0,1]^3: at level l (root l = 0) the child bit of axis a
 * is min(floor(p_a 2^(l+1)), 2^(l+1) - 1) & 1.
 * elem_box  host double [n_elem][6], every knot a multiple of 2^-24 (else
 *           LR_EKNOT), tiling [0,1]^3 (gaps and overlaps: LR_EPARTITION).
 * stats     optional: n_heads = 1, n_nodes, n_direct = 1 if the root is an
 *           element; depth statistics over the leaves (depth = level). */
typedef struct lr_octree_host lr_octree_host;   /* opaque host-side octree */

lr_status lr_build_octree(const double* elem_box, int64_t n_elem, lr_octree_host** out,
                          lr_forest_stats* stats);

/* Copies a built octree into host buffers (root: one uint32; nodes:
 * uint32 [n_nodes][8]); either pointer may be NULL to skip it. */
lr_status lr_octree_export(const lr_octree_host* o, uint32_t* root, uint32_t* nodes);

void lr_octree_free(lr_octree_host* o);

/* Element ids of n points by the octree descent above (root, nodes on the
 * device); points and elem_out as for lr_lookup. */
lr_status lr_lookup_octree(const uint32_t* root, const uint32_t* nodes, int64_t n_nodes, int64_t n_elem,
                           const float* points, int64_t n, int32_t* elem_out, void* stream);

/* ------------------------------------------------------------- Bezier blocks
 * Sec. 3.2.3: on each element the LR-spline is one polynomial of tri-degree p;
 * it is rewritten in the tensor Bernstein basis of the element (a change of
 * basis, not an approximation), giving (p1+1)(p2+1)(p3+1) coefficients per
 * component for every element.
 *
 * Block layout: row e of the output holds component q's coefficient
 * (jx, jy, jz) at q*nc + jx + (px+1)*(jy + (py+1)*jz), nc = (px+1)(py+1)(pz+1);
 * rows are lr_bezier_stride() elements long (16-byte rows, zero padded). */
int64_t lr_bezier_stride(const int32_t p[3], int32_t ncomp, int32_t dtype);

/* Which B-splines act on which element: CSR over elements of the indices of
 * the B-splines whose support contains the element (ascending), built on the
 * host.  knots host double [n_bspl][3][kstride] (axis d uses p[d]+2 knots),
 * elem_box host double [n_elem][6].  csr_ptr host int64 [n_elem+1] is always
 * filled; csr_idx host int32 [idx_cap] is filled if idx_cap >= the count,
 * which is returned in *nnz (else LR_ECAPACITY; pass csr_idx = NULL, idx_cap = 0
 * to size it).  An element covered by fewer than (p1+1)(p2+1)(p3+1)
 * B-splines is an error (LR_EPARTITION). */
lr_status lr_build_support(const double* knots, int64_t n_bspl, int32_t kstride, const int32_t p[3],
                           const double* elem_box, int64_t n_elem, int64_t* csr_ptr,
                           int32_t* csr_idx, int64_t idx_cap, int64_t* nnz);

typedef struct {
    int32_t p[3];             /* tri-degree, each 1..3 */
    int32_t ncomp;            /* components, 1..4 */
    int32_t kstride;          /* knots per axis slot, >= max(p)+2 */
    int32_t pad;
    int64_t n_bspl;
    int64_t n_elem;
    const double* knots;      /* device [n_bspl][3][kstride] */
    const double* coef;       /* device [n_bspl][ncomp] */
    const double* gamma;      /* device [n_bspl] */
    const double* elem_box;   /* device [n_elem][6] */
    const int64_t* csr_ptr;   /* device [n_elem+1], from lr_build_support */
    const int32_t* csr_idx;   /* device [csr_ptr[n_elem]] */
} lr_lrspline;

/* FP64 change of basis on the GPU: for every element e and B-spline i acting
 * on it, the 1-D Bernstein coefficients of N_i's polynomial piece on e are the
 * blossom of that piece at (lo^(p-j), hi^j) (de Boor's recurrence), and
 *   C_e[q][j] = sum_i gamma_i c_i[q] bx_i[jx] by_i[jy] bz_i[jz]
 * is summed in FP64 in csr order and rounded once (RNE) to out_dtype
 * (LR_F32, LR_F16 or LR_F64).  bezier: device [n_elem][stride].
 * range: optional device double[2]: (min, max) of all coefficients for
 * ncomp == 1, (0, max_j |C_e[.][j]|) otherwise (FP64, before rounding). */
lr_status lr_extract_bezier(const lr_lrspline* spl, int32_t out_dtype, void* bezier, double* range,
                            void* stream);

/* Adjoint of lr_extract_bezier with respect to the LR coefficients c_i of
 * Eq. 2.  The change of basis of Sec. 3.2.3 is linear in c, so for a gradient
 * G_e = dL/dC_e of every Bezier block
 *   dL/dc_i[q] += gamma_i sum_{e in supp N_i} sum_j G_e[q][j] bx_i[jx] by_i[jy] bz_i[jz]
 * with the 1-D Bernstein vectors of the forward (FP64 throughout).
 * grad_bezier: device, the block layout of grad_dtype (LR_F32 or LR_F64; rows
 * of lr_bezier_stride(p, ncomp, grad_dtype)).  grad_coef: device double
 * [n_bspl][ncomp], accumulated (+=) by FP64 atomic adds, so the order of the
 * additions is unspecified (results agree to FP64 rounding); the caller
 * zeroes it.  spl->coef is not read and may be NULL.  Elements whose gradient
 * block is all zero are skipped. */
lr_status lr_extract_bezier_backward(const lr_lrspline* spl, int32_t grad_dtype, const void* grad_bezier,
                                     double* grad_coef, void* stream);

/* ------------------------------------------------------------------- render */
typedef struct {
    int32_t p[3];             /* tri-degree; the render kernels take p1 = p2 = p3 in 1..3 */
    int32_t ncomp;            /* 1 with LR_COLOR_LUT, 3 with LR_COLOR_HUE */
    int64_t n_elem;
    const float* elem_box;    /* device float [n_elem][6] */
    const void* bezier;       /* device [n_elem][stride] of bezier_dtype */
    int32_t bezier_dtype;     /* LR_F32 or LR_F16 (FP32 arithmetic either way) */
    int32_t blocks[3];        /* forest blocks per axis (LR_LOOKUP_FOREST) */
    const uint32_t* heads;    /* device: forest heads, or the octree root */
    const void* nodes;        /* device: lr_kdnode [n_nodes] (forest) or uint32 [n_nodes][8] (octree) */
    int64_t n_nodes;
    const float* lut;         /* device float [256][4] RGBA transfer function */
    float vmin, vmax;         /* value range mapped onto the table */
    float xi;                 /* standard length of Alg. 2 */
    float alpha_clamp;        /* alpha_src <- min(alpha_src, alpha_clamp) */
    float term_alpha;         /* stop a ray once its opacity reaches this */
    int32_t step_mode;        /* LR_STEP_FIXED or LR_STEP_ADAPTIVE */
    int32_t n_fixed_steps;    /* for LR_STEP_FIXED, >= 1 */
    int32_t color_mode;       /* LR_COLOR_LUT or LR_COLOR_HUE */
    int32_t max_samples;      /* per-ray sample cap, >= 1 */
    int32_t lookup;           /* LR_LOOKUP_FOREST or LR_LOOKUP_OCTREE (heads, nodes, n_nodes) */
    int32_t shading;          /* LR_SHADE_NONE, _DIRECTIONAL or _HEADLIGHT (forest look-up only) */
    float light[3];           /* direction towards the light for LR_SHADE_DIRECTIONAL (any length > 0) */
} lr_scene;

/* One camera (values in FP32).  Pixel (i, j), row 0 at the top, writes
 * out[out_offset + j*width + i].  Rays (every operation an FP32 IEEE
 * operation, no fused multiply-add, correctly rounded / and sqrt):
 *   sx = ((2i+1)/width - 1)*tx,   sy = (1 - (2j+1)/height)*ty
 *   LR_PERSP: d' = (fwd + sx*right) + sy*up, d = d'/sqrt((d'x^2 + d'y^2) + d'z^2), o = eye
 *   LR_ORTHO: o = (eye + sx*right) + sy*up, d = fwd
 * clipped to [0,1]^3 by the slab test; sample at t: clamp(o + t*d, 0, 1). */
typedef struct {
    int32_t proj;             /* LR_PERSP or LR_ORTHO */
    int32_t width, height;
    int32_t pad;
    int64_t out_offset;       /* in pixels */
    float eye[3], fwd[3], right[3], up[3];
    float tx, ty;
} lr_view;

/* Forward render (Sec. 4): for every pixel of every view, march the ray
 * (fixed steps, or Eq. 4), find each sample's element through the forest
 * (Alg. 1), evaluate the Bezier block, map through the table and composite
 * front to back (Alg. 2) as T_acc <- T_acc (1 - a), C += T_acc a C_src with
 * a = 1 - (1 - alpha_src)^(ds/xi); write (C_r, C_g, C_b, 1 - T_acc).
 * views     host array of n_views (any number; launched 16 per kernel)
 * rgba      device float [sum of width*height][4] at the views' out_offsets
 * nsamples  optional device uint32 [same pixels]: samples taken per pixel */
lr_status lr_render(const lr_scene* sc, const lr_view* views, int32_t n_views, float* rgba,
                    uint32_t* nsamples, void* stream);

/* lr_render with a dispatch order estimated per launch: the same images, bit
 * for bit, and the same errors, in less time when the work per pixel is
 * uneven.  A block of 16x16 pixels is estimated from the element sizes (Eq. 4
 * steps) at 32 points along its centre ray; groups of 2x2 blocks are dealt to
 * the GPU's eight XCDs longest first (each group whole to one XCD, whose
 * cache its rays share).  lr_render instead deals the blocks from the middle
 * of each view outwards.
 * workspace        device memory, 256-byte aligned, of at least the bytes
 *                  lr_render_workspace_size returns for the same views; the
 *                  caller owns it; it is read and written on stream only, so
 *                  it may be reused once this call's work on stream is done
 * workspace_bytes  its size: LR_ECAPACITY if too small, LR_EINVAL if null or
 *                  misaligned */
lr_status lr_render_scheduled(const lr_scene* sc, const lr_view* views, int32_t n_views, float* rgba,
                              uint32_t* nsamples, void* workspace, int64_t workspace_bytes,
                              void* stream);

/* lr_render_scheduled for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid it): the
 * workspace is a 2 MiB + 64 KiB array the library holds on each GPU it runs
 * on, until the process ends, so no call allocates.  It holds the workspace of a launch
 * of up to 16 views with about 262 144 blocks of 16x16 pixels (16 views of
 * 2048^2 fit exactly); larger requests return LR_ECAPACITY and render
 * nothing.  Calls that overlap on one GPU share the array and race:
 * serialise them (one stream, or events). */
lr_status lr_render_scheduled_noalloc(const lr_scene* sc, const lr_view* views, int32_t n_views,
                                      float* rgba, uint32_t* nsamples, void* stream);

/* Bytes of workspace lr_render_scheduled needs for these views (host only,
 * no GPU work), for the largest launch (16 views per launch): 4 bytes per
 * 16x16-pixel block for the estimates, then, with s slots of the dealing
 * order (per view, 32 for every 8 groups of 2x2 blocks, rounded up), s / 4
 * bytes for the groups' XCDs and 4 s bytes for the order, each part rounded
 * up to 256.  LR_EINVAL for null arguments or invalid views. */
lr_status lr_render_workspace_size(const lr_view* views, int32_t n_views, int64_t* bytes);

/* lr_render through persistent workgroups that take the launch's 8x8-pixel
 * tiles from atomic counters in device memory: the same images, bit for bit,
 * and the same errors.  It is the form of work distribution the hardware's
 * own dispatch replaces in lr_render and lr_render_scheduled (faster on this
 * GPU); it is kept so that the two can be compared.  Forest look-up without
 * shading only (LR_EINVAL otherwise).
 * queues           1: one counter hands out the tiles in dealing order to
 *                  whichever workgroup asks; 8: one counter per XCD, shared
 *                  by the workgroups the hardware deals to that XCD, handing
 *                  out the tiles lr_render renders there
 * cost_order       0: tiles dealt from the middle of each view outwards, as
 *                  lr_render; 1: longest first, as lr_render_scheduled
 * workgroups       single-wave workgroups to start, at most 2^20; 0: as many
 *                  as the GPU holds at once; rounded up to a multiple of 8
 * workspace, workspace_bytes
 *                  as for lr_render_scheduled (lr_render_workspace_size
 *                  bytes, 256-byte aligned, owned by the caller); the
 *                  counters live in its first 256 bytes */
lr_status lr_render_persistent(const lr_scene* sc, const lr_view* views, int32_t n_views, float* rgba,
                               uint32_t* nsamples, int32_t queues, int32_t cost_order, int32_t workgroups,
                               void* workspace, int64_t workspace_bytes, void* stream);

/* Adjoint of lr_render for scalar fields (ncomp 1, LR_COLOR_LUT, F32 blocks,
 * either look-up structure, no shading).
 * Re-marches each ray with the forward's schedule (no per-sample storage) and
 * uses the forward image to form the suffix sums.  Accumulates (+=) into
 * grad_bezier (device float, the bezier layout) and grad_lut (device float
 * [256][4]); the caller zeroes them.  rgba_fwd: the forward output for the
 * same scene and views; grad_rgba: dL/d(rgba), same layout. */
lr_status lr_render_backward(const lr_scene* sc, const lr_view* views, int32_t n_views,
                             const float* rgba_fwd, const float* grad_rgba, float* grad_bezier,
                             float* grad_lut, void* stream);

/* Sample schedule of single rays, for verification: for pixel k
 * (pix device int32 [n][2] = (i, j) of views[0]) writes up to max_out samples
 * (t, element id, composited segment length) at t_out/elem_out/ds_out
 * [k*max_out + s] (device) and the number of samples taken in count [k]. */
lr_status lr_trace_rays(const lr_scene* sc, const lr_view* view, const int32_t* pix, int64_t n,
                        int32_t max_out, float* t_out, int32_t* elem_out, float* ds_out,
                        int32_t* count, void* stream);

/* --------------------------------------------------------------- streamlines
 * Sec. 5: a streamline from seed x0 solves dx/dt = f(x), x(0) = x0 (Eq. 5),
 * here by an explicit Runge-Kutta method (Eq. 6) with published tableaus:
 * k_i = f(x_n + h sum_{j<i} a_ij k_j), x_{n+1} = x_n + h sum_i b_i k_i. */
#define LR_RK1 0      /* explicit Euler */
#define LR_RK2 1      /* midpoint */
#define LR_RK3 2      /* Kutta's third order */
#define LR_RK4 3      /* classic fourth order */
#define LR_RK4_38 4   /* 3/8 rule */
#define LR_RKF5 5     /* Fehlberg's pair, fifth-order weights */
#define LR_HE 6       /* Heun-Euler 2(1) */
#define LR_BS 7       /* Bogacki-Shampine 3(2) */
#define LR_RKF45 8    /* Fehlberg 4(5), fifth order propagated */

/* Step sizes.  HEURISTIC (Sec. 5.2): h = base * 2^-d * min side of the element
 * holding x_n, the Eq. 4 distance used as the time step (the element is found
 * at x_n rounded to FP32).  CONSTANT: h = base.  EMBEDDED (LR_HE, LR_BS,
 * LR_RKF45): the higher-order solution is kept; err = |x_high - x_low|_2; a
 * step is accepted if err <= tol, or h <= 1e-14, or after 64 rejections; a
 * rejected step retries with h * max(0.2, 0.9 (tol/err)^(1/q)) (at least
 * 1e-14); the next step is h * min(5, max(0.2, 0.9 (tol/err)^(1/q))), q the
 * propagated order (5 if err = 0); the first h is the heuristic step at the seed. */
#define LR_STREAM_HEURISTIC 0
#define LR_STREAM_CONSTANT 1
#define LR_STREAM_EMBEDDED 2

/* Sec. 5.6: MIXED keeps x, t, h and the stage sums in FP64 and evaluates the
 * field in FP32; SINGLE does everything in FP32. */
#define LR_PREC_MIXED 0
#define LR_PREC_SINGLE 1

typedef struct {
    int32_t method;        /* LR_RK1 .. LR_RKF45 */
    int32_t step_mode;     /* LR_STREAM_* */
    int32_t precision;     /* LR_PREC_MIXED or LR_PREC_SINGLE */
    int32_t max_samples;   /* points stored per line, the seed included, >= 1 */
    double base;           /* step factor (see the step sizes), > 0 */
    double t_end;          /* time limit, > 0: the last step is shortened to land on it */
    double tol;            /* local error tolerance of LR_STREAM_EMBEDDED, > 0 */
} lr_stream_params;

/* The compute stage of Sec. 5.3 for n seeds (device double [n][3]).
 * The field is the scene's 3-component volume (FP32 blocks, either look-up
 * structure; the table and shading fields are not used).  Stage positions are
 * clamped to [0,1]^3 before evaluation.  A line ends when t reaches t_end,
 * when a step would leave [0,1]^3 (that step is not taken) or after
 * max_samples points.
 * points  device float [n][max_samples][4]: (x, y, z, 1) for the points of the
 *         line, (0, 0, 0, 0) after its end
 * times   optional device double [n][max_samples]: t of each point (0 after the end)
 * count   optional device int32 [n]: points stored */
lr_status lr_streamlines(const lr_scene* sc, const lr_stream_params* prm, const double* seeds, int64_t n,
                         float* points, double* times, int32_t* count, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LRVR_H */
