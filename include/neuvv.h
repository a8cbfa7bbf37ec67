/*
 * neuvv.h - C ABI of libneuvv.so, a VOctree renderer for MI355X (gfx950).
 *
 * Implements the rendering hot path of NeuVV (arXiv 2202.06088): a Video
 * Octree (VOctree) whose leaves hold hyperspherical-harmonic (HH) colour
 * coefficients and density weights on a shared temporal basis, rendered per
 * ray by octree traversal and front-to-back compositing (Sec. 4.3), its
 * adjoint (Sec. 4.3 "Optimization"), instance placement and re-timing
 * (Sec. 5.1, Eq. 13) and depth-aware blending of rendered layers (Alg. 1).
 *
 * Conventions shared by every call
 *   - Pointers named "device" are HIP device pointers owned by the caller;
 *     pointers named "host" are host memory owned by the caller. The library
 *     keeps no pointer after a call returns. The only device memory it
 *     allocates is per-call scratch of the render calls: neuvv_render,
 *     neuvv_render_trace, neuvv_render_multi, neuvv_render_backward,
 *     neuvv_render_backward_trace and neuvv_find_terminal_leaves take 2 KiB
 *     of work-queue counters plus a candidate list of 4 bytes per work slot
 *     (rounded up to 64 slots; the adjoint of a traced forward takes two);
 *     the adjoints also take the records of their two-phase reduction (4
 *     bytes per leaf plus 32 bytes per record of room, see there), and
 *     neuvv_render_multi the segment lists of its instances (see there). Scratch
 *     is taken in stream order on the call's stream from a memory pool the
 *     library keeps per device (it keeps freed memory for later calls) and
 *     freed in stream order after the kernels; each call has its own, so
 *     calls on different streams do not interfere.
 *   - "stream" is a hipStream_t (NULL = the null stream). GPU work is queued
 *     on it asynchronously; the caller synchronises. Argument errors are
 *     detected on the host before anything is queued.
 *   - Every call returns NEUVV_OK (0) or a negative neuvv_status; then
 *     neuvv_last_error() gives a message (thread-local, valid until the next
 *     call on the same thread). No C++ exception crosses this boundary.
 *   - Floating-point outputs are float32; integer outputs int32/int64.
 *   - Gradient outputs accumulate (+=) into caller-zeroed float32 buffers, so
 *     several instances of one tree (Sec. 5.1, "varied manifestations") sum
 *     their gradients into the same leaves.
 */
#ifndef NEUVV_H
#define NEUVV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NEUVV_OK = 0,
    NEUVV_ERR_ARG = -1,         /* null pointer, negative size, bad enum */
    NEUVV_ERR_RANGE = -2,       /* a value outside its documented range */
    NEUVV_ERR_DUPLICATE = -3,   /* the same leaf cell listed twice */
    NEUVV_ERR_CAPACITY = -4,    /* an output buffer smaller than required */
    NEUVV_ERR_UNSUPPORTED = -5, /* K, C, Cg or dtype without a compiled kernel */
    NEUVV_ERR_HIP = -6          /* a HIP launch or runtime error */
} neuvv_status;

/* Arrangement of the leaf payload arrays (see "Leaf payload layout"). */
typedef enum { NEUVV_LAYOUT_VEC_SOA = 0, NEUVV_LAYOUT_LEAF_ROWS = 1 } neuvv_layout;

/* Storage type of the leaf coefficients. Evaluation and compositing are
   always float32; 16-bit storage is converted with round-to-nearest-even. */
typedef enum { NEUVV_F32 = 0, NEUVV_F16 = 1, NEUVV_BF16 = 2 } neuvv_dtype;

/* Density activation of Eq. 5 (Sec. 4.2): sigma = act(sum_c wsig_c b_c).
   SOFTPLUS (log(1 + e^x), derivative sigmoid(x)) is the default; RELU is
   max(x, 0) as Eq. 5 prints it, with derivative 1 for x > 0 and 0 otherwise
   (a leaf whose logit is <= 0 is transparent and takes no gradient). */
typedef enum { NEUVV_DENSITY_SOFTPLUS = 0, NEUVV_DENSITY_RELU = 1 } neuvv_density;

/*
 * Leaf payload layout. A leaf has R_hh = 3K colour coefficients, value
 * r = ch*K + k for colour channel ch and HH function k (Eq. 4), R_sig = C
 * density weights (Eq. 5) and, in the per-point hyperangle form, R_gam = Cg
 * hyperangle weights (Eq. 6). Each array is stored in 16-byte vectors of
 * V = 16 / sizeof(element) values (4 for float32, 8 for 16-bit), padding
 * values (r >= R) zero, leaves in slot (Morton) order, in one of two layouts:
 *   NEUVV_LAYOUT_LEAF_ROWS: a[n_leaves][ceil(R / V)][V]: value r of slot s at
 *     element s * ceil(R / V) * V + r; one leaf's values are contiguous (the
 *     renderer gathers one whole leaf per lane and sample).
 *   NEUVV_LAYOUT_VEC_SOA: a[ceil(R / V)][n_leaves][V]: value r of slot s at
 *     element (r / V) * n_leaves * V + s * V + r % V.
 * neuvv_payload_words() gives the sizes (the wgam array has the size of a
 * wsig array with C = Cg); neuvv_pack_leaves() and neuvv_pack_rows() fill
 * them.
 *
 * Leaf gradient layout ("rows"). Gradients are float32 and leaf-major:
 *     grad_leaf[n_leaves][ROW],  ROW = neuvv_grad_row_elems(K, C, Cg) = 3K + C + Cg rounded up to 64,
 * row s holding d/d hh of slot s at r = ch*K + k (r < 3K), d/d wsig at 3K + c,
 * d/d wgam at 3K + C + c, and zeros after 3K + C + Cg. The adjoint adds one
 * sample's row with wavefront-wide atomic instructions (one per 64 values),
 * each of which the L2 serves as a couple of line operations.
 */

/* A built tree on the device. All pointers are device pointers. */
typedef struct {
    int32_t depth;        /* D in [1, 12]: leaf grid [0, 2^D)^3 in tree-local units */
    int32_t K;            /* HH functions per colour channel (compiled: 16, or 14 with Cg = 31) */
    int32_t C;            /* density basis size (compiled: 8, or 31 with Cg = 31) */
    int32_t dtype;        /* neuvv_dtype of hh and wsig */
    int64_t n_nodes;      /* rows of nodes */
    int64_t n_leaves;     /* leaf slots */
    const int32_t* nodes; /* [n_nodes][4] from neuvv_build_voctree, 16-byte aligned */
    const void* hh;       /* colour coefficients, layout above */
    const void* wsig;     /* density weights, layout above */
    int32_t T;            /* frames of the temporal tables */
    int32_t box[6];       /* occupied-cell bounds from neuvv_build_voctree (lo x,y,z; hi x,y,z
                             exclusive): rays are clipped to this box instead of the whole grid.
                             All zero = the whole grid [0, 2^D)^3. */
    int32_t layout;       /* neuvv_layout of hh and wsig */
    const float* basis;   /* [T][C] density basis, row t = frame t (Eq. 5: A transposed) */
    const float* gamma;   /* [T] hyperangle per frame, in [0, pi] (Eq. 4's gamma(t)); used when
                             Cg = 0, may be NULL otherwise */
    int32_t Cg;           /* 0: one hyperangle per frame (gamma). 31 (with K = 14, C = 31): the
                             per-point hyperangle of Eq. 6, gamma = pi sigmoid(sum_c wgam_c Bg_c(t)),
                             the paper's 104-value leaf */
    const void* wgam;     /* hyperangle weights, storage dtype and layout of wsig (Cg > 0) */
    const float* basis_g; /* [T][Cg] hyperangle basis (Cg > 0) */
    const float* edit;    /* NULL, or appearance edits (Sec. 5.2): [n_leaves][8] float32 rows in slot
                             order, 16-byte aligned: target r, g, b; target density (< 0: keep the
                             leaf's own); first frame t_d (the edit is active at local times
                             tau >= t_d, +inf: never); a word used by neuvv_paint; 2 unused. K = 16,
                             C = 8 form only; neuvv_render_backward rejects trees with edits */
    int32_t density;      /* neuvv_density: the activation of Eq. 5 (0 = softplus) */
    const int32_t* dir;   /* the brick directory of nodes, from neuvv_build_directory (required) */
} neuvv_tree;

/* Placement and re-timing of one tree instance (Eq. 13). A world point x is
   the tree-local point R^T (x - trans) / scale (R = rot, row-major 3x3,
   orthonormal); a world time t is the tree-local time tau = t + time_offset,
   wrapped into [0, T) when time_wrap != 0 (looping) and clamped into
   [0, T-1] otherwise. NULL instance = identity rotation, zero translation,
   scale 1, no offset, clamping. */
typedef struct {
    float rot[9];
    float trans[3];
    float scale;
    float time_offset;
    int32_t time_wrap;
} neuvv_instance;

/* Pinhole camera, OpenCV axes (x right, y down, z forward), pixel (u, v)
   centred at (u + 0.5, v + 0.5); c2w is the row-major 3x4 camera-to-world
   matrix [R | centre]. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float c2w[12];
} neuvv_camera;

/*
 * neuvv_build_voctree - host-side construction of the sparse octree over
 * the occupied leaf cells (Sec. 4.3 "Initialization" leaves the voxels with
 * non-negligible density; this call receives them as a list of cells).
 *
 * depth           D in [1, 12].
 * n_leaves        number of cells, >= 0.
 * leaf_ijk        host [n_leaves][3] int32, each in [0, 2^D); no duplicates.
 * nodes           host [node_capacity][4] int32 output, or NULL to only count.
 *                 The octree is stored two levels per node. There are
 *                 L = ceil(D/2) node levels; a node of level w is a cube of
 *                 edge 2^e_w split into child cells of edge 2^(e_w - b_w),
 *                 with b_0 = 1 for odd D (else 2), b_w = 2 for w > 0,
 *                 e_0 = D and e_(w+1) = e_w - b_w; the children of the last
 *                 level are the leaves. Child cell (x, y, z) (coordinates
 *                 local to the node, in [0, 2^b_w)) is bit q = x0 | y0<<1 |
 *                 z0<<2 | x1<<3 | y1<<4 | z1<<5 (xk = bit k of x).
 *                 Row r: words 0 and 1 = low and high half of the 64-bit
 *                 occupancy mask (bit q set: child cell q holds a leaf);
 *                 word 2 = index of the first occupied child, a node row
 *                 (levels w < L-1) or a leaf slot (last level); occupied
 *                 children follow consecutively in bit order, so child q is
 *                 word2 + popcount(mask & (2^q - 1)); word 3 = 0. Row 0 is
 *                 the root; rows are stored level by level from the root,
 *                 Morton order within a level.
 * node_capacity   rows available in nodes (ignored when nodes is NULL).
 * n_nodes_out     host output, the number of nodes (always written on OK).
 * slot_of_input   host [n_leaves] int64 output or NULL: the leaf slot
 *                 (rank in Morton order) of input cell i.
 * box_out         host [6] int32 output or NULL: bounds of the occupied cells,
 *                 lo (inclusive) x, y, z then hi (exclusive) x, y, z; all zero
 *                 when there are no leaves. Goes into neuvv_tree.box.
 * Errors: ARG (null leaf_ijk with n_leaves > 0, null n_nodes_out), RANGE
 * (depth, coordinates), DUPLICATE, CAPACITY (node_capacity < n_nodes).
 */
int neuvv_build_voctree(int32_t depth, int64_t n_leaves, const int32_t* leaf_ijk, int32_t* nodes,
                        int64_t node_capacity, int64_t* n_nodes_out, int64_t* slot_of_input, int32_t* box_out);

/*
 * neuvv_directory_entries - entries of the brick directory of a depth-D
 * tree: E^3 with E = 2^(D-2) (E = 1 for D <= 2), 4 bytes each (8 MiB at
 * D = 9, 64 MiB at D = 10, 4 GiB at D = 12). -1 for D outside [1, 12].
 */
int64_t neuvv_directory_entries(int32_t depth);

/*
 * neuvv_build_directory - fills the brick directory that the octree walk of
 * every render call reads (Sec. 4.3 "Rendering": it serves the same walk as
 * the node table, so that leaving a 4^3 region of leaf cells costs at most
 * two dependent reads instead of one per node level). Entry (k E + j) E + i
 * describes the region of cells [4i, 4i+4) x [4j, 4j+4) x [4k, 4k+4):
 *   >= 0       the row of nodes of the region's last-level node (the region
 *              holds a leaf; for D <= 2, row 0, the root);
 *   -(1 + s)   the region holds no leaf; 2^s (2 <= s < D) is the edge of the
 *              largest aligned cube around it that holds none, at the node
 *              levels of neuvv_build_voctree (a child cell, or a 2^3 group of
 *              child cells of a 2-bit node).
 * Build it once per node table, after uploading the nodes; the renders then
 * take it in neuvv_tree.dir. Queued on stream; nodes must be the table of
 * neuvv_build_voctree for this depth (its child indices are followed as they
 * are).
 * depth      D in [1, 12].
 * n_nodes    rows of nodes.
 * nodes      device [n_nodes][4] int32, 16-byte aligned.
 * dir        device int32 [capacity] output, 4-byte aligned.
 * capacity   entries available, >= neuvv_directory_entries(depth).
 * Errors: RANGE (depth, n_nodes), ARG (NULL or misaligned buffer), CAPACITY,
 * HIP (launch).
 */
int neuvv_build_directory(int32_t depth, int64_t n_nodes, const int32_t* nodes, int32_t* dir, int64_t capacity,
                          void* stream);

/*
 * neuvv_payload_words - element counts of the payload arrays for n_leaves
 * leaves: *hh_elems = ceil(3K/V)*n_leaves*V, *wsig_elems = ceil(C/V)*n_leaves*V
 * for the storage dtype (V = 4 for float32, 8 for 16-bit). Host only.
 */
int neuvv_payload_words(int32_t K, int32_t C, int32_t dtype, int64_t n_leaves, int64_t* hh_elems,
                        int64_t* wsig_elems);

/*
 * neuvv_grad_row_elems - floats per leaf gradient row for K, C and Cg
 * (3K + C + Cg rounded up to 64), or NEUVV_ERR_RANGE. Host only.
 */
int neuvv_grad_row_elems(int32_t K, int32_t C, int32_t Cg);

/*
 * neuvv_pack_leaves - convert leaf coefficients given per input leaf into
 * the payload layout above, in Morton slot order and in the storage dtype
 * (round to nearest even for 16-bit).
 * hh_in           device [n_leaves][3][K] float32, input leaf order.
 * wsig_in         device [n_leaves][C] float32, input leaf order.
 * slot_of_input   device [n_leaves] int64 from neuvv_build_voctree, or NULL
 *                 when the inputs are already in slot order.
 * hh_out, wsig_out device outputs of neuvv_payload_words() elements; the
 *                 padding elements are written with zero.
 * layout          neuvv_layout of the outputs.
 * Errors: ARG, UNSUPPORTED (dtype, layout).
 */
int neuvv_pack_leaves(int32_t K, int32_t C, int32_t dtype, int32_t layout, int64_t n_leaves, const float* hh_in,
                      const float* wsig_in, const int64_t* slot_of_input, void* hh_out, void* wsig_out,
                      void* stream);

/*
 * neuvv_pack_rows - convert one per-leaf array of R float32 values (e.g. the
 * Cg hyperangle weights of Eq. 6) into the payload layout above, in slot
 * order and the storage dtype (round to nearest even for 16-bit).
 * R               values per leaf, [1, 256].
 * in              device [n_leaves][R] float32, input leaf order.
 * slot_of_input   device [n_leaves] int64, or NULL (inputs in slot order).
 * out             device output of ceil(R/V) * n_leaves * V elements.
 * Errors: ARG, RANGE (R), UNSUPPORTED (dtype, layout), HIP.
 */
int neuvv_pack_rows(int32_t R, int32_t dtype, int32_t layout, int64_t n_leaves, const float* in,
                    const int64_t* slot_of_input, void* out, void* stream);

/*
 * neuvv_render - volume rendering of a VOctree along n rays (Sec. 4.3
 * "Rendering", Eq. 4, 5, 8, 9).
 *
 * For ray r with world origin o, direction d (need not be unit) and time t:
 * the tree-local ray is x_l(u) = R^T (o + u d - trans) / scale, u >= 0; the
 * leaves it crosses are found in the octree (its last-level nodes through the
 * tree's brick directory), empty space being skipped one empty octree node
 * at a time; delta is the length of the ray inside a
 * leaf in leaf units (cells are half-open [i, i+1); zero-length crossings are
 * not samples). Per ray: h = the first K real HH at the unit local view
 * direction and gamma(tau), b = the density basis at tau, both linearly
 * interpolated between frames floor(tau) and floor(tau)+1 (the last frame
 * is held on [T-1, T)). Per sample in front-to-back order:
 *     sigma = softplus(sum_c wsig_c b_c),  c_ch = sigmoid(sum_k hh_ch,k h_k),
 *     a = 1 - exp(-sigma delta), w = T a, rgb += w c, T *= exp(-sigma delta),
 * stopping after the first sample that leaves T < t_stop (t_stop = 0 never
 * stops early). The K = 16 HH functions are n <= 2 (14) then (3,0,0), (3,1,-1)
 * in the order n, l, m. With the per-point hyperangle (Cg > 0) gamma is
 * evaluated per sample, gamma = pi sigmoid(sum_c wgam_c bg_c) with bg the
 * hyperangle basis at tau, and h = the first K = 14 HH at (direction, gamma).
 *
 * tree            device tree (pointer to a host struct).
 * inst            host struct or NULL (identity).
 * n_rays          >= 0.
 * ray_o, ray_d    device [n][3] world origins and directions.
 * ray_t           device [n] world times, or NULL to use t_scalar for all.
 * image_width     0, or W > 0 when rays are a row-major image W pixels wide:
 *                 each wavefront then takes 8x8 pixel tiles (coherence hint,
 *                 results are identical).
 * t_stop          early-termination threshold on transmittance, >= 0.
 * rgb             device [n][3] premultiplied colour (Eq. 8).
 * alpha           device [n] 1 - T_final = sum of weights (Eq. 9).
 * depth           device [n] or NULL: sum(w * s_mid) / sum(w), s_mid the world
 *                 distance |d| u of the segment midpoint; +inf if sum(w) = 0.
 * nsamp           device [n] int32 samples composited (needed by backward).
 * Errors: ARG, RANGE, UNSUPPORTED, HIP.
 */
int neuvv_render(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                 const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width, float t_stop,
                 float* rgb, float* alpha, float* depth, int32_t* nsamp, void* stream);

/*
 * neuvv_render_noalloc - neuvv_render for callers that cannot allocate device
 * memory: code under stream or graph capture, serving loops and harnesses
 * that forbid allocation. Same arguments, kernels and results (bit for bit)
 * as neuvv_render, which takes its scratch (work-queue counters and the
 * candidate list of the cull pass) from a stream-ordered pool; this call
 * takes it instead from one fixed device array that the library holds on
 * every device it runs on until the process ends (64 MiB + 2 KiB), and
 * calls no allocating routine. The array fits launches of at most 2^24 work
 * slots: n_rays, or with image_width = W > 0, ceil(W/8) * ceil(rows/8) * 64
 * for rows = ceil(n_rays/W) (the 8-camera 1920x1080 ring stacked as one
 * image is 16,588,800). Larger launches return NEUVV_ERR_CAPACITY before
 * anything is queued. Every call on a device shares that device's array
 * (the counters are cleared by a kernel at the start of each call): calls
 * that may overlap on one device, on different streams or from different
 * threads, race and give wrong results; serialise them.
 * Errors: those of neuvv_render, and CAPACITY.
 */
int neuvv_render_noalloc(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                         const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width, float t_stop,
                         float* rgb, float* alpha, float* depth, int32_t* nsamp, void* stream);

/*
 * neuvv_render_backward - adjoint of neuvv_render (Sec. 4.3 "Optimization")
 * for L = sum_r <grad_rgb_r, rgb_r> + grad_alpha_r alpha_r. Each ray replays
 * its nsamp samples front to back with the transmittance recomputed (nothing
 * per sample is stored by the forward pass):
 *     dL/dsigma_k = delta_k (T_{k+1} <g, c_k> - <g, rgb - rgb_{<=k}>) + g_a delta_k T_final
 *     dL/dz_k,ch  = g_ch w_k c_k,ch (1 - c_k,ch)
 * and adds them (atomically) into the leaf gradients and the basis rows.
 * Two-phase adjoint: each sample's dL/dz and dL/dsigma (and dL/dy, Cg > 0)
 * are written once as a 32-byte record linked into its leaf's list; a second
 * kernel sums every list and adds each touched leaf's row once. The room for
 * records is 2 per ray, or the trace's room (trace_cap) in
 * neuvv_render_backward_trace when that is more, at least 2^20, at most
 * 2^31 - 1 (the environment
 * variable NEUVV_BWD_RECORDS, read at every call, sets it; 0 turns records
 * off); samples beyond it are added per sample in the same call. Records
 * are used with image_width or not, for n_rays and n_leaves below 2^31, and
 * with Cg > 0 only when ray_t is NULL (one time for all rays). Summation
 * order follows the atomics, so results may differ between runs in the last
 * bits, as with any atomic accumulation.
 * Arguments as neuvv_render, plus
 * rgb, alpha, nsamp  device forward outputs for the same rays and inputs.
 * grad_rgb        device [n][3]; grad_alpha device [n] or NULL (zero).
 * grad_leaf       device float32 [n_leaves][ROW] leaf gradient rows (layout
 *                 above), accumulated (+=).
 * grad_basis      device [T][C] float32 accumulated, or NULL to skip.
 * grad_basis_g    device [T][Cg] float32 accumulated, or NULL to skip
 *                 (ignored when Cg = 0). With Cg > 0 the chain rule also runs
 *                 through gamma: dL/dgamma_k = sum_ch dL/dz_k,ch sum_j hh_ch,j
 *                 dh_j/dgamma, dL/dy_k = pi sigmoid'(y_k) dL/dgamma_k.
 * The gradient with respect to the gamma table (Cg = 0) is not computed.
 * Errors: ARG, RANGE, UNSUPPORTED, HIP.
 */
int neuvv_render_backward(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays,
                          const float* ray_o, const float* ray_d, const float* ray_t, float t_scalar,
                          int32_t image_width, float t_stop, const float* rgb, const float* alpha,
                          const int32_t* nsamp, const float* grad_rgb, const float* grad_alpha,
                          float* grad_leaf, float* grad_basis, float* grad_basis_g, void* stream);

/*
 * Traced training step (both compiled forms). neuvv_render_trace renders as
 * neuvv_render and also records every composited sample of the call in a
 * caller-owned trace buffer, linked in ray order: the leaf, the segment
 * length delta, the density logit x and the colours c (Eq. 4, 5, 8), and for
 * the per-point form (Cg > 0) the hyperangle logit y and dz/dgamma of the
 * three colour logits (Eq. 6). neuvv_render_backward_trace is
 * neuvv_render_backward for the same tree, rays, times, instance and t_stop,
 * replaying each ray's samples from the trace instead of walking the tree and
 * evaluating the leaves again; the gradients are the same up to rounding. A
 * ray whose samples do not all fit is marked untraced and its adjoint walks
 * as in neuvv_render_backward, so any trace_cap >= 0 is correct (room near
 * the call's total of nsamp avoids walking).
 * trace           device buffer of neuvv_trace_bytes(n_rays, trace_cap) bytes,
 *                 256-byte aligned, owned by the caller; written by
 *                 neuvv_render_trace, read by neuvv_render_backward_trace, and
 *                 valid until the next neuvv_render_trace into it. Its content
 *                 is private to the library.
 * trace_cap       room in 32-byte entries, in [0, 2^31); the same value in both
 *                 calls. A sample takes one entry in the K = 16, C = 8 form and
 *                 two in the per-point form.
 * n_rays          below 2^31 for the traced calls.
 * grad_basis_g    as in neuvv_render_backward (per-point form only).
 * Errors: those of neuvv_render / neuvv_render_backward.
 */
int64_t neuvv_trace_bytes(int64_t n_rays, int64_t trace_cap);   /* -1 for negative arguments */
int neuvv_render_trace(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                       const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width, float t_stop,
                       float* rgb, float* alpha, float* depth, int32_t* nsamp, void* trace, int64_t trace_cap,
                       void* stream);
int neuvv_render_backward_trace(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays,
                                const float* ray_o, const float* ray_d, const float* ray_t, float t_scalar,
                                int32_t image_width, float t_stop, const float* rgb, const float* alpha,
                                const int32_t* nsamp, const float* grad_rgb, const float* grad_alpha,
                                float* grad_leaf, float* grad_basis, float* grad_basis_g, const void* trace,
                                int64_t trace_cap, void* stream);

/*
 * neuvv_compose - depth-aware alpha blending of L rendered layers (Alg. 1),
 * per pixel: sort the layers by depth (equal depth: the later layer is in
 * front), then premultiplied "over":
 *     out_rgb = sum_k prod_{j<k} (1 - A_j) P_k,  out_alpha = 1 - prod_k (1 - A_k),
 *     out_depth = depth of the front layer.
 * L in [1, 16]; rgb device [L][n][3] premultiplied; alpha, depth device
 * [L][n]; outputs device [n][3], [n], [n] (out_depth may be NULL).
 * Errors: ARG, RANGE, HIP.
 */
int neuvv_compose(int32_t L, int64_t n_pix, const float* rgb, const float* alpha, const float* depth,
                  float* out_rgb, float* out_alpha, float* out_depth, void* stream);

/*
 * neuvv_compose_backward - gradient of <g_rgb, out_rgb> + <g_alpha, out_alpha>
 * with respect to every layer's rgb and alpha (depth is a sort key and has
 * none). grad_rgb device [L][n][3], grad_alpha device [L][n] are overwritten
 * (not accumulated). grad_out_alpha may be NULL (zero).
 * Errors: ARG, RANGE, HIP.
 */
int neuvv_compose_backward(int32_t L, int64_t n_pix, const float* rgb, const float* alpha,
                           const float* depth, const float* grad_out_rgb, const float* grad_out_alpha,
                           float* grad_rgb, float* grad_alpha, void* stream);

/*
 * neuvv_pinhole_rays - world rays of a pinhole camera: origin = camera
 * centre, direction = normalize(R (x_c, y_c, 1)) with x_c = (u + 0.5 - cx)/fx,
 * y_c = (v + 0.5 - cy)/fy, computed in compensated float32 arithmetic and
 * rounded once (agrees with the correctly rounded result except within
 * about 2^-40 relative of a rounding boundary).
 * cam             host struct. n >= 0.
 * pix             device [n] int32 linear pixel indices v*W + u, or NULL for
 *                 all W*H pixels in row-major order (then n must be W*H).
 * ray_o, ray_d    device [n][3] outputs.
 * Errors: ARG, RANGE, HIP.
 */
int neuvv_pinhole_rays(const neuvv_camera* cam, int64_t n, const int32_t* pix, float* ray_o, float* ray_d,
                       void* stream);

/*
 * neuvv_eval_hh - the first K real HH (K in {1..30}) at unit directions
 * dirs device [n][3] and hyperangles gam device [n] into out device [n][K]
 * (the per-ray basis of Eq. 4; exposed for testing).
 * Errors: ARG, RANGE, HIP.
 */
int neuvv_eval_hh(int32_t K, int64_t n, const float* dirs, const float* gam, float* out, void* stream);

/* Thread-local message for the last non-OK return on this thread. */
const char* neuvv_last_error(void);

/*
 * neuvv_render_multi - exact rendering of n_inst (1..4) placed instances that
 * may interpenetrate or duplicate one another (Sec. 5.1; Alg. 1 blends
 * separately rendered layers, which is exact only when they are disjoint in
 * depth along each ray). Every instance k maps the world ray to its local ray
 * with the same parameter u (neuvv_instance), and its leaves give intervals
 * of u with constant density sigma (per leaf unit) and colour c. The ray is
 * cut at every boundary of every instance; on each piece [u, u + du) the
 * instances covering it contribute extinction kappa_k = sigma |d| / scale_k
 * per unit u, the piece's optical depth is sum_k kappa_k du and its colour the
 * kappa-weighted mean of theirs, and the pieces are composited front to back
 * as in neuvv_render (Eq. 8; same early stop; nsamp counts pieces; depth is
 * the weighted mean world distance of the piece midpoints). With one
 * instance the result is neuvv_render's.
 * Scratch: besides the work-queue counters and candidate lists, 4 KiB, 4
 * bytes per ray and instance, 4 bytes per work slot, and room for 2 list
 * entries of 32 bytes per ray and instance (each instance's segments along a
 * ray, written by a walk of that instance, then merged). Rays whose lists do
 * not fit that room are rendered by a kernel that walks every instance of the
 * ray together; the result is the same either way.
 * trees           host array of n_inst tree pointers (the same tree may appear
 *                 several times); K = 16, C = 8, no per-point hyperangle, no
 *                 edits, one storage dtype.
 * insts           host array of n_inst instances, or NULL (all identity).
 * Other arguments as neuvv_render.
 * Errors: ARG, RANGE, UNSUPPORTED, HIP.
 */
int neuvv_render_multi(int32_t n_inst, const neuvv_tree* const* trees, const neuvv_instance* insts, int64_t n_rays,
                       const float* ray_o, const float* ray_d, const float* ray_t, float t_scalar,
                       int32_t image_width, float t_stop, float* rgb, float* alpha, float* depth, int32_t* nsamp,
                       void* stream);

/*
 * neuvv_find_terminal_leaves - for appearance editing by painting from a view
 * (Sec. 5.2 "Appearance editing"): traces each ray as neuvv_render does and
 * returns the leaf slot of the first sample after which the accumulated alpha
 * 1 - T exceeds alpha_threshold (0.99 in the paper), or -1 when it never
 * does. Equivalent to neuvv_render with t_stop = 1 - alpha_threshold,
 * reporting the leaf of the sample that stopped the ray.
 * alpha_threshold in (0, 1); last_leaf device [n] int32. Other arguments as
 * neuvv_render. K = 16, C = 8 form only.
 * Errors: ARG, RANGE, UNSUPPORTED, HIP.
 */
int neuvv_find_terminal_leaves(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                               const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width,
                               float alpha_threshold, int32_t* last_leaf, void* stream);

/*
 * neuvv_paint - writes appearance edits: every ray r with last_leaf[r] >= 0
 * (from neuvv_find_terminal_leaves) claims that leaf; the lowest ray index
 * wins, and the leaf's edit row becomes (colours[r], sigma_d, t_d). Rows of
 * leaves no ray ends in are left as they are (initialise the table with
 * t_d = +inf). last_leaf device [n_rays] int32 (entries outside
 * [0, n_leaves) are ignored); colours device [n_rays][3]; edit device
 * [n_leaves][8] (layout in neuvv_tree).
 * Errors: ARG, RANGE, HIP.
 */
int neuvv_paint(int64_t n_rays, const int32_t* last_leaf, const float* colours, float sigma_d, float t_d,
                int64_t n_leaves, float* edit, void* stream);

/* Point light for the shading call (Sec. 5.2 "Spotlight Lighting"). */
typedef struct {
    neuvv_camera camera;     /* the light's pinhole camera; its centre (c2w column 3) is the point light,
                                its image is the shadow map's */
    float ground_z;          /* the ground: world plane z = ground_z */
    float ground_rgb[3];     /* lit ground colour */
    float background_rgb[3]; /* colour of rays that miss the ground */
    float shadow_strength;   /* k in [0, 1]: shadowed ground is scaled by 1 - k A */
    float falloff_r0;        /* > 0: performer colour scaled by (r0 / max(r, r0))^2; 0: no falloff */
} neuvv_light;

/*
 * neuvv_blur - the Gaussian low-pass of a rendered shadow map (Sec. 5.2: a
 * low-resolution map is filtered to remove moire): taps proportional to
 * exp(-i^2 / (2 sigma^2)) for |i| <= round(3 sigma), normalised to sum 1,
 * applied along rows and columns, borders clamped to the edge.
 * height, width   map size (row-major [height][width] float32, device).
 * in, out         device maps; distinct buffers.
 * sigma           in (0, 16] pixels.
 * Errors: ARG, RANGE, HIP.
 */
int neuvv_blur(int32_t height, int32_t width, const float* in, float sigma, float* out, void* stream);

/*
 * neuvv_shade - spotlight shadow on the ground and distance falloff
 * (Sec. 5.2 "Spotlight Lighting") for a rendered performer layer. Per viewer
 * ray (o, d) with the layer's premultiplied rgb, alpha and depth (outputs of
 * neuvv_render or neuvv_compose for the same rays):
 *   - falloff: F = (r0 / max(r, r0))^2, r = |o + depth d / |d| - light|
 *     (F = 1 when r0 = 0 or depth is infinite);
 *   - ground: if d_z != 0 and t = (ground_z - o_z) / d_z > 0 the ray meets the
 *     ground at q = o + t d; q is projected into the light camera and the
 *     shadow map sampled bilinearly at that image position (pixel centres at
 *     +1/2, clamped to the edge inside the image, 0 outside it or behind the
 *     light): G = ground_rgb (1 - k A); otherwise G = background_rgb;
 *   - out = G where the ground is met before the layer's depth (t |d| <
 *     depth), else rgb F + (1 - alpha) G.
 * shadow_map      device [camera.height][camera.width] float32 (the light's
 *                 alpha map, low-passed), or NULL for no shadow.
 * ray_o, ray_d    device [n][3]; rgb device [n][3]; alpha, depth device [n].
 * out_rgb         device [n][3].
 * Errors: ARG, RANGE, HIP.
 */
int neuvv_shade(const neuvv_light* light, const float* shadow_map, int64_t n, const float* ray_o, const float* ray_d,
                const float* rgb, const float* alpha, const float* depth, float* out_rgb, void* stream);

/* Library ABI version (major * 100 + minor). */
int neuvv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NEUVV_H */
