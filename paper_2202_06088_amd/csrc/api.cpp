// C ABI of libneuvv.so (declared in include/neuvv.h): argument validation,
// dtype/K/C dispatch and error reporting around the kernels. Nothing here
// keeps pointers to caller buffers beyond a call. The render calls take
// their scratch (work-queue counters, candidate lists, adjoint records) from
// a stream-ordered memory pool the library keeps per device (render.hip),
// except neuvv_render_noalloc, which uses a fixed device array.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <cmath>
#include <exception>
#include <string>

#include "../../include/neuvv.h"
#include "launch.h"

namespace neuvv {
int build_voctree_host(int32_t depth, int64_t n, const int32_t* ijk, int32_t* nodes, int64_t capacity,
                       int64_t* n_nodes_out, int64_t* slot_of_input, int32_t* box_out, std::string& err);
}

namespace {

thread_local std::string g_err;

// Idle lanes that trigger a wavefront refill in the render kernels: 32 unless
// NEUVV_REFILL_MIN (1..64) is set in the environment (a tuning knob).
int refill_min() {
    static int v = [] {
        const char* e = getenv("NEUVV_REFILL_MIN");
        int x = e ? atoi(e) : 32;
        return x >= 1 && x <= 64 ? x : 32;
    }();
    return v;
}

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return NEUVV_OK;
    return fail(NEUVV_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int check_tree(const neuvv_tree* t) {
    if (!t) return fail(NEUVV_ERR_ARG, "tree is NULL");
    if (t->depth < 1 || t->depth > neuvv::kMaxDepth) return fail(NEUVV_ERR_RANGE, "depth %d outside [1, 12]", t->depth);
    if (t->dtype < 0 || t->dtype > 2) return fail(NEUVV_ERR_ARG, "unknown dtype %d", t->dtype);
    if (t->layout < 0 || t->layout > 1) return fail(NEUVV_ERR_ARG, "unknown layout %d", t->layout);
    if (!neuvv::render_supported(t->K, t->C, t->Cg, t->dtype))
        return fail(NEUVV_ERR_UNSUPPORTED,
                    "no kernel compiled for K=%d C=%d Cg=%d (have K in {14,16,30} x C in {8,31} with Cg=0, and "
                    "K=14 C=31 Cg=31)", t->K, t->C,
                    t->Cg);
    if (t->n_nodes < 1 || t->n_nodes > INT32_MAX) return fail(NEUVV_ERR_RANGE, "n_nodes %lld", (long long)t->n_nodes);
    if (t->n_leaves < 0 || t->n_leaves > INT32_MAX)
        return fail(NEUVV_ERR_RANGE, "n_leaves %lld", (long long)t->n_leaves);
    if (t->T < 1) return fail(NEUVV_ERR_RANGE, "T = %d must be >= 1", t->T);
    if (!t->nodes || !t->basis) return fail(NEUVV_ERR_ARG, "tree nodes/basis pointer is NULL");
    if (!t->dir) return fail(NEUVV_ERR_ARG, "tree dir is NULL (neuvv_build_directory fills it)");
    if (reinterpret_cast<uintptr_t>(t->dir) % 4 != 0) return fail(NEUVV_ERR_ARG, "tree dir must be 4-byte aligned");
    if (t->Cg == 0 && !t->gamma) return fail(NEUVV_ERR_ARG, "tree gamma pointer is NULL");
    if (t->Cg > 0 && !t->basis_g) return fail(NEUVV_ERR_ARG, "tree basis_g pointer is NULL");
    if (reinterpret_cast<uintptr_t>(t->nodes) % 16 != 0) return fail(NEUVV_ERR_ARG, "tree nodes must be 16-byte aligned");
    const bool box_unset = !(t->box[0] | t->box[1] | t->box[2] | t->box[3] | t->box[4] | t->box[5]);
    if (!box_unset)
        for (int a = 0; a < 3; ++a)
            if (t->box[a] < 0 || t->box[a] >= t->box[3 + a] || t->box[3 + a] > (1 << t->depth))
                return fail(NEUVV_ERR_RANGE, "tree box must satisfy 0 <= lo < hi <= 2^depth on every axis");
    if (t->n_leaves > 0 && (!t->hh || !t->wsig || (t->Cg > 0 && !t->wgam)))
        return fail(NEUVV_ERR_ARG, "tree payload pointer is NULL");
    if (t->edit && reinterpret_cast<uintptr_t>(t->edit) % 16 != 0)
        return fail(NEUVV_ERR_ARG, "tree edit rows must be 16-byte aligned");
    if (t->edit && (t->Cg > 0 || t->K != 16 || t->C != 8))
        return fail(NEUVV_ERR_UNSUPPORTED, "appearance edits are compiled for the K=16 C=8 form only");
    if (t->density != NEUVV_DENSITY_SOFTPLUS && t->density != NEUVV_DENSITY_RELU)
        return fail(NEUVV_ERR_ARG, "unknown density activation %d", t->density);
    return NEUVV_OK;
}

int make_inst(const neuvv_instance* in, neuvv::InstArgs& a) {
    if (!in) {
        for (int i = 0; i < 9; ++i) a.rot[i] = (i % 4 == 0) ? 1.0f : 0.0f;
        a.trans[0] = a.trans[1] = a.trans[2] = 0.0f;
        a.scale = 1.0f;
        a.time_offset = 0.0f;
        a.wrap = 0;
        a.identity = 1;
        return NEUVV_OK;
    }
    if (!(in->scale > 0.0f) || !std::isfinite(in->scale)) return fail(NEUVV_ERR_RANGE, "instance scale must be > 0");
    if (!std::isfinite(in->time_offset)) return fail(NEUVV_ERR_RANGE, "instance time_offset must be finite");
    for (int i = 0; i < 9; ++i) {
        if (!std::isfinite(in->rot[i])) return fail(NEUVV_ERR_RANGE, "instance rotation must be finite");
        a.rot[i] = in->rot[i];
    }
    for (int i = 0; i < 3; ++i) {
        if (!std::isfinite(in->trans[i])) return fail(NEUVV_ERR_RANGE, "instance translation must be finite");
        a.trans[i] = in->trans[i];
    }
    a.scale = in->scale;
    a.time_offset = in->time_offset;
    a.wrap = in->time_wrap != 0;
    a.identity = 0;
    return NEUVV_OK;
}

int make_rays(int64_t n, const float* o, const float* d, const float* t, float t_scalar, int32_t image_width,
              neuvv::RayArgs& ra) {
    if (n < 0) return fail(NEUVV_ERR_ARG, "n_rays < 0");
    if (n > 0 && (!o || !d)) return fail(NEUVV_ERR_ARG, "ray_o / ray_d is NULL");
    if (image_width < 0) return fail(NEUVV_ERR_RANGE, "image_width < 0");
    if (!std::isfinite(t_scalar)) return fail(NEUVV_ERR_RANGE, "t_scalar must be finite");
    ra.o = o;
    ra.d = d;
    ra.t = t;
    ra.t_scalar = t_scalar;
    ra.n = n;
    ra.img_w = image_width;
    ra.refill_min = refill_min();
    ra.queue = nullptr;
    ra.list = nullptr;
    ra.count = nullptr;
    if (image_width > 0) {
        const int64_t rows = (n + image_width - 1) / image_width;
        ra.tiles_x = (image_width + 7) / 8;
        ra.n_slots = (int64_t)ra.tiles_x * ((rows + 7) / 8) * 64;
    } else {
        ra.tiles_x = 0;
        ra.n_slots = n;
    }
    return NEUVV_OK;
}

// Sample records of the two-phase adjoint: NEUVV_BWD_RECORDS overrides (0
// turns the records off); by default room for two samples per ray or, after a
// traced forward, for as many samples as the trace has room for if that is
// more (every replayed sample has a trace entry); at least 2^20, at most
// 2^31 - 1. Samples beyond the room take per-sample atomics.
int64_t record_cap(int64_t n_rays, int64_t trace_cap) {
    const char* e = getenv("NEUVV_BWD_RECORDS");
    int64_t cap = 2 * n_rays > trace_cap ? 2 * n_rays : trace_cap;
    if (cap < (int64_t)1 << 20) cap = (int64_t)1 << 20;
    if (e && *e) cap = atoll(e);
    if (cap < 0) cap = 0;
    if (cap > (int64_t)INT32_MAX) cap = INT32_MAX;
    return cap;
}

neuvv::TreeArgs tree_args(const neuvv_tree* t) {
    neuvv::TreeArgs a;
    a.nodes = reinterpret_cast<const int4*>(t->nodes);
    a.hh = t->hh;
    a.wsig = t->wsig;
    a.basis = t->basis;
    a.gamma = t->gamma;
    a.Cg = t->Cg;
    a.wgam = t->wgam;
    a.basis_g = t->basis_g;
    a.edit = reinterpret_cast<const float4*>(t->edit);
    a.dir = t->dir;
    a.n_nodes = t->n_nodes;
    a.n_leaves = t->n_leaves;
    a.depth = t->depth;
    a.T = t->T;
    const bool box_unset = !(t->box[0] | t->box[1] | t->box[2] | t->box[3] | t->box[4] | t->box[5]);
    for (int i = 0; i < 3; ++i) {
        a.box_lo[i] = box_unset ? 0 : t->box[i];
        a.box_hi[i] = box_unset ? (1 << t->depth) : t->box[3 + i];
    }
    a.layout = t->layout;
    a.relu = t->density == NEUVV_DENSITY_RELU;
    return a;
}

}  // namespace

#define NEUVV_GUARD_BEGIN try {
#define NEUVV_GUARD_END                                                   \
    }                                                                     \
    catch (const std::exception& e) {                                     \
        return fail(NEUVV_ERR_ARG, "internal exception: %s", e.what());   \
    }                                                                     \
    catch (...) {                                                         \
        return fail(NEUVV_ERR_ARG, "internal exception");                 \
    }

extern "C" {

int neuvv_version(void) { return 200; }

const char* neuvv_last_error(void) { return g_err.c_str(); }

int neuvv_build_voctree(int32_t depth, int64_t n_leaves, const int32_t* leaf_ijk, int32_t* nodes,
                        int64_t node_capacity, int64_t* n_nodes_out, int64_t* slot_of_input, int32_t* box_out) {
    NEUVV_GUARD_BEGIN
    if (depth < 1 || depth > neuvv::kMaxDepth) return fail(NEUVV_ERR_RANGE, "depth %d outside [1, 12]", depth);
    if (n_leaves < 0) return fail(NEUVV_ERR_ARG, "n_leaves < 0");
    if (n_leaves > 0 && !leaf_ijk) return fail(NEUVV_ERR_ARG, "leaf_ijk is NULL");
    if (!n_nodes_out) return fail(NEUVV_ERR_ARG, "n_nodes_out is NULL");
    std::string err;
    const int rc = neuvv::build_voctree_host(depth, n_leaves, leaf_ijk, nodes, node_capacity, n_nodes_out,
                                             slot_of_input, box_out, err);
    if (rc != 0) return fail(rc, "%s", err.c_str());
    return NEUVV_OK;
    NEUVV_GUARD_END
}

int neuvv_payload_words(int32_t K, int32_t C, int32_t dtype, int64_t n_leaves, int64_t* hh_elems,
                        int64_t* wsig_elems) {
    if (K < 1 || K > 30 || C < 1 || C > 64) return fail(NEUVV_ERR_RANGE, "K in [1,30] and C in [1,64] required");
    if (dtype < 0 || dtype > 2) return fail(NEUVV_ERR_ARG, "unknown dtype %d", dtype);
    if (n_leaves < 0 || !hh_elems || !wsig_elems) return fail(NEUVV_ERR_ARG, "bad n_leaves or NULL output");
    const int V = dtype == NEUVV_F32 ? 4 : 8;
    *hh_elems = (int64_t)((3 * K + V - 1) / V) * n_leaves * V;
    *wsig_elems = (int64_t)((C + V - 1) / V) * n_leaves * V;
    return NEUVV_OK;
}

int neuvv_grad_row_elems(int32_t K, int32_t C, int32_t Cg) {
    if (K < 1 || K > 30 || C < 1 || C > 64 || Cg < 0 || Cg > 64)
        return fail(NEUVV_ERR_RANGE, "K in [1,30], C in [1,64] and Cg in [0,64] required");
    return neuvv::grad_row_elems(K, C, Cg);
}

int neuvv_pack_rows(int32_t R, int32_t dtype, int32_t layout, int64_t n_leaves, const float* in,
                    const int64_t* slot_of_input, void* out, void* stream) {
    NEUVV_GUARD_BEGIN
    if (R < 1 || R > 256) return fail(NEUVV_ERR_RANGE, "R in [1,256] required");
    if (dtype < 0 || dtype > 2) return fail(NEUVV_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (layout < 0 || layout > 1) return fail(NEUVV_ERR_UNSUPPORTED, "unknown layout %d", layout);
    if (n_leaves < 0) return fail(NEUVV_ERR_ARG, "n_leaves < 0");
    if (n_leaves > 0 && (!in || !out)) return fail(NEUVV_ERR_ARG, "NULL buffer");
    return hip_status(neuvv::launch_pack_rows(R, dtype, layout, n_leaves, in, slot_of_input, out, (hipStream_t)stream),
                      "pack_rows launch");
    NEUVV_GUARD_END
}

int neuvv_pack_leaves(int32_t K, int32_t C, int32_t dtype, int32_t layout, int64_t n_leaves, const float* hh_in,
                      const float* wsig_in, const int64_t* slot_of_input, void* hh_out, void* wsig_out,
                      void* stream) {
    NEUVV_GUARD_BEGIN
    if (K < 1 || K > 30 || C < 1 || C > 64) return fail(NEUVV_ERR_RANGE, "K in [1,30] and C in [1,64] required");
    if (dtype < 0 || dtype > 2) return fail(NEUVV_ERR_UNSUPPORTED, "unknown dtype %d", dtype);
    if (layout < 0 || layout > 1) return fail(NEUVV_ERR_UNSUPPORTED, "unknown layout %d", layout);
    if (n_leaves < 0) return fail(NEUVV_ERR_ARG, "n_leaves < 0");
    if (n_leaves > 0 && (!hh_in || !wsig_in || !hh_out || !wsig_out)) return fail(NEUVV_ERR_ARG, "NULL buffer");
    return hip_status(neuvv::launch_pack(K, C, dtype, layout, n_leaves, hh_in, wsig_in, slot_of_input, hh_out, wsig_out,
                                         (hipStream_t)stream),
                      "pack_leaves launch");
    NEUVV_GUARD_END
}

int64_t neuvv_directory_entries(int32_t depth) {
    if (depth < 1 || depth > neuvv::kMaxDepth) return -1;
    return neuvv::directory_entries(depth);
}

int neuvv_build_directory(int32_t depth, int64_t n_nodes, const int32_t* nodes, int32_t* dir, int64_t capacity,
                          void* stream) {
    NEUVV_GUARD_BEGIN
    if (depth < 1 || depth > neuvv::kMaxDepth) return fail(NEUVV_ERR_RANGE, "depth %d outside [1, 12]", depth);
    if (n_nodes < 1 || n_nodes > INT32_MAX) return fail(NEUVV_ERR_RANGE, "n_nodes %lld", (long long)n_nodes);
    if (!nodes || !dir) return fail(NEUVV_ERR_ARG, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(nodes) % 16 != 0) return fail(NEUVV_ERR_ARG, "nodes must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(dir) % 4 != 0) return fail(NEUVV_ERR_ARG, "dir must be 4-byte aligned");
    const int64_t need = neuvv::directory_entries(depth);
    if (capacity < need)
        return fail(NEUVV_ERR_CAPACITY, "dir holds %lld entries, depth %d needs %lld", (long long)capacity, depth,
                    (long long)need);
    return hip_status(neuvv::launch_build_directory(reinterpret_cast<const int4*>(nodes), depth, dir,
                                                    (hipStream_t)stream),
                      "build_directory launch");
    NEUVV_GUARD_END
}

// Checks a trace buffer argument (traced calls only).
static int check_trace(int64_t n_rays, const void* trace, int64_t trace_cap) {
    if (!trace) return fail(NEUVV_ERR_ARG, "trace is NULL");
    if (reinterpret_cast<uintptr_t>(trace) % 256) return fail(NEUVV_ERR_ARG, "trace must be 256-byte aligned");
    if (trace_cap < 0 || trace_cap > (int64_t)INT32_MAX) return fail(NEUVV_ERR_RANGE, "trace_cap outside [0, 2^31)");
    if (n_rays > (int64_t)INT32_MAX) return fail(NEUVV_ERR_RANGE, "traced calls take fewer than 2^31 rays");
    return NEUVV_OK;
}

// fixed: take the call's scratch from the library's fixed device array (no
// allocation) instead of the pool; launches beyond its room are rejected.
static int render_impl(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width, float t_stop, float* rgb,
                float* alpha, float* depth, int32_t* nsamp, void* trace, int64_t trace_cap, void* stream,
                bool fixed = false) {
    int rc = check_tree(tree);
    if (rc) return rc;
    neuvv::InstArgs in;
    if ((rc = make_inst(inst, in))) return rc;
    neuvv::RayArgs ra;
    if ((rc = make_rays(n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, ra))) return rc;
    if (!(t_stop >= 0.0f) || !std::isfinite(t_stop)) return fail(NEUVV_ERR_RANGE, "t_stop must be >= 0");
    if (n_rays > 0 && (!rgb || !alpha || !nsamp)) return fail(NEUVV_ERR_ARG, "rgb / alpha / nsamp is NULL");
    void* ws = nullptr;
    if (fixed) {
        if (ra.n_slots > neuvv::kFixedScratchSlots)
            return fail(NEUVV_ERR_CAPACITY,
                        "neuvv_render_noalloc takes at most %lld work slots (rays, or 8x8 tiles x 64 with "
                        "image_width); this call has %lld",
                        (long long)neuvv::kFixedScratchSlots, (long long)ra.n_slots);
        if (ra.n_slots == 0) return NEUVV_OK;
        rc = hip_status(neuvv::fixed_scratch(&ws), "device address of the fixed scratch");
        if (rc) return rc;
    }
    neuvv::RenderOut out{rgb, alpha, depth, nsamp, nullptr};
    if (trace) out.trace = neuvv::trace_layout(trace, n_rays, trace_cap);
    const hipError_t e = tree->Cg > 0
                             ? neuvv::launch_render_pp_fwd(tree->dtype, tree_args(tree), in, ra, t_stop, out,
                                                           (hipStream_t)stream, ws)
                             : neuvv::launch_render_fwd(tree->K, tree->C, tree->dtype, tree_args(tree), in, ra,
                                                        t_stop, out, (hipStream_t)stream, ws);
    return hip_status(e, "render launch");
}

static int backward_impl(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                  const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width, float t_stop,
                  const float* rgb, const float* alpha, const int32_t* nsamp, const float* grad_rgb,
                  const float* grad_alpha, float* grad_leaf, float* grad_basis, float* grad_basis_g,
                  const void* trace, int64_t trace_cap, void* stream) {
    int rc = check_tree(tree);
    if (rc) return rc;
    neuvv::InstArgs in;
    if ((rc = make_inst(inst, in))) return rc;
    neuvv::RayArgs ra;
    if ((rc = make_rays(n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, ra))) return rc;
    if (!(t_stop >= 0.0f) || !std::isfinite(t_stop)) return fail(NEUVV_ERR_RANGE, "t_stop must be >= 0");
    if (n_rays > 0 && (!rgb || !alpha || !nsamp || !grad_rgb))
        return fail(NEUVV_ERR_ARG, "rgb / alpha / nsamp / grad_rgb is NULL");
    if (tree->n_leaves > 0 && !grad_leaf) return fail(NEUVV_ERR_ARG, "grad_leaf is NULL");
    if (tree->edit) return fail(NEUVV_ERR_UNSUPPORTED, "no adjoint through appearance edits");
    neuvv::BackwardIO io{rgb, alpha, nsamp, grad_rgb, grad_alpha, grad_leaf, grad_basis,
                         tree->Cg > 0 ? grad_basis_g : nullptr, record_cap(n_rays, trace ? trace_cap : 0)};
    if (trace) io.trace = neuvv::trace_layout(const_cast<void*>(trace), n_rays, trace_cap);
    const hipError_t e = tree->Cg > 0
                             ? neuvv::launch_render_pp_bwd(tree->dtype, tree_args(tree), in, ra, io,
                                                           (hipStream_t)stream)
                             : neuvv::launch_render_bwd(tree->K, tree->C, tree->dtype, tree_args(tree), in, ra, io,
                                                        (hipStream_t)stream);
    return hip_status(e, "render_backward launch");
}

int neuvv_render(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                 const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width, float t_stop,
                 float* rgb, float* alpha, float* depth, int32_t* nsamp, void* stream) {
    NEUVV_GUARD_BEGIN
    return render_impl(tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop, rgb, alpha, depth,
                       nsamp, nullptr, 0, stream);
    NEUVV_GUARD_END
}

int neuvv_render_noalloc(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                         const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width, float t_stop,
                         float* rgb, float* alpha, float* depth, int32_t* nsamp, void* stream) {
    NEUVV_GUARD_BEGIN
    return render_impl(tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop, rgb, alpha, depth,
                       nsamp, nullptr, 0, stream, true);
    NEUVV_GUARD_END
}

int neuvv_render_backward(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays,
                          const float* ray_o, const float* ray_d, const float* ray_t, float t_scalar,
                          int32_t image_width, float t_stop, const float* rgb, const float* alpha,
                          const int32_t* nsamp, const float* grad_rgb, const float* grad_alpha, float* grad_leaf,
                          float* grad_basis, float* grad_basis_g, void* stream) {
    NEUVV_GUARD_BEGIN
    return backward_impl(tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop, rgb, alpha, nsamp,
                         grad_rgb, grad_alpha, grad_leaf, grad_basis, grad_basis_g, nullptr, 0, stream);
    NEUVV_GUARD_END
}

int64_t neuvv_trace_bytes(int64_t n_rays, int64_t trace_cap) {
    if (n_rays < 0 || trace_cap < 0) return -1;
    return (int64_t)neuvv::trace_bytes(n_rays, trace_cap);
}

int neuvv_render_trace(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                       const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width, float t_stop,
                       float* rgb, float* alpha, float* depth, int32_t* nsamp, void* trace, int64_t trace_cap,
                       void* stream) {
    NEUVV_GUARD_BEGIN
    int rc = check_tree(tree);
    if (rc) return rc;
    if ((rc = check_trace(n_rays, trace, trace_cap))) return rc;
    return render_impl(tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop, rgb, alpha, depth,
                       nsamp, trace, trace_cap, stream);
    NEUVV_GUARD_END
}

int neuvv_render_backward_trace(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays,
                                const float* ray_o, const float* ray_d, const float* ray_t, float t_scalar,
                                int32_t image_width, float t_stop, const float* rgb, const float* alpha,
                                const int32_t* nsamp, const float* grad_rgb, const float* grad_alpha,
                                float* grad_leaf, float* grad_basis, float* grad_basis_g, const void* trace,
                                int64_t trace_cap, void* stream) {
    NEUVV_GUARD_BEGIN
    int rc = check_tree(tree);
    if (rc) return rc;
    if ((rc = check_trace(n_rays, trace, trace_cap))) return rc;
    return backward_impl(tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop, rgb, alpha, nsamp,
                         grad_rgb, grad_alpha, grad_leaf, grad_basis, grad_basis_g, trace, trace_cap, stream);
    NEUVV_GUARD_END
}

int neuvv_compose(int32_t L, int64_t n_pix, const float* rgb, const float* alpha, const float* depth,
                  float* out_rgb, float* out_alpha, float* out_depth, void* stream) {
    NEUVV_GUARD_BEGIN
    if (L < 1 || L > 16) return fail(NEUVV_ERR_RANGE, "L = %d outside [1, 16]", L);
    if (n_pix < 0) return fail(NEUVV_ERR_ARG, "n_pix < 0");
    if (n_pix > 0 && (!rgb || !alpha || !depth || !out_rgb || !out_alpha)) return fail(NEUVV_ERR_ARG, "NULL buffer");
    return hip_status(neuvv::launch_compose_fwd(L, n_pix, rgb, alpha, depth, out_rgb, out_alpha, out_depth,
                                                (hipStream_t)stream),
                      "compose launch");
    NEUVV_GUARD_END
}

int neuvv_compose_backward(int32_t L, int64_t n_pix, const float* rgb, const float* alpha, const float* depth,
                           const float* grad_out_rgb, const float* grad_out_alpha, float* grad_rgb,
                           float* grad_alpha, void* stream) {
    NEUVV_GUARD_BEGIN
    if (L < 1 || L > 16) return fail(NEUVV_ERR_RANGE, "L = %d outside [1, 16]", L);
    if (n_pix < 0) return fail(NEUVV_ERR_ARG, "n_pix < 0");
    if (n_pix > 0 && (!rgb || !alpha || !depth || !grad_out_rgb || !grad_rgb || !grad_alpha))
        return fail(NEUVV_ERR_ARG, "NULL buffer");
    return hip_status(neuvv::launch_compose_bwd(L, n_pix, rgb, alpha, depth, grad_out_rgb, grad_out_alpha, grad_rgb,
                                                grad_alpha, (hipStream_t)stream),
                      "compose_backward launch");
    NEUVV_GUARD_END
}

int neuvv_pinhole_rays(const neuvv_camera* cam, int64_t n, const int32_t* pix, float* ray_o, float* ray_d,
                       void* stream) {
    NEUVV_GUARD_BEGIN
    if (!cam) return fail(NEUVV_ERR_ARG, "camera is NULL");
    if (cam->width < 1 || cam->height < 1) return fail(NEUVV_ERR_RANGE, "camera size must be positive");
    if ((int64_t)cam->width * cam->height > INT32_MAX) return fail(NEUVV_ERR_RANGE, "camera too large");
    if (cam->width > (1 << 23) || cam->height > (1 << 23)) return fail(NEUVV_ERR_RANGE, "camera too large");
    if (!(cam->fx != 0.0f) || !(cam->fy != 0.0f) || !std::isfinite(cam->fx) || !std::isfinite(cam->fy))
        return fail(NEUVV_ERR_RANGE, "focal lengths must be finite and non-zero");
    if (n < 0) return fail(NEUVV_ERR_ARG, "n < 0");
    if (!pix && n != (int64_t)cam->width * cam->height) return fail(NEUVV_ERR_ARG, "pix NULL requires n = W*H");
    if (n > 0 && (!ray_o || !ray_d)) return fail(NEUVV_ERR_ARG, "ray_o / ray_d is NULL");
    const float intr[4] = {cam->fx, cam->fy, cam->cx, cam->cy};
    return hip_status(neuvv::launch_pinhole(cam->width, cam->height, intr, cam->c2w, n, pix, ray_o, ray_d,
                                            (hipStream_t)stream),
                      "pinhole launch");
    NEUVV_GUARD_END
}

int neuvv_eval_hh(int32_t K, int64_t n, const float* dirs, const float* gam, float* out, void* stream) {
    NEUVV_GUARD_BEGIN
    if (K < 1 || K > 30) return fail(NEUVV_ERR_RANGE, "K = %d outside [1, 30]", K);
    if (n < 0) return fail(NEUVV_ERR_ARG, "n < 0");
    if (n > 0 && (!dirs || !gam || !out)) return fail(NEUVV_ERR_ARG, "NULL buffer");
    return hip_status(neuvv::launch_eval_hh(K, n, dirs, gam, out, (hipStream_t)stream), "eval_hh launch");
    NEUVV_GUARD_END
}

int neuvv_render_multi(int32_t n_inst, const neuvv_tree* const* trees, const neuvv_instance* insts, int64_t n_rays,
                       const float* ray_o, const float* ray_d, const float* ray_t, float t_scalar,
                       int32_t image_width, float t_stop, float* rgb, float* alpha, float* depth, int32_t* nsamp,
                       void* stream) {
    NEUVV_GUARD_BEGIN
    if (n_inst < 1 || n_inst > 4) return fail(NEUVV_ERR_RANGE, "n_inst = %d outside [1, 4]", n_inst);
    if (!trees) return fail(NEUVV_ERR_ARG, "trees is NULL");
    neuvv::MultiArgs ma;
    int dtype = -1;
    for (int k = 0; k < n_inst; ++k) {
        int rc = check_tree(trees[k]);
        if (rc) return rc;
        if (trees[k]->K != 16 || trees[k]->C != 8 || trees[k]->Cg != 0 || trees[k]->edit)
            return fail(NEUVV_ERR_UNSUPPORTED, "the exact merge is compiled for the K=16 C=8 form without edits");
        if (dtype >= 0 && trees[k]->dtype != dtype)
            return fail(NEUVV_ERR_UNSUPPORTED, "all trees of one merge must share the storage dtype");
        dtype = trees[k]->dtype;
        ma.tr[k] = tree_args(trees[k]);
        if ((rc = make_inst(insts ? &insts[k] : nullptr, ma.in[k]))) return rc;
    }
    for (int k = n_inst; k < 4; ++k) {
        ma.tr[k] = ma.tr[0];
        ma.in[k] = ma.in[0];
    }
    neuvv::RayArgs ra;
    int rc = make_rays(n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, ra);
    if (rc) return rc;
    if (!(t_stop >= 0.0f) || !std::isfinite(t_stop)) return fail(NEUVV_ERR_RANGE, "t_stop must be >= 0");
    if (n_rays > 0 && (!rgb || !alpha || !nsamp)) return fail(NEUVV_ERR_ARG, "rgb / alpha / nsamp is NULL");
    neuvv::RenderOut out{rgb, alpha, depth, nsamp, nullptr};
    return hip_status(neuvv::launch_render_multi(n_inst, dtype, ma, ra, t_stop, out, (hipStream_t)stream),
                      "render_multi launch");
    NEUVV_GUARD_END
}

int neuvv_find_terminal_leaves(const neuvv_tree* tree, const neuvv_instance* inst, int64_t n_rays, const float* ray_o,
                               const float* ray_d, const float* ray_t, float t_scalar, int32_t image_width,
                               float alpha_threshold, int32_t* last_leaf, void* stream) {
    NEUVV_GUARD_BEGIN
    int rc = check_tree(tree);
    if (rc) return rc;
    if (tree->Cg > 0)
        return fail(NEUVV_ERR_UNSUPPORTED, "terminal leaves are compiled for the global-hyperangle form only");
    neuvv::InstArgs in;
    if ((rc = make_inst(inst, in))) return rc;
    neuvv::RayArgs ra;
    if ((rc = make_rays(n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, ra))) return rc;
    if (!(alpha_threshold > 0.0f && alpha_threshold < 1.0f))
        return fail(NEUVV_ERR_RANGE, "alpha_threshold must be in (0, 1)");
    if (n_rays > 0 && !last_leaf) return fail(NEUVV_ERR_ARG, "last_leaf is NULL");
    neuvv::RenderOut out{nullptr, nullptr, nullptr, nullptr, last_leaf};
    return hip_status(neuvv::launch_render_fwd(tree->K, tree->C, tree->dtype, tree_args(tree), in, ra,
                                               1.0f - alpha_threshold, out, (hipStream_t)stream),
                      "terminal leaves launch");
    NEUVV_GUARD_END
}

int neuvv_paint(int64_t n_rays, const int32_t* last_leaf, const float* colours, float sigma_d, float t_d,
                int64_t n_leaves, float* edit, void* stream) {
    NEUVV_GUARD_BEGIN
    if (n_rays < 0 || n_rays > INT32_MAX) return fail(NEUVV_ERR_RANGE, "n_rays outside [0, 2^31)");
    if (n_leaves < 0) return fail(NEUVV_ERR_ARG, "n_leaves < 0");
    if (n_rays > 0 && (!last_leaf || !colours || !edit)) return fail(NEUVV_ERR_ARG, "NULL buffer");
    if (std::isnan(sigma_d) || std::isnan(t_d)) return fail(NEUVV_ERR_RANGE, "sigma_d and t_d must not be NaN");
    return hip_status(neuvv::launch_paint(n_rays, last_leaf, colours, sigma_d, t_d, n_leaves, edit,
                                          (hipStream_t)stream),
                      "paint launch");
    NEUVV_GUARD_END
}

int neuvv_blur(int32_t height, int32_t width, const float* in, float sigma, float* out, void* stream) {
    NEUVV_GUARD_BEGIN
    if (height < 1 || width < 1 || (int64_t)height * width > INT32_MAX)
        return fail(NEUVV_ERR_RANGE, "map size %d x %d", height, width);
    if (!(sigma > 0.0f) || !(sigma <= 16.0f)) return fail(NEUVV_ERR_RANGE, "sigma must be in (0, 16]");
    if (!in || !out) return fail(NEUVV_ERR_ARG, "in / out is NULL");
    if (in == out) return fail(NEUVV_ERR_ARG, "the low-pass cannot run in place");
    neuvv::BlurTaps taps;
    taps.radius = (int)(3.0 * (double)sigma + 0.5);
    double w[2 * neuvv::kMaxBlurRadius + 1], sum = 0.0;
    for (int i = -taps.radius; i <= taps.radius; ++i) {
        w[i + taps.radius] = std::exp(-(double)i * i / (2.0 * (double)sigma * sigma));
        sum += w[i + taps.radius];
    }
    for (int i = 0; i <= 2 * taps.radius; ++i) taps.w[i] = (float)(w[i] / sum);
    return hip_status(neuvv::launch_blur(height, width, in, taps, out, (hipStream_t)stream), "blur launch");
    NEUVV_GUARD_END
}

int neuvv_shade(const neuvv_light* light, const float* shadow_map, int64_t n, const float* ray_o, const float* ray_d,
                const float* rgb, const float* alpha, const float* depth, float* out_rgb, void* stream) {
    NEUVV_GUARD_BEGIN
    if (!light) return fail(NEUVV_ERR_ARG, "light is NULL");
    const neuvv_camera& c = light->camera;
    if (c.width < 1 || c.height < 1 || (int64_t)c.width * c.height > INT32_MAX)
        return fail(NEUVV_ERR_RANGE, "light camera size must be positive");
    if (!(c.fx != 0.0f) || !(c.fy != 0.0f) || !std::isfinite(c.fx) || !std::isfinite(c.fy))
        return fail(NEUVV_ERR_RANGE, "light focal lengths must be finite and non-zero");
    if (!(light->shadow_strength >= 0.0f && light->shadow_strength <= 1.0f))
        return fail(NEUVV_ERR_RANGE, "shadow_strength must be in [0, 1]");
    if (!(light->falloff_r0 >= 0.0f) || !std::isfinite(light->falloff_r0))
        return fail(NEUVV_ERR_RANGE, "falloff_r0 must be >= 0");
    if (!std::isfinite(light->ground_z)) return fail(NEUVV_ERR_RANGE, "ground_z must be finite");
    if (n < 0) return fail(NEUVV_ERR_ARG, "n < 0");
    if (n > 0 && (!ray_o || !ray_d || !rgb || !alpha || !depth || !out_rgb))
        return fail(NEUVV_ERR_ARG, "NULL buffer");
    neuvv::LightArgs L;
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) L.R[3 * r + q] = c.c2w[4 * r + q];
        L.C[r] = c.c2w[4 * r + 3];
        L.ground[r] = light->ground_rgb[r];
        L.bg[r] = light->background_rgb[r];
    }
    L.fx = c.fx; L.fy = c.fy; L.cx = c.cx; L.cy = c.cy;
    L.W = c.width; L.H = c.height;
    L.ground_z = light->ground_z;
    L.k = light->shadow_strength;
    L.r0 = light->falloff_r0;
    return hip_status(neuvv::launch_shade(L, shadow_map, n, ray_o, ray_d, rgb, alpha, depth, out_rgb,
                                          (hipStream_t)stream),
                      "shade launch");
    NEUVV_GUARD_END
}

}  // extern "C"
