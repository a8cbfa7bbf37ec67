// Host-side launchers shared by the C ABI (api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "neuvv_device.h"

namespace neuvv {

// Per-sample trace of a forward call, replayed by the adjoint of the same
// call instead of walking the tree and evaluating the leaves again.
struct TraceArgs {
    int32_t* head;                 // [n_rays] first sample of the ray's trace; -1: none (the adjoint walks)
    int4* smp;                     // [cap][2] (32-byte entries). K = 16, C = 8 form, one entry per sample:
                                   // {leaf, delta, x, c_r} {c_g, c_b, next (-1: last), 0}; per-point form,
                                   // two: {leaf, delta, x, y} {c_r, c_g, c_b, next} {dz/dgamma [3], 0} {-}
    unsigned long long* counter;   // kQueues counters 128 bytes apart: the first 1024 bytes of a 2048-byte
                                   // header whose second half takes the stores of samples without a slot
    int64_t cap;
};
// Bytes of a trace buffer for n rays and room for cap samples, and its layout.
size_t trace_bytes(int64_t n, int64_t cap);
TraceArgs trace_layout(void* buf, int64_t n, int64_t cap);

struct RenderOut {
    float* rgb;          // each output may be nullptr (not written)
    float* alpha;
    float* depth;
    int32_t* nsamp;
    int32_t* last_leaf;  // slot of the last sample of a ray that stopped early, else -1
    TraceArgs trace;     // head == nullptr: no trace (K = 16, C = 8 form only)
};

struct BackwardIO {
    const float* rgb;
    const float* alpha;
    const int32_t* nsamp;
    const float* grad_rgb;
    const float* grad_alpha;
    float* grad_leaf;    // [n_leaves][grad_row_elems(K, C, Cg)]
    float* grad_basis;
    float* grad_basis_g;   // per-point hyperangle basis gradient (Cg > 0), or nullptr
    int64_t record_cap;    // two-phase adjoint: sample records at most (0: per-sample atomics only)
    TraceArgs trace;       // head == nullptr: walk every ray (K = 16, C = 8 form only)
};

// Per-sample records of the two-phase adjoint: a sample's gradient with
// respect to its colour logits and density logit is written once and linked
// into its leaf's list; a second pass sums each leaf's list into its
// gradient row (one row addition per leaf instead of one per sample).
struct RecordArgs {
    int32_t* head;                 // [n_leaves] first record of the leaf's list, -1: none
    int4* rec;                     // [cap][2]: {dL/dz_r, dL/dz_g, dL/dz_b, dL/dx} (float bits),
                                   //           {next record of the same leaf (-1: end), ray, 0, 0};
                                   // K = 16, C = 8 form with one time for every ray: {next, ray
                                   // direction (world, float bits)} instead
    unsigned long long* counter;   // records handed out so far, one counter per XCD part of the room
    unsigned long long* leaf_cursor;   // second pass: leaves handed out so far
    int64_t cap;
};

// Each returns hipSuccess or the launch error. K, C, dtype must be supported
// (checked by the caller with render_supported()).
bool render_supported(int K, int C, int Cg, int dtype);
// Floats per row of the leaf-major gradient array: 3K + C + Cg rounded up to 64.
int grad_row_elems(int K, int C, int Cg);
// ws: scratch of at least list_scratch_bytes(ra.n_slots) bytes that the call
// uses instead of taking its own from the pool (nothing is then allocated),
// or nullptr.
hipError_t launch_render_fwd(int K, int C, int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                             float t_stop, const RenderOut& out, hipStream_t stream, void* ws = nullptr);
hipError_t launch_render_bwd(int K, int C, int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                             const BackwardIO& io, hipStream_t stream);
// The same for one compiled shape (instantiated in render_k*.hip).
template <int K, int C>
hipError_t launch_render_fwd_shape(int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                                   float t_stop, const RenderOut& out, hipStream_t stream, void* ws);
template <int K, int C>
hipError_t launch_render_bwd_shape(int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                                   const BackwardIO& io, hipStream_t stream);
// Exact merge of up to 4 instances along each ray (K = 16, C = 8 form).
struct MultiArgs {
    TreeArgs tr[4];
    InstArgs in[4];
};
hipError_t launch_render_multi(int L, int dtype, const MultiArgs& ma, const RayArgs& ra, float t_stop,
                               const RenderOut& out, hipStream_t stream);
// Per-point hyperangle form (K = 14, C = 31, Cg = 31).
hipError_t launch_render_pp_fwd(int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, float t_stop,
                                const RenderOut& out, hipStream_t stream, void* ws = nullptr);
hipError_t launch_render_pp_bwd(int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                                const BackwardIO& io, hipStream_t stream);
hipError_t launch_compose_fwd(int L, int64_t n, const float* rgb, const float* alpha, const float* depth,
                              float* out_rgb, float* out_alpha, float* out_depth, hipStream_t stream);
hipError_t launch_compose_bwd(int L, int64_t n, const float* rgb, const float* alpha, const float* depth,
                              const float* g_rgb, const float* g_alpha, float* grad_rgb, float* grad_alpha,
                              hipStream_t stream);
hipError_t launch_pinhole(int W, int H, const float intr[4], const float c2w[12], int64_t n, const int32_t* pix,
                          float* ray_o, float* ray_d, hipStream_t stream);
hipError_t launch_eval_hh(int K, int64_t n, const float* dirs, const float* gam, float* out, hipStream_t stream);
hipError_t launch_pack_rows(int R, int dtype, int layout, int64_t n, const float* in, const int64_t* slot_of_input,
                            void* out, hipStream_t stream);
hipError_t launch_pack(int K, int C, int dtype, int layout, int64_t n, const float* hh_in, const float* wsig_in,
                       const int64_t* slot_of_input, void* hh_out, void* wsig_out, hipStream_t stream);
// The brick directory of a depth-D node table (directory_entries(D) entries).
hipError_t launch_build_directory(const int4* nodes, int depth, int32_t* dir, hipStream_t stream);

// Lighting (Sec. 5.2): Gaussian taps of the shadow-map low-pass, and the light.
constexpr int kMaxBlurRadius = 48;
struct BlurTaps {
    int radius;
    float w[2 * kMaxBlurRadius + 1];
};
struct LightArgs {
    float R[9], C[3];            // light camera: row-major rotation (camera to world) and centre
    float fx, fy, cx, cy;
    int W, H;                    // shadow-map size
    float ground_z, ground[3], bg[3];
    float k, r0;                 // shadow strength, falloff reference distance (0: off)
};
hipError_t launch_blur(int H, int W, const float* in, const BlurTaps& taps, float* out, hipStream_t stream);
hipError_t launch_shade(const LightArgs& L, const float* shadow_map, int64_t n, const float* ray_o, const float* ray_d,
                        const float* rgb, const float* alpha, const float* depth, float* out, hipStream_t stream);

// Appearance edits: rays ending in a leaf write its edit row (lowest ray index wins).
hipError_t launch_paint(int64_t n, const int32_t* last_leaf, const float* colours, float sigma_d, float t_d,
                        int64_t n_leaves, float* edit, hipStream_t stream);

// Device properties used to size persistent grids (cached per device).
int device_cu_count();

// Scratch of a forward launch in the candidate form: a 2 KiB header (the
// work-queue counters, then the per-part list counts, 128 bytes apart) and
// one int32 list entry per work slot.
constexpr size_t kListHeaderBytes = 2048;
inline size_t list_scratch_bytes(int64_t n_slots) {
    return kListHeaderBytes + (size_t)((n_slots + 63) >> 6) * 64 * sizeof(int32_t);
}

// The fixed device scratch of neuvv_render_noalloc: room for the candidate
// form of launches of at most kFixedScratchSlots work slots (64 MiB + 2 KiB,
// held by every device the library runs on until the process ends).
constexpr int64_t kFixedScratchSlots = (int64_t)1 << 24;
constexpr size_t kFixedScratchBytes = kListHeaderBytes + (size_t)kFixedScratchSlots * sizeof(int32_t);
// Device address of that array on the current device (looked up once per
// device; the array's host-side name is not a device address).
hipError_t fixed_scratch(void** p);

// Stream-ordered scratch of a launch (work-queue counters, candidate lists):
// taken from a memory pool the library keeps per device, which holds on to
// its memory between calls instead of returning it at every synchronisation.
hipError_t work_alloc(void** p, size_t bytes, hipStream_t stream);
hipError_t work_free(void* p, hipStream_t stream);

}  // namespace neuvv
