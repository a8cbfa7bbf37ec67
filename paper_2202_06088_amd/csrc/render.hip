// Dispatch of the render calls to the compiled shapes of the
// global-hyperangle form (K HH functions per channel, C density weights), and
// the host-side pieces the render calls share: the scratch pool, the trace
// layout, the device's compute-unit count and the fixed scratch of
// neuvv_render_noalloc. The kernels are in render_kernels.h; each shape is
// compiled in its own file (render_k*.hip).
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.h"

namespace neuvv {

// ----------------------------------------------------------------------------
// launchers

// Compiled shapes: the global-hyperangle form with K in {14, 16, 30} and C in
// {8, 31} (Table 3's N = 14 and 30, the workloads' 16; the workloads' C = 8
// and the paper's 31), and the per-point form with K = 14, C = Cg = 31.
bool render_supported(int K, int C, int Cg, int dtype) {
    const bool global = Cg == 0 && (K == 14 || K == 16 || K == 30) && (C == 8 || C == 31);
    const bool shape = global || (K == 14 && C == 31 && Cg == 31);
    return shape && dtype >= 0 && dtype <= 2;
}

int grad_row_elems(int K, int C, int Cg) { return ((3 * K + C + Cg + 63) / 64) * 64; }

namespace {
std::mutex g_pool_mu;
hipMemPool_t g_pool[64] = {};
bool g_pool_tried[64] = {};
}  // namespace

hipError_t work_alloc(void** p, size_t bytes, hipStream_t stream) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipMemPool_t pool = nullptr;
    if (dev >= 0 && dev < 64) {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (!g_pool_tried[dev]) {
            g_pool_tried[dev] = true;
            hipMemPoolProps props = {};
            props.allocType = hipMemAllocationTypePinned;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = dev;
            hipMemPool_t mp = nullptr;
            if (hipMemPoolCreate(&mp, &props) == hipSuccess) {
                uint64_t keep = ~0ull;   // keep freed memory for the next call
                if (hipMemPoolSetAttribute(mp, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess)
                    g_pool[dev] = mp;
                else
                    (void)hipMemPoolDestroy(mp);
            }
        }
        pool = g_pool[dev];
    }
    return pool ? hipMallocFromPoolAsync(p, bytes, pool, stream) : hipMallocAsync(p, bytes, stream);
}

hipError_t work_free(void* p, hipStream_t stream) { return hipFreeAsync(p, stream); }

size_t trace_bytes(int64_t n, int64_t cap) {
    const size_t head_b = ((size_t)(n > 0 ? n : 0) * sizeof(int32_t) + 255) & ~(size_t)255;
    return 2048 + head_b + (size_t)(cap > 0 ? cap : 0) * 2 * sizeof(int4);
}

TraceArgs trace_layout(void* buf, int64_t n, int64_t cap) {
    TraceArgs t{};
    if (!buf) return t;
    const size_t head_b = ((size_t)(n > 0 ? n : 0) * sizeof(int32_t) + 255) & ~(size_t)255;
    char* p = static_cast<char*>(buf);
    t.counter = reinterpret_cast<unsigned long long*>(p);
    t.head = reinterpret_cast<int32_t*>(p + 2048);
    t.smp = reinterpret_cast<int4*>(p + 2048 + head_b);
    t.cap = cap;
    return t;
}

int device_cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
        cached[dev] = cu;
    }
    return cached[dev];
}

#define NEUVV_SHAPES(X) X(14, 8) X(16, 8) X(30, 8) X(14, 31) X(16, 31) X(30, 31)

hipError_t launch_render_fwd(int K, int C, int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                             float t_stop, const RenderOut& out, hipStream_t stream, void* ws) {
    if (ra.n_slots <= 0) return hipSuccess;
#define NEUVV_FWD_CASE(k, c) \
    if (K == k && C == c) return launch_render_fwd_shape<k, c>(dtype, tr, in, ra, t_stop, out, stream, ws);
    NEUVV_SHAPES(NEUVV_FWD_CASE)
#undef NEUVV_FWD_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_render_bwd(int K, int C, int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                             const BackwardIO& io, hipStream_t stream) {
    if (ra.n_slots <= 0) return hipSuccess;
#define NEUVV_BWD_CASE(k, c) \
    if (K == k && C == c) return launch_render_bwd_shape<k, c>(dtype, tr, in, ra, io, stream);
    NEUVV_SHAPES(NEUVV_BWD_CASE)
#undef NEUVV_BWD_CASE
    return hipErrorInvalidValue;
}

// The fixed scratch of neuvv_render_noalloc. Host code never uses the
// array's name as an address: fixed_scratch() looks its device address up
// once per device (with that device current) and the launches take that.
// Calls that overlap on one device share the array and race.
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};
}  // namespace

hipError_t fixed_scratch(void** p) {
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!q) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = q;
    }
    *p = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace neuvv
