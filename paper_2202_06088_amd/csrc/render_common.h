// Building blocks shared by the render kernels (render_kernels.h, render_pp.hip):
// payload gathers, work queues, cull passes and candidate lists, launch
// sizing. Device code for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include "launch.h"
#include "neuvv_device.h"

namespace neuvv {

constexpr int kBlock = 256;

// cells a lane's walk visits per iteration of the wavefront's loop: one step
// at a time, so that a lane with a sample to evaluate never waits for lanes
// crossing long empty stretches (those finish their stretch over several
// iterations instead)
constexpr int kWalkBudget = 1;

template <int DT>
struct StoreTraits;
template <>
struct StoreTraits<0> { static constexpr int V = 4; };
template <>
struct StoreTraits<1> { static constexpr int V = 8; };
template <>
struct StoreTraits<2> { static constexpr int V = 8; };

template <int DT>
__device__ __forceinline__ void unpack16(const uint4& v, float (&out)[StoreTraits<DT>::V]) {
    if constexpr (DT == 0) {
        out[0] = __uint_as_float(v.x);
        out[1] = __uint_as_float(v.y);
        out[2] = __uint_as_float(v.z);
        out[3] = __uint_as_float(v.w);
    } else {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint16_t lo = (uint16_t)(w[i] & 0xffffu), hi = (uint16_t)(w[i] >> 16);
            if constexpr (DT == 1) {
                out[2 * i] = (float)__builtin_bit_cast(_Float16, lo);
                out[2 * i + 1] = (float)__builtin_bit_cast(_Float16, hi);
            } else {
                out[2 * i] = __uint_as_float((uint32_t)lo << 16);
                out[2 * i + 1] = __uint_as_float((uint32_t)hi << 16);
            }
        }
    }
}

// Gathers R values of leaf `slot` from a [ceil(R/V)][N][V] array (layout 0) or
// a [N][ceil(R/V)][V] array (layout 1).
template <int DT, int R>
__device__ __forceinline__ void load_leaf(const void* base, int64_t N, int64_t slot, int layout,
                                          float (&out)[R]) {
    constexpr int V = StoreTraits<DT>::V;
    constexpr int NG = (R + V - 1) / V;
    const int64_t stride = layout ? 1 : N;
    const uint4* p = reinterpret_cast<const uint4*>(base) + (layout ? slot * NG : slot);
    uint4 raw[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) raw[g] = p[(int64_t)g * stride];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        float tmp[V];
        unpack16<DT>(raw[g], tmp);
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (g * V + e < R) out[g * V + e] = tmp[e];
    }
}

// Per-sample transcendentals on the hardware base-2 exponential, base-2
// logarithm and reciprocal (about 1 ulp each) instead of the correctly
// rounded library sequences, which cost several times the instructions.
// exp_hw: e^x = 2^(x log2 e); relative error 1 ulp plus |x| * 6e-8 from
// rounding the scaled argument (below 1e-6 for the |x| < 15 of colour
// logits and optical depths).
__device__ __forceinline__ float exp_hw(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ __forceinline__ float sigmoid_f(float x) { return __builtin_amdgcn_rcpf(1.0f + exp_hw(-x)); }
// log(1 + e), e in [0, 1]: the logarithm of the rounded u = 1 + e, scaled by
// e / (u - 1) to undo the rounding of u (a few ulp).
__device__ __forceinline__ float log1p_hw(float e) {
    const float u = 1.0f + e;
    const float lg = __builtin_amdgcn_logf(u) * 0.693147180559945309f;
    return u == 1.0f ? e : lg * (e * __builtin_amdgcn_rcpf(u - 1.0f));
}
__device__ __forceinline__ float softplus_f(float x) { return fmaxf(x, 0.0f) + log1p_hw(exp_hw(-fabsf(x))); }
// Density activation of Eq. 5 (relu = 0: softplus, the workloads' reading;
// relu != 0: ReLU as Eq. 5 prints it) and its derivative (0 at x <= 0 for ReLU).
// relu is a kernel argument, so the branch is uniform.
__device__ __forceinline__ float density_f(float x, int relu) { return relu ? fmaxf(x, 0.0f) : softplus_f(x); }
__device__ __forceinline__ float density_dx(float x, int relu) { return relu ? (x > 0.0f ? 1.0f : 0.0f) : sigmoid_f(x); }
// Opacity a = 1 - e^-od and transmittance factor e = e^-od of an optical
// depth od >= 0 (Eq. 8). Below od = 1/4 the series of 1 - e^-od to the
// seventh power (truncation below 2e-9 relative) keeps a accurate where
// 1 - e would cancel; above it a = 1 - e loses at most 3e-7 relative.
__device__ __forceinline__ void absorb(float od, float& a, float& e) {
    const float s = od * fmaf(od, fmaf(od, fmaf(od, fmaf(od, fmaf(od, fmaf(od, 1.0f / 5040.0f, -1.0f / 720.0f),
                                                                      1.0f / 120.0f), -1.0f / 24.0f), 1.0f / 6.0f),
                                         -0.5f), 1.0f);
    const float x = exp_hw(-od);
    const bool small = od < 0.25f;
    a = small ? s : 1.0f - x;
    e = small ? 1.0f - s : x;
}

__device__ __forceinline__ int lane_rank(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Dynamic chunk distribution: kQueues counters, 128 bytes apart, one per XCD.
// The chunk range [0, n_chunks) is cut into kQueues contiguous parts. In the
// candidate form a cull pass has listed the rays worth walking of part x in
// list[lo_x * 64 ...] (count[x] of them), and chunks are 64 consecutive
// entries of that list.
constexpr int kQueues = 8;
constexpr int kQueueStride = 16;

struct ChunkCursor {
    int home;       // this block's XCD
    int tried;      // queues drained so far (wave-uniform)
    int pos;        // slots of the current chunk handed out; 64 = take a new chunk
    int px0;        // x of the tile's first pixel (images)
    int len;        // candidate form: entries in the current chunk
    int64_t base;   // ray index of the chunk's first slot (candidate form: list index)
};

__device__ __forceinline__ ChunkCursor chunk_cursor() {
    ChunkCursor c;
    c.home = (int)(blockIdx.x & (kQueues - 1));
    c.tried = 0;
    c.pos = kWave;
    c.px0 = 0;
    c.len = 0;
    c.base = 0;
    return c;
}

// Moves the (converged) wavefront to its next chunk; false when every queue
// is drained. One lane takes the ticket; the result is wave-uniform.
__device__ __forceinline__ bool next_chunk(const RayArgs& ra, ChunkCursor& cc) {
    const int64_t n_chunks = (ra.n_slots + 63) >> 6;
    const int leader = __builtin_ctzll(__ballot(1));
    while (cc.tried < kQueues) {
        const int x = (cc.home + cc.tried) & (kQueues - 1);
        const int64_t lo = n_chunks * x / kQueues, hi = n_chunks * (x + 1) / kQueues;
        unsigned long long t = 0;
        if ((int)(threadIdx.x & 63) == leader) t = atomicAdd(ra.queue + x * kQueueStride, 1ull);
        const uint32_t t_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)t);
        const uint32_t t_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(t >> 32));
        const int64_t t64 = (int64_t)(((uint64_t)t_hi << 32) | t_lo);
        if (ra.list) {
            const int64_t cnt = (int64_t)ra.count[x * kQueueStride];
            if (t64 * 64 < cnt) {
                cc.pos = 0;
                cc.base = lo * 64 + t64 * 64;
                cc.len = cnt - t64 * 64 < 64 ? (int)(cnt - t64 * 64) : 64;
                return true;
            }
            ++cc.tried;
            continue;
        }
        const int64_t k = lo + t64;
        if (k < hi) {
            cc.pos = 0;
            if (ra.img_w > 0) {
                const int64_t ty = k / ra.tiles_x, tx = k - ty * ra.tiles_x;
                cc.px0 = (int)(tx * 8);
                cc.base = ty * 8 * (int64_t)ra.img_w + cc.px0;
            } else {
                cc.base = k * 64;
            }
            return true;
        }
        ++cc.tried;
    }
    return false;
}

// Ray index of slot `within` (0..63) of the current chunk, -1 for padding.
__device__ __forceinline__ int64_t chunk_ray(const RayArgs& ra, const ChunkCursor& cc, int within) {
    if (ra.list) return within < cc.len ? (int64_t)ra.list[cc.base + within] : -1;
    int64_t r;
    if (ra.img_w > 0) {
        if (cc.px0 + (within & 7) >= ra.img_w) return -1;
        r = cc.base + (int64_t)(within >> 3) * ra.img_w + (within & 7);
    } else {
        r = cc.base + within;
    }
    return r < ra.n ? r : -1;
}

// True when a candidate-form launch has no candidates at all (every block
// then leaves before staging anything; the same answer for every thread).
__device__ __forceinline__ bool no_candidates(const RayArgs& ra) {
    if (!ra.list) return false;
    unsigned long long total = 0;
#pragma unroll
    for (int x = 0; x < kQueues; ++x) total += ra.count[x * kQueueStride];
    return total == 0;
}

// 12-byte vector access to a ray's origin or direction, or a pixel's colour
// (one dwordx3 memory instruction instead of three).
typedef float f3v __attribute__((ext_vector_type(3)));
__device__ __forceinline__ f3v load3(const float* p) {
    f3v v;
    __builtin_memcpy(&v, p, 12);
    return v;
}
__device__ __forceinline__ void store3(float* p, float x, float y, float z) {
    const f3v v = {x, y, z};
    __builtin_memcpy(p, &v, 12);
}

__device__ __forceinline__ void write_miss(const RenderOut& out, int64_t ray) {
    if (out.rgb) store3(out.rgb + 3 * ray, 0.0f, 0.0f, 0.0f);
    if (out.alpha) out.alpha[ray] = 0.0f;
    if (out.depth) out.depth[ray] = INFINITY;
    if (out.nsamp) out.nsamp[ray] = 0;
    if (out.last_leaf) out.last_leaf[ray] = -1;
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <typename KernelT>
static int grid_for(KernelT kernel, const RayArgs& ra) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu <= 0)
        per_cu = 2;
    const int64_t chunks = (ra.n_slots + 63) / 64;
    const int64_t want = (chunks + (kBlock / kWave) - 1) / (kBlock / kWave);
    const int64_t cap = (int64_t)per_cu * device_cu_count();
    const int64_t g = want < cap ? want : cap;
    return (int)(g > 0 ? g : 1);
}

// Work-queue counters of one launch: 1 KiB of stream-ordered scratch, zeroed
// by a one-block kernel (no memset node, so the sequence may be captured in a
// graph) and freed after the render kernel in stream order. The candidate
// form adds kQueues counts (the second KiB) and a list of n_chunks * 64
// int32 ray indices.
static __global__ void zero_queue_kernel(unsigned long long* q) { q[threadIdx.x] = 0ull; }

// Cull pass of the candidate form: each wavefront tests kCullGroup chunks of
// one XCD part at a time (64 slots per chunk, one per lane), reserves room for
// the rays it keeps with one atomic on the part's count (atomics on one
// address serialise, so the groups are large), and lists them in slot order.
// MODE 0 (forward): keep the rays the plain-float box test cannot reject and
// write the miss outputs of the others. MODE 1 (adjoint): keep the rays whose
// forward composited a sample (the others carry no gradient); MODE 2 and 3
// (adjoint of a traced forward): of those, the rays without a trace (head
// < 0, none when out.trace's counters show that every request for trace
// room was met) and the rays with one. MODE 4: keep the rays hit.keep(ray) accepts
// and write the miss outputs of the others (no ray loads). The
// pass is bound by the 24 bytes of ray per slot it reads; at high occupancy
// it runs near HBM bandwidth, where the render kernel's refill rounds would
// take one memory latency per round for every ray. Launches of fewer than
// kCullSmall chunks that are not images use groups of kCullGroupSmall chunks,
// so that they still spread over many wavefronts (each group is a chain of
// dependent loads).
constexpr int kCullGroup = 32;
constexpr int kCullGroupSmall = 4;
constexpr int64_t kCullSmall = 16384;

// Coarse test of one placed tree (the forward's cull).
template <bool IDENT>
struct TreeHit {
    TreeArgs tr;
    InstArgs in;
    __device__ __forceinline__ bool operator()(const float o[3], const float d[3]) const {
        return ray_may_hit<IDENT>(tr, in, o, d);
    }
};

template <int MODE, class Hit, int GROUP = kCullGroup>
static __global__ __launch_bounds__(kBlock) void cull_kernel(Hit hit, RayArgs ra, RenderOut out,
                                                              const int32_t* nsamp, const int32_t* head,
                                                              int32_t* list,
                                                              unsigned long long* count) {
    if constexpr (MODE == 2) {
        // After a traced forward, out.trace holds its allocation counters and the
        // room in samples. A trace is incomplete only where a block request of its
        // XCD part went past the part's end; with none, no ray walks.
        if (out.trace.counter) {
            bool over = false;
#pragma unroll
            for (int p = 0; p < kQueues; ++p) {
                const int64_t part = out.trace.cap * (p + 1) / kQueues - out.trace.cap * p / kQueues;
                over = over || (int64_t)out.trace.counter[p * kQueueStride] > part;
            }
            if (!over) return;
        }
    }
    const int lane = threadIdx.x & 63;
    const int x = (int)(blockIdx.x & (kQueues - 1));
    const int64_t n_chunks = (ra.n_slots + 63) >> 6;
    const int64_t lo = n_chunks * x / kQueues, hi = n_chunks * (x + 1) / kQueues;
    const int64_t nw = (int64_t)(gridDim.x / kQueues) * (kBlock / kWave);
    const int64_t wi = (int64_t)(blockIdx.x / kQueues) * (kBlock / kWave) + (threadIdx.x >> 6);
    if (ra.img_w > 0) {
        // Images: a wavefront takes a segment of up to 8 horizontally adjacent
        // tiles and walks its 8 pixel rows, one row of 64 pixels per pass, so
        // its ray loads and miss stores are contiguous; the rays kept are then
        // listed tile by tile in slot order from the per-row ballots.
        if (hi <= lo) return;
        const int64_t tiles_x = ra.tiles_x;
        const int64_t ty_lo = lo / tiles_x, ty_hi = (hi - 1) / tiles_x;
        const int64_t nseg = (tiles_x + 7) / 8;
        const int64_t n_seg = (ty_hi - ty_lo + 1) * nseg;
        const int jt = lane >> 3;   // tile of the lane within the segment
        for (int64_t sg = wi; sg < n_seg; sg += nw) {
            const int64_t ty = ty_lo + sg / nseg, j = sg - (sg / nseg) * nseg;
            const int64_t row0 = ty * tiles_x;
            int64_t kx0 = 8 * j, kx1 = 8 * j + 8 < tiles_x ? 8 * j + 8 : tiles_x;
            if (kx0 < lo - row0) kx0 = lo - row0;
            if (kx1 > hi - row0) kx1 = hi - row0;
            if (kx0 >= kx1) continue;   // wave-uniform
            const int64_t tx = 8 * j + jt;
            const int64_t px = 8 * tx + (lane & 7);
            const bool lane_ok = tx >= kx0 && tx < kx1 && px < ra.img_w;
            uint64_t keep[8];
            int total = 0;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int64_t ray = (8 * ty + r) * ra.img_w + px;
                bool k = false;
                if (lane_ok && ray < ra.n) {
                    if constexpr (MODE == 0) {
                        const f3v ov = load3(ra.o + 3 * ray), dv = load3(ra.d + 3 * ray);
                        const float o[3] = {ov.x, ov.y, ov.z};
                        const float d[3] = {dv.x, dv.y, dv.z};
                        k = hit(o, d);
                        if (!k) write_miss(out, ray);
                    } else if constexpr (MODE == 4) {
                        k = hit.keep(ray);
                        if (!k) write_miss(out, ray);
                    } else {
                        k = nsamp[ray] > 0;
                        if constexpr (MODE == 2) k = k && head[ray] < 0;
                        if constexpr (MODE == 3) k = k && head[ray] >= 0;
                    }
                }
                keep[r] = __ballot(k);
                total += __popcll(keep[r]);
            }
            if (total == 0) continue;   // wave-uniform
            unsigned long long b = 0;
            if (lane == 0) b = atomicAdd(count + x * kQueueStride, (unsigned long long)total);
            const uint32_t b_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
            const uint32_t b_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
            const int64_t at = lo * 64 + (int64_t)(((uint64_t)b_hi << 32) | b_lo);
            // this lane's tile: its kept-slot mask (bit 8r + column) and the rays
            // kept in the segment's earlier tiles
            uint64_t tm = 0ull;
            int before = 0;
            const uint64_t below = jt ? (~0ull >> (64 - 8 * jt)) : 0ull;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                tm |= ((keep[r] >> (8 * jt)) & 0xffull) << (8 * r);
                before += __popcll(keep[r] & below);
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if ((keep[r] >> lane) & 1ull) {
                    const int within = 8 * r + (lane & 7);
                    const int64_t ray = (8 * ty + r) * ra.img_w + px;
                    list[at + before + __popcll(tm & ((1ull << within) - 1ull))] = (int32_t)ray;
                }
            }
        }
        return;
    }
    for (int64_t c0 = lo + wi * GROUP; c0 < hi; c0 += nw * GROUP) {
        uint64_t keep[GROUP];
        int32_t rays[GROUP];
        int total = 0;
#pragma unroll
        for (int j = 0; j < GROUP; ++j) {
            const int64_t c = c0 + j;
            const int64_t ray = c < hi ? slot_to_ray(ra, c * 64 + lane) : -1;
            bool k = false;
            if (ray >= 0) {
                if constexpr (MODE == 0) {
                    const f3v ov = load3(ra.o + 3 * ray), dv = load3(ra.d + 3 * ray);
                    const float o[3] = {ov.x, ov.y, ov.z};
                    const float d[3] = {dv.x, dv.y, dv.z};
                    k = hit(o, d);
                    if (!k) write_miss(out, ray);
                } else if constexpr (MODE == 4) {
                    k = hit.keep(ray);
                    if (!k) write_miss(out, ray);
                } else {
                    k = nsamp[ray] > 0;
                    if constexpr (MODE == 2) k = k && head[ray] < 0;
                    if constexpr (MODE == 3) k = k && head[ray] >= 0;
                }
            }
            keep[j] = __ballot(k);
            rays[j] = (int32_t)ray;
            total += __popcll(keep[j]);
        }
        if (total == 0) continue;   // wave-uniform
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd(count + x * kQueueStride, (unsigned long long)total);
        const uint32_t b_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
        const uint32_t b_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
        int64_t at = lo * 64 + (int64_t)(((uint64_t)b_hi << 32) | b_lo);
#pragma unroll
        for (int j = 0; j < GROUP; ++j) {
            if ((keep[j] >> lane) & 1ull) list[at + lane_rank(keep[j])] = rays[j];
            at += __popcll(keep[j]);
        }
    }
}

template <int MODE, class Hit>
static hipError_t launch_cull_hit(const Hit& hit, const RayArgs& ra, const RenderOut& out, const int32_t* nsamp,
                                  const int32_t* head, int32_t* list, unsigned long long* count, hipStream_t st) {
    const int64_t n_chunks = (ra.n_slots + 63) >> 6;
    const bool small = ra.img_w <= 0 && n_chunks < kCullSmall;
    const int group = small ? kCullGroupSmall : kCullGroup;
    const int64_t groups = (n_chunks / kQueues + 1 + group - 1) / group;   // per part, at most
    int64_t blocks = (groups + (kBlock / kWave) - 1) / (kBlock / kWave);
    const int64_t cap = (int64_t)device_cu_count() * 2;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    const dim3 grid((unsigned)(blocks * kQueues));
    if (small)
        hipLaunchKernelGGL((cull_kernel<MODE, Hit, kCullGroupSmall>), grid, dim3(kBlock), 0, st, hit, ra, out, nsamp,
                           head, list, count);
    else
        hipLaunchKernelGGL((cull_kernel<MODE, Hit>), grid, dim3(kBlock), 0, st, hit, ra, out, nsamp, head, list, count);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_cull(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, const RenderOut& out,
                              const int32_t* nsamp, const int32_t* head, int32_t* list, unsigned long long* count,
                              hipStream_t st) {
    if (in.identity) return launch_cull_hit<MODE>(TreeHit<true>{tr, in}, ra, out, nsamp, head, list, count, st);
    return launch_cull_hit<MODE>(TreeHit<false>{tr, in}, ra, out, nsamp, head, list, count, st);
}

// Runs launch(ra) with the launch's queue counters set; rays are the slots.
// ws: caller-provided scratch of at least list_scratch_bytes(n_slots) bytes
// (nothing is allocated), or nullptr to take it from the pool.
template <typename Launch>
static hipError_t with_queue(const RayArgs& ra_in, hipStream_t st, Launch&& launch, void* ws = nullptr) {
    RayArgs ra = ra_in;
    void* q = ws;
    hipError_t e = ws ? hipSuccess : work_alloc(&q, kQueues * kQueueStride * sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    ra.queue = static_cast<unsigned long long*>(q);
    hipLaunchKernelGGL(zero_queue_kernel, dim3(1), dim3(kQueues * kQueueStride), 0, st, ra.queue);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch(ra);
    const hipError_t f = ws ? hipSuccess : work_free(q, st);
    return e != hipSuccess ? e : f;
}

static_assert(2 * kQueues * kQueueStride * sizeof(unsigned long long) == kListHeaderBytes,
              "candidate-list header size");

// Candidate form: cull(list, count) lists the rays, then launch(ra) runs over
// them. Ray indices must fit int32; larger launches take the slot form (the
// render kernels then test every ray themselves). ws as in with_queue.
template <typename Cull, typename Launch>
static hipError_t with_list(const RayArgs& ra_in, hipStream_t st, Cull&& cull, Launch&& launch,
                            void* ws = nullptr) {
    if (ra_in.n > (int64_t)INT32_MAX) return with_queue(ra_in, st, launch, ws);
    const size_t qbytes = kListHeaderBytes;
    RayArgs ra = ra_in;
    void* q = ws;
    hipError_t e = ws ? hipSuccess : work_alloc(&q, list_scratch_bytes(ra_in.n_slots), st);
    if (e != hipSuccess) return e;
    ra.queue = static_cast<unsigned long long*>(q);
    unsigned long long* count = ra.queue + kQueues * kQueueStride;
    int32_t* list = reinterpret_cast<int32_t*>(static_cast<char*>(q) + qbytes);
    ra.count = count;
    ra.list = list;
    hipLaunchKernelGGL(zero_queue_kernel, dim3(1), dim3(2 * kQueues * kQueueStride), 0, st, ra.queue);
    e = hipGetLastError();
    if (e == hipSuccess) e = cull(list, count);
    if (e == hipSuccess) e = launch(ra);
    const hipError_t f = ws ? hipSuccess : work_free(q, st);
    return e != hipSuccess ? e : f;
}

// Candidate form with the cull pass of one placed tree (MODE as in cull_kernel).
template <int MODE, typename Launch>
static hipError_t with_candidates(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra_in,
                                  const RenderOut& out, const int32_t* nsamp, hipStream_t st, Launch&& launch,
                                  const int32_t* head = nullptr, void* ws = nullptr) {
    return with_list(
        ra_in, st,
        [&](int32_t* list, unsigned long long* count) {
            return launch_cull<MODE>(tr, in, ra_in, out, nsamp, head, list, count, st);
        },
        launch, ws);
}

// ----------------------------------------------------------------------------
// records of the two-phase adjoint (see RecordArgs)

// records a wavefront takes from its XCD's counter at a time
constexpr int kRecBlock = 2048;
// LDS rows per wavefront for the transposition of finished leaf rows
constexpr int kFlushSlots = 16;

static __global__ void record_init_kernel(int32_t* head, int64_t n, unsigned long long* counter,
                                          unsigned long long* leaf_cursor) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) head[i] = -1;
    if (i < kQueues) counter[i * kQueueStride] = 0ull;
    if (i == 0) *leaf_cursor = 0ull;
}

// Wave-uniform allocation of n (<= kRecBlock) consecutive items from blocks of
// kRecBlock taken from one counter per XCD; XCD x owns items
// [cap x / kQueues, cap (x + 1) / kQueues). [cur, end) is what is left of the
// wavefront's current block. Returns the first item, or -1 when the XCD's
// part is exhausted. Call with every lane of the wavefront active.
__device__ __forceinline__ int take_items(unsigned long long* counter, int64_t cap, int home, int n, int& cur,
                                          int& end) {
    if (cur + n > end) {
        const int64_t lo = cap * home / kQueues, hi = cap * (home + 1) / kQueues;
        unsigned long long b = 0;
        if ((threadIdx.x & 63) == 0) b = atomicAdd(counter + home * kQueueStride, (unsigned long long)kRecBlock);
        const uint32_t b_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
        const uint32_t b_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
        const int64_t first = lo + (int64_t)(((uint64_t)b_hi << 32) | b_lo);
        // the room is below 2^31 items, so the block's bounds fit int32 once clamped to the part
        cur = (int)(first < hi ? first : hi);
        end = (int)(first + kRecBlock <= hi ? first + kRecBlock : hi);
    }
    if (cur + n > end) return -1;
    const int at = cur;
    cur += n;
    return at;
}

// Linking one iteration's records into their leaves' lists. The records of
// the lanes with a sample (mask hm) are consecutive in lane order. A run is a
// maximal sequence of such lanes, consecutive in that order, on one leaf: its
// first lane links the whole run with one atomic exchange of the leaf's head
// (the head becomes the run's last record, and the first record links to the
// old head), and every other lane links its record to the record before it.
// count: the run's length for its first lane, 0 for the others. Call with
// every lane of the wavefront active.
struct RecordRun {
    int count;
};
__device__ __forceinline__ RecordRun record_run(uint64_t hm, bool has, int leaf) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const uint64_t hb = hm & below;
    const int pred = hb ? 63 - __builtin_clzll(hb) : lane;   // the previous lane with a sample
    const int pleaf = __builtin_amdgcn_ds_bpermute(pred << 2, leaf);
    const bool start = has && (hb == 0ull || pleaf != leaf);
    const uint64_t starts = __ballot(start);
    RecordRun r{0};
    if (start) {
        const uint64_t later = starts & ~((2ull << lane) - 1ull);   // starts above this lane (none: lane 63)
        const uint64_t upto = later ? (1ull << __builtin_ctzll(later)) - 1ull : ~0ull;
        r.count = __popcll(hm & upto & ~below);
    }
    return r;
}

// Hands leaves with records to the idle lanes of a reduction wavefront.
// Wavefront w takes 64-leaf batches w, w + W, ...; a batch's heads are read in
// one load (lane = leaf) and its leaves with records are compacted into a
// per-wavefront LDS queue of {leaf, first record}, from which idle lanes take
// entries in lane order.
struct LeafFeeder {
    int64_t batch;     // next batch of this wavefront
    int64_t n_waves;
    int cnt, pos;      // wave-uniform: queue entries, entries handed out
    bool more;         // wave-uniform: batches may be left
};

__device__ __forceinline__ LeafFeeder leaf_feeder(int wave_in_block) {
    LeafFeeder f;
    f.batch = (int64_t)blockIdx.x * (kBlock / kWave) + wave_in_block;
    f.n_waves = (int64_t)gridDim.x * (kBlock / kWave);
    f.cnt = f.pos = 0;
    f.more = true;
    return f;
}

// Gives idle lanes (leaf < 0) a leaf and its first record while leaves are left.
// q: this wavefront's LDS queue of kWave entries. Call with every lane active.
__device__ __forceinline__ void feed_leaves(LeafFeeder& f, const RecordArgs& rec, int64_t n_leaves, int2* q,
                                            int& leaf, int& first) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        const uint64_t idle = __ballot(leaf < 0);
        if (!idle || !f.more) break;
        if (f.pos >= f.cnt) {
            const int64_t b0 = f.batch * kWave;
            f.batch += f.n_waves;
            if (b0 >= n_leaves) {
                f.more = false;
                break;
            }
            const int64_t L = b0 + lane;
            const int h = L < n_leaves ? rec.head[L] : -1;
            const uint64_t m = __ballot(h >= 0);
            __builtin_amdgcn_wave_barrier();
            if (h >= 0) q[lane_rank(m)] = make_int2((int)L, h);
            __builtin_amdgcn_wave_barrier();
            f.cnt = __popcll(m);
            f.pos = 0;
            continue;
        }
        const int avail = f.cnt - f.pos, n_idle = __popcll(idle);
        if (leaf < 0) {
            const int r = lane_rank(idle);
            if (r < avail) {
                const int2 e = q[f.pos + r];
                leaf = e.x;
                first = e.y;
            }
        }
        f.pos += n_idle < avail ? n_idle : avail;
    }
}

// Takes the record scratch of one adjoint launch (cap > 0) from the pool and
// queues its initialisation: kQueues counters 128 bytes apart and a leaf
// cursor, the leaf heads (-1) and room for cap records of 32 bytes. With
// cap == 0 rec stays empty (per-sample atomics only).
static hipError_t records_begin(const TreeArgs& tr, int64_t cap, hipStream_t st, RecordArgs& rec, void*& mem) {
    rec = RecordArgs{};
    mem = nullptr;
    if (cap <= 0) return hipSuccess;
    const size_t head_b = ((size_t)tr.n_leaves * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t rec_b = (size_t)cap * 2 * sizeof(int4);
    constexpr size_t hdr = 2048;
    hipError_t e = work_alloc(&mem, hdr + head_b + rec_b, st);
    if (e != hipSuccess) return e;
    char* p = static_cast<char*>(mem);
    rec.counter = reinterpret_cast<unsigned long long*>(p);
    rec.leaf_cursor = reinterpret_cast<unsigned long long*>(p + 1024);
    rec.head = reinterpret_cast<int32_t*>(p + hdr);
    rec.rec = reinterpret_cast<int4*>(p + hdr + head_b);
    rec.cap = cap;
    hipLaunchKernelGGL(record_init_kernel, dim3((unsigned)((tr.n_leaves + 255) / 256)), dim3(256), 0, st, rec.head,
                       tr.n_leaves, rec.counter, rec.leaf_cursor);
    return hipGetLastError();
}

}  // namespace neuvv
