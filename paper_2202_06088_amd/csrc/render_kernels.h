// VOctree volume rendering on gfx950: forward (Sec. 4.3 "Rendering", Eq. 4,
// 5, 8, 9) and adjoint (Sec. 4.3 "Optimization").
//
// Work distribution: persistent wavefronts fed from work queues. Rays are
// grouped in chunks of 64 work slots (an 8x8 pixel tile when the rays form an
// image). The chunk range is cut into one contiguous part per XCD (hardware
// places block b on XCD b % 8), so that neighbouring tiles, which hit the
// same leaves, share an L2; each part has an atomic counter. A wavefront
// takes chunks one at a time from its own XCD's counter, then from the other
// parts in turn once its own is drained, so no wavefront idles while work is
// left anywhere (the cost of a tile varies by orders of magnitude between
// sky and subject). A lane whose ray has finished is refilled from the
// current chunk: the wavefront takes a ballot of the idle lanes, hands the
// next slots to them in lane order with mbcnt, and advances its
// (wave-uniform) cursor by the popcount.
//
// Per lane: each iteration of the wavefront's loop advances the walk by one
// cell (the current brick's node in registers; entering another 4^3 region,
// its directory entry and brick row from L2/HBM); a lane whose cell is an
// occupied leaf gathers the
// leaf's payload (one contiguous row per leaf, or 16-byte-vector
// structure-of-arrays) in 16-byte loads, evaluates colour and density in
// float32 and composites. The per-sample HH contraction is a 3xK times K
// matrix-vector product with a different matrix per sample, so it stays on
// the vector ALUs; the kernel is bound by memory traffic and latency.
//
// The kernels and their host launchers are templates over the leaf shape
// (K HH functions per channel, C density weights); render_k*.hip instantiate
// the compiled shapes.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include <type_traits>

#include "launch.h"
#include "neuvv_device.h"
#include "render_common.h"

namespace neuvv {

// At least this many wavefronts per SIMD for the kernels of shape (K, C)
// (the compiler then keeps their registers within the budget): want for the
// K = 16, C = 8 leaf, one (no constraint) for the larger leaves.
template <int K, int C>
__host__ __device__ constexpr int min_waves(int want) { return 3 * K + C <= 56 ? want : 1; }


template <int K, int C>
__device__ __forceinline__ void ray_basis(const TreeArgs& tr, const RaySetup& rs, float (&h)[K], float (&b)[C]) {
    float hall[30];
    const float gam = (1.0f - rs.f) * tr.gamma[rs.i0] + rs.f * tr.gamma[rs.i1];
    hh_all(rs.dir[0], rs.dir[1], rs.dir[2], gam, hall);
#pragma unroll
    for (int k = 0; k < K; ++k) h[k] = hall[k];
    const float* b0 = tr.basis + (int64_t)rs.i0 * C;
    const float* b1 = tr.basis + (int64_t)rs.i1 * C;
#pragma unroll
    for (int c = 0; c < C; ++c) b[c] = (1.0f - rs.f) * b0[c] + rs.f * b1[c];
}

// ----------------------------------------------------------------------------
// forward


// EDIT: the tree carries appearance edits (Sec. 5.2): from its first frame on,
// an edited leaf's target colour (and target density, when >= 0) replace the
// evaluated ones.
// TRACE: every sample is also written to out.trace (its leaf, segment length,
// density logit and colours, linked in ray order), so that the adjoint of the
// same call replays the samples instead of walking and evaluating again. The
// samples of one iteration take consecutive entries in lane order, from
// blocks per wavefront; a ray whose samples do not all fit gets head -1.
// A sample's entry is stored one sample later, when the slot it links to is
// known, right after that sample's payload loads: vector-memory counters
// retire in issue order, so stores issued before a load would make every wait
// on that load (the walk's node reads, the payload) wait for them too. The
// ray's last entry is stored when it finishes. The store is unconditional for
// every lane with a sample: a ray's first sample stores a placeholder into
// its own slot (which the same lane overwrites later), and a ray whose trace
// is incomplete stores into its last slot, or, if it has none, into the spare
// half of the trace header.
template <int K, int C, int DT, bool IDENT, bool EDIT, bool TRACE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(min_waves<K, C>(3), 8))) void render_fwd_kernel(
    TreeArgs tr, InstArgs in, RayArgs ra, float t_stop, RenderOut out) {
    if (no_candidates(ra)) return;
    __shared__ float s_h[kBlock * K];
    __shared__ float s_b[kBlock * C];
    // traced: the output addresses, needed once per ray, wait in LDS rather than in scalar
    // registers, which the trace's allocation takes
    __shared__ RenderOut s_out;
    if constexpr (TRACE) {
        if (threadIdx.x == 0) s_out = out;
        __syncthreads();
    }
    const RenderOut& fo = TRACE ? s_out : out;
    ChunkCursor cc = chunk_cursor();
    bool more = true;   // wave-uniform: chunks may be left

    bool alive = false;
    int64_t ray = -1;
    RaySetup rs;
    Walk w;
    // the ray's basis h and density row b live in LDS (this lane's columns)
    float* const hl = s_h + threadIdx.x * K;
    float* const bl = s_b + threadIdx.x * C;
    float Tr = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f, wsum = 0.0f, dsum = 0.0f;
    int ns = 0, last = -1;
    int t_first = -1;                // trace: the ray's first entry; -2: broken
    // trace: the previous sample, written once the slot of the next is known
    int pslot = -1, pleaf = 0;
    float pdelta = 0.0f, px = 0.0f, pc0 = 0.0f, pc1 = 0.0f, pc2 = 0.0f;
    int tcur = 0, tend = 0;      // trace: what is left of the wavefront's block (wave-uniform)

    for (;;) {
        const uint64_t idle = __ballot(!alive);
        const int n_idle = __popcll(idle);
        if (more && (n_idle >= ra.refill_min || n_idle == kWave)) {
            // Acquisition: idle lanes take the next slots; rays the plain-float
            // test rejects get their miss outputs at once and the lane takes
            // another slot, while at least refill_min lanes are idle. Then the
            // compensated setup runs once for all accepted rays together.
            bool cand = false;
            float o[3], d[3], t = 0.0f;
            for (;;) {
                const uint64_t need = __ballot(!alive && !cand);
                const int n_need = __popcll(need);
                if (n_need < ra.refill_min) break;
                if (cc.pos == kWave && !next_chunk(ra, cc)) {
                    more = false;
                    break;
                }
                const int take = n_need < kWave - cc.pos ? n_need : kWave - cc.pos;
                if (!alive && !cand) {
                    const int r = lane_rank(need);
                    if (r < take) {
                        ray = chunk_ray(ra, cc, cc.pos + r);
                        if (ray >= 0) {
                            o[0] = ra.o[3 * ray]; o[1] = ra.o[3 * ray + 1]; o[2] = ra.o[3 * ray + 2];
                            d[0] = ra.d[3 * ray]; d[1] = ra.d[3 * ray + 1]; d[2] = ra.d[3 * ray + 2];
                            t = ra.t ? ra.t[ray] : ra.t_scalar;
                            cand = ra.list != nullptr || ray_may_hit<IDENT>(tr, in, o, d);
                            if (!cand) write_miss(out, ray);
                        }
                    }
                }
                cc.pos += take;
            }
            if (cand) {
                ray_setup<IDENT>(tr, in, o, d, t, rs);
                Tr = 1.0f; acc0 = acc1 = acc2 = 0.0f; wsum = dsum = 0.0f; ns = 0;
                if (rs.hit) {
                    {
                        float h[K], bv[C];
                        ray_basis<K, C>(tr, rs, h, bv);
#pragma unroll
                        for (int k = 0; k < K; ++k) hl[k] = h[k];
#pragma unroll
                        for (int c = 0; c < C; ++c) bl[c] = bv[c];
                    }
                    walk_begin(tr, rs, w);
                    alive = true;
                    t_first = -1;
                    pslot = -1;
                } else {
                    write_miss(out, ray);
                }
            }
            continue;
        }
        if (n_idle == kWave) break;
        bool finish = false, stopped = false;
        int leaf = -1;
        float delta = 0.0f, umid = 0.0f;
        if (alive) {
            leaf = walk_next<kWalkBudget>(tr, rs, w, delta, umid);
            finish = leaf == -1;
        }
        int cur = -1;
        if constexpr (TRACE) {
            const uint64_t hm = __ballot(leaf >= 0);
            const int n_s = __popcll(hm);
            const int at = n_s > 0 ? take_items(out.trace.counter, out.trace.cap, cc.home, n_s, tcur, tend) : -1;
            if (leaf >= 0) {
                if (at >= 0 && t_first != -2) {
                    cur = (int)(at + lane_rank(hm));
                    if (t_first == -1) t_first = cur;
                } else {
                    t_first = -2;   // incomplete: the adjoint walks this ray
                }
            }
        }
        if (leaf >= 0) {
            {
                float wv[3 * K], sv[C];
                load_leaf<DT, 3 * K>(tr.hh, tr.n_leaves, leaf, tr.layout, wv);
                load_leaf<DT, C>(tr.wsig, tr.n_leaves, leaf, tr.layout, sv);
                if constexpr (TRACE) {
                    // the previous sample's entry, linked to this one
                    const int tgt = pslot >= 0 ? pslot : cur;
                    int4* dst = tgt >= 0 ? out.trace.smp + 2 * (int64_t)tgt
                                         : reinterpret_cast<int4*>(reinterpret_cast<char*>(out.trace.counter) + 1024) +
                                               2 * (threadIdx.x & 31);
                    dst[0] = make_int4(pleaf, __float_as_int(pdelta), __float_as_int(px), __float_as_int(pc0));
                    dst[1] = make_int4(__float_as_int(pc1), __float_as_int(pc2), cur, 0);
                }
                float x = 0.0f;
#pragma unroll
                for (int c = 0; c < C; ++c) x = fmaf(sv[c], bl[c], x);
                float z0 = 0.0f, z1 = 0.0f, z2 = 0.0f;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float hk = hl[k];
                    z0 = fmaf(wv[k], hk, z0);
                    z1 = fmaf(wv[K + k], hk, z1);
                    z2 = fmaf(wv[2 * K + k], hk, z2);
                }
                float sig = density_f(x, tr.relu);
                float c0 = sigmoid_f(z0), c1 = sigmoid_f(z1), c2 = sigmoid_f(z2);
                if constexpr (EDIT) {
                    const float4 e0 = tr.edit[2 * (int64_t)leaf], e1 = tr.edit[2 * (int64_t)leaf + 1];
                    if (rs.tau >= e1.x) {
                        c0 = e0.x; c1 = e0.y; c2 = e0.z;
                        if (e0.w >= 0.0f) sig = e0.w;
                    }
                }
                const float od = sig * delta;
                float a, e_od;
                absorb(od, a, e_od);
                const float wt = Tr * a;
                acc0 = fmaf(wt, c0, acc0);
                acc1 = fmaf(wt, c1, acc1);
                acc2 = fmaf(wt, c2, acc2);
                wsum += wt;
                dsum = fmaf(wt, umid * rs.len_world, dsum);
                Tr *= e_od;
                ++ns;
                last = leaf;
                finish = t_stop > 0.0f && Tr < t_stop;
                stopped = finish;
                if constexpr (TRACE) {
                    if (cur >= 0) pslot = cur;
                    pleaf = leaf; pdelta = delta; px = x; pc0 = c0; pc1 = c1; pc2 = c2;
                }
            }
        }
        if (alive && finish) {
            if (fo.rgb) store3(fo.rgb + 3 * ray, acc0, acc1, acc2);
            if (fo.alpha) fo.alpha[ray] = 1.0f - Tr;
            if (fo.depth) fo.depth[ray] = wsum > 0.0f ? dsum / wsum : INFINITY;
            if (fo.nsamp) fo.nsamp[ray] = ns;
            if (fo.last_leaf) fo.last_leaf[ray] = stopped ? last : -1;
            if constexpr (TRACE) {
                if (t_first >= 0) {
                    out.trace.smp[2 * (int64_t)pslot] =
                        make_int4(pleaf, __float_as_int(pdelta), __float_as_int(px), __float_as_int(pc0));
                    out.trace.smp[2 * (int64_t)pslot + 1] = make_int4(__float_as_int(pc1), __float_as_int(pc2), -1, 0);
                }
                fo.trace.head[ray] = t_first >= 0 ? t_first : -1;
            }
            alive = false;
        }
    }
}

// ----------------------------------------------------------------------------
// adjoint
//
// Two phases. Here each ray replays its samples and writes, per sample, a
// 32-byte record of its gradients with respect to the colour logits and the
// density logit, linked into the list of its leaf; reduce_records_kernel
// below then sums every leaf's list and adds the leaf's row once. Records
// are taken in blocks per wavefront and written at consecutive indices, so
// the record stores of a wavefront are contiguous, and lanes next to each
// other on one leaf link their records with one atomic exchange (record_run).
//
// Samples without a record (the room is full, or records are off) take the
// per-sample scatter: a sample's 3K + C gradient values form one row of the
// leaf-major gradient array, and the whole wavefront adds that row with one
// atomic instruction (lane c = component c). An atomic whose lanes fall in
// one 256-byte row is handled as a couple of line operations, where one
// whose lanes hit 64 different leaves costs 64; the per-ray basis h and
// density row b every lane needs for this are kept in LDS.

template <int K, int C>
__host__ __device__ constexpr int grad_row() { return ((3 * K + C + 63) / 64) * 64; }



// REPLAY: every ray of the launch has a trace in io.trace (the forward's
// samples) and replays it (segment length, density logit and colours)
// without walking the tree or reading the HH coefficients; otherwise the
// rays walk.
template <int K, int C, int DT, bool IDENT, bool REPLAY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(min_waves<K, C>(REPLAY ? 4 : 3), 8))) void render_bwd_kernel(
    TreeArgs tr, InstArgs in, RayArgs ra, BackwardIO io, RecordArgs rec) {
    if (no_candidates(ra)) return;
    constexpr int ROW = grad_row<K, C>();
    __shared__ float s_h[kBlock * K];
    __shared__ float s_b[kBlock * C];
    __shared__ float s_gb[C];
    if (threadIdx.x < C) s_gb[threadIdx.x] = 0.0f;
    __syncthreads();
    ChunkCursor cc = chunk_cursor();
    bool more = true;   // wave-uniform: chunks may be left
    const int64_t N = tr.n_leaves;
    const bool per_ray_t = ra.t != nullptr;
    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x - lane;
    // one time for every ray and records: the basis gradient of recorded samples
    // is summed per leaf by the reduction (sum gx times w^sigma), not here
    const bool basis_late = rec.head != nullptr && !per_ray_t;
    const bool basis_here = io.grad_basis != nullptr && !basis_late;

    bool alive = false;
    int64_t ray = -1;
    RaySetup rs;
    Walk w;
    // basis-row gradient: per ray when rays carry their own time, else one running
    // sum over all rays of the lane (they share the frames and the weight f)
    float gb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) gb[c] = 0.0f;
    float Tr = 1.0f, Tfin = 0.0f, p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, F0 = 0.0f, F1 = 0.0f, F2 = 0.0f;
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, ga = 0.0f;
    int ns = 0, ns_fwd = 0;
    int tnext = -1;        // replay: the ray's next sample
    float dw0 = 0.0f, dw1 = 0.0f, dw2 = 0.0f;   // the ray's direction (world), for its records
    // records: the wavefront fills blocks of kRecBlock consecutive records,
    // taken from its XCD's part of the room; [wrec, wend) is what is left of
    // the current block (wave-uniform)
    int wrec = 0, wend = 0;

    for (;;) {
        const uint64_t idle = __ballot(!alive);
        const int n_idle = __popcll(idle);
        if (more && (n_idle >= ra.refill_min || n_idle == kWave)) {
            // Acquisition: idle lanes take the next slots while at least refill_min
            // lanes are idle; rays that composited no sample carry no gradient and
            // are passed over. The setup then runs once for all taken rays together.
            bool cand = false;
            for (;;) {
                const uint64_t need = __ballot(!alive && !cand);
                const int n_need = __popcll(need);
                if (n_need < ra.refill_min) break;
                if (cc.pos == kWave && !next_chunk(ra, cc)) {
                    more = false;
                    break;
                }
                const int take = n_need < kWave - cc.pos ? n_need : kWave - cc.pos;
                if (!alive && !cand) {
                    const int r = lane_rank(need);
                    if (r < take) {
                        ray = chunk_ray(ra, cc, cc.pos + r);
                        cand = ray >= 0 && (ra.list != nullptr || io.nsamp[ray] > 0);
                    }
                }
                cc.pos += take;
            }
            if (cand) {
                const float o[3] = {ra.o[3 * ray], ra.o[3 * ray + 1], ra.o[3 * ray + 2]};
                const float d[3] = {ra.d[3 * ray], ra.d[3 * ray + 1], ra.d[3 * ray + 2]};
                const float t = per_ray_t ? ra.t[ray] : ra.t_scalar;
                ray_setup<IDENT>(tr, in, o, d, t, rs);
                dw0 = d[0];
                dw1 = d[1];
                dw2 = d[2];
                if (rs.hit) {
                    {
                        float h[K], bv[C];
                        ray_basis<K, C>(tr, rs, h, bv);
#pragma unroll
                        for (int k = 0; k < K; ++k) s_h[threadIdx.x * K + k] = h[k];
#pragma unroll
                        for (int c = 0; c < C; ++c) s_b[threadIdx.x * C + c] = bv[c];
                    }
                    if constexpr (REPLAY) tnext = io.trace.head[ray];
                    else walk_begin(tr, rs, w);
                    ns_fwd = io.nsamp[ray];
                    ns = 0;
                    Tr = 1.0f;
                    Tfin = 1.0f - io.alpha[ray];
                    F0 = io.rgb[3 * ray]; F1 = io.rgb[3 * ray + 1]; F2 = io.rgb[3 * ray + 2];
                    g0 = io.grad_rgb[3 * ray]; g1 = io.grad_rgb[3 * ray + 1]; g2 = io.grad_rgb[3 * ray + 2];
                    ga = io.grad_alpha ? io.grad_alpha[ray] : 0.0f;
                    p0 = p1 = p2 = 0.0f;
                    if (per_ray_t) {
#pragma unroll
                        for (int c = 0; c < C; ++c) gb[c] = 0.0f;
                    }
                    alive = true;
                }
            }
            continue;
        }
        if (n_idle == kWave) break;
        bool has = false;
        int leaf = -1, my_rec = -1;
        float gz0 = 0.0f, gz1 = 0.0f, gz2 = 0.0f, gx = 0.0f;
        if (alive) {
            float delta = 0.0f;
            bool finish;
            float x = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
            float sv[C];
            if constexpr (REPLAY) {
                // replay the forward's sample
                if (tnext >= 0) {
                    const int4 A = io.trace.smp[2 * (int64_t)tnext], B = io.trace.smp[2 * (int64_t)tnext + 1];
                    leaf = A.x;
                    delta = __int_as_float(A.y);
                    x = __int_as_float(A.z);
                    c0 = __int_as_float(A.w);
                    c1 = __int_as_float(B.x);
                    c2 = __int_as_float(B.y);
                    tnext = B.z;
                    if (basis_here) load_leaf<DT, C>(tr.wsig, N, leaf, tr.layout, sv);
                }
                finish = leaf < 0;
            } else {
                float umid;
                leaf = walk_next<kWalkBudget>(tr, rs, w, delta, umid);
                finish = leaf == -1;
                if (leaf >= 0) {
                    float wv[3 * K];
                    load_leaf<DT, 3 * K>(tr.hh, N, leaf, tr.layout, wv);
                    load_leaf<DT, C>(tr.wsig, N, leaf, tr.layout, sv);
                    const float* hl = s_h + threadIdx.x * K;
                    const float* bl = s_b + threadIdx.x * C;
#pragma unroll
                    for (int c = 0; c < C; ++c) x = fmaf(sv[c], bl[c], x);
                    float z0 = 0.0f, z1 = 0.0f, z2 = 0.0f;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const float hk = hl[k];
                        z0 = fmaf(wv[k], hk, z0);
                        z1 = fmaf(wv[K + k], hk, z1);
                        z2 = fmaf(wv[2 * K + k], hk, z2);
                    }
                    c0 = sigmoid_f(z0);
                    c1 = sigmoid_f(z1);
                    c2 = sigmoid_f(z2);
                }
            }
            if (leaf >= 0) {
                const float sig = density_f(x, tr.relu);
                const float od = sig * delta;
                float a, e;
                absorb(od, a, e);
                const float wt = Tr * a;
                const float Tn = Tr * e;
                p0 = fmaf(wt, c0, p0);
                p1 = fmaf(wt, c1, p1);
                p2 = fmaf(wt, c2, p2);
                const float gdotc = g0 * c0 + g1 * c1 + g2 * c2;
                const float gsuf = g0 * (F0 - p0) + g1 * (F1 - p1) + g2 * (F2 - p2);
                // dL/dsigma = delta (T_{k+1} <g, c_k> - <g, rgb - rgb_<=k>) + g_a delta T_final
                const float gsig = delta * (Tn * gdotc - gsuf) + ga * delta * Tfin;
                gx = gsig * density_dx(x, tr.relu);
                gz0 = g0 * wt * c0 * (1.0f - c0);
                gz1 = g1 * wt * c1 * (1.0f - c1);
                gz2 = g2 * wt * c2 * (1.0f - c2);
                if (basis_here) {
#pragma unroll
                    for (int c = 0; c < C; ++c) gb[c] = fmaf(gx, sv[c], gb[c]);
                }
                has = true;
                Tr = Tn;
                ++ns;
                finish = ns >= ns_fwd;
            }
            if (finish) {
                if (io.grad_basis && per_ray_t) {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        unsafeAtomicAdd(io.grad_basis + (int64_t)rs.i0 * C + c, (1.0f - rs.f) * gb[c]);
                        if (rs.f != 0.0f) unsafeAtomicAdd(io.grad_basis + (int64_t)rs.i1 * C + c, rs.f * gb[c]);
                    }
                }
                alive = false;
            }
        }
        if (rec.head) {
            // this iteration's samples take consecutive records in lane order, so
            // the record stores of the wavefront are contiguous
            const uint64_t hm = __ballot(has);
            const int n_has = __popcll(hm);
            const int at = n_has > 0 ? take_items(rec.counter, rec.cap, cc.home, n_has, wrec, wend) : -1;
            if (at >= 0) {
                const RecordRun run = record_run(hm, has, leaf);
                if (has) {
                    my_rec = (int)(at + lane_rank(hm));
                    rec.rec[2 * (int64_t)my_rec] =
                        make_int4(__float_as_int(gz0), __float_as_int(gz1), __float_as_int(gz2), __float_as_int(gx));
                    const int nxt = run.count > 0 ? atomicExch(rec.head + leaf, my_rec + run.count - 1) : my_rec - 1;
                    // one time for every ray: the record carries the ray's direction
                    // (all the reduction needs of the ray), else the ray's index
                    rec.rec[2 * (int64_t)my_rec + 1] =
                        per_ray_t ? make_int4(nxt, (int)ray, 0, 0)
                                  : make_int4(nxt, __float_as_int(dw0), __float_as_int(dw1), __float_as_int(dw2));
                }
            }
        }
        if (basis_late && io.grad_basis && has && my_rec < 0) {
            // a sample without a record: its basis gradient stays here
            float sw[C];
            load_leaf<DT, C>(tr.wsig, N, leaf, tr.layout, sw);
#pragma unroll
            for (int c = 0; c < C; ++c) gb[c] = fmaf(gx, sw[c], gb[c]);
        }
        // samples without a record: every lane of the wavefront adds one
        // component of each produced row
        uint64_t m = __ballot(has && my_rec < 0);
        __builtin_amdgcn_wave_barrier();
        while (m) {
            const int src = __builtin_ctzll(m);
            m &= m - 1;
            const int L = __builtin_amdgcn_readlane(leaf, src);
            const float a0 = readlane_f(gz0, src), a1 = readlane_f(gz1, src), a2 = readlane_f(gz2, src);
            const float ax = readlane_f(gx, src);
            float* row = io.grad_leaf + (int64_t)L * ROW;
#pragma unroll
            for (int c0 = 0; c0 < 3 * K + C; c0 += kWave) {
                const int c = c0 + lane;
                if (c < 3 * K) {
                    const int ch = c / K;
                    const float gzc = ch == 0 ? a0 : (ch == 1 ? a1 : a2);
                    unsafeAtomicAdd(row + c, gzc * s_h[(wbase + src) * K + (c - ch * K)]);
                } else if (c < 3 * K + C) {
                    unsafeAtomicAdd(row + c, ax * s_b[(wbase + src) * C + (c - 3 * K)]);
                }
            }
        }
    }
    // one shared time for every ray: reduce the basis gradient over the block
    if (io.grad_basis && !per_ray_t) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float v = gb[c];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if ((threadIdx.x & 63) == 0) atomicAdd(&s_gb[c], v);
        }
        __syncthreads();
        if (threadIdx.x < C) {
            int i0, i1;
            float f;
            time_setup(tr, in, ra.t_scalar, i0, i1, f);
            const float v = s_gb[threadIdx.x];
            unsafeAtomicAdd(io.grad_basis + (int64_t)i0 * C + threadIdx.x, (1.0f - f) * v);
            if (f != 0.0f) unsafeAtomicAdd(io.grad_basis + (int64_t)i1 * C + threadIdx.x, f * v);
        }
    }
}

// ----------------------------------------------------------------------------
// second pass of the two-phase adjoint
//
// Each lane sums one leaf's record list into a row held in registers: per
// record it redoes the ray's local direction, time frames and basis (the
// functions and inputs of the adjoint, so h and b are those the sample used)
// and adds gz_ch h_k and gx b_c. Lists differ in length by an order of
// magnitude, so a lane whose list has ended takes the next leaf of its
// wavefront's batch instead of waiting for the longest list of the
// wavefront (batches of 64 leaves, wavefront w taking batches w, w + W, ...:
// a shared cursor would serialise on its one address). A finished row is
// transposed through LDS and added to the gradient array with one atomic
// instruction per 64 of its 3K + C values, as the per-sample scatter did,
// but once per leaf. The link of a lane's next record is loaded one record ahead.


// COMMON_T (one time for every ray): the hyperangle gamma(tau) and the
// density-basis row b(tau) are the same for all records, so the radial factors
// of the HH basis and b are computed once, a record costs only its ray's
// harmonics, and a lane holds the 3K HH sums and sum gx; the row's density
// part is then (sum gx) b and the basis gradient (sum gx) w^sigma per leaf,
// summed over the block and spread over the two interpolated rows (when
// grad_basis is given). Otherwise every record redoes its ray's time frames
// and basis, and the basis gradient stays with the adjoint.
template <int K, int C, int DT, bool IDENT, bool COMMON_T>
__global__ __launch_bounds__(kBlock) void reduce_records_kernel(TreeArgs tr, InstArgs in, RayArgs ra,
                                                                RecordArgs rec, float* grad_leaf, float* grad_basis) {
    constexpr int ROW = grad_row<K, C>();
    constexpr int R = 3 * K + C;
    constexpr int NA = COMMON_T ? 3 * K : R;   // row sums a lane holds; acc[NA] = sum gx
    // a finished leaf's slot: its sums, sum gx, its w^sigma
    __shared__ float s_row[kBlock / kWave][kFlushSlots][NA + 1 + C + 1];
    __shared__ float s_gb[C];
    __shared__ float s_bc[C];
    // scalar time: radial factors and density row of the common frame (the
    // arithmetic of ray_basis, so the values are the adjoint's)
    float gq[10];
    if constexpr (COMMON_T) {
        int ci0, ci1;
        float cf;
        time_setup(tr, in, ra.t_scalar, ci0, ci1, cf);
        const float gam = (1.0f - cf) * tr.gamma[ci0] + cf * tr.gamma[ci1];
        hh_radial(gam, gq);
        if (threadIdx.x < C)
            s_bc[threadIdx.x] = (1.0f - cf) * tr.basis[(int64_t)ci0 * C + threadIdx.x] +
                                cf * tr.basis[(int64_t)ci1 * C + threadIdx.x];
    }
    if (threadIdx.x < C) s_gb[threadIdx.x] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int N = (int)tr.n_leaves;
    float bacc = 0.0f;   // lane c < C: component c of the basis gradient

    int leaf = -1;                // this lane's leaf; -1: idle
    int4 ra0 = make_int4(0, 0, 0, 0), ra1 = make_int4(-1, 0, 0, 0);   // its current record
    float acc[NA + 1];
#pragma unroll
    for (int c = 0; c <= NA; ++c) acc[c] = 0.0f;
    LeafFeeder feeder = leaf_feeder(wv);
    __shared__ int2 s_q[kBlock / kWave][kWave];

    for (;;) {
        // hand leaves with records to idle lanes; a lane that got one loads its first record
        int first = -1;
        feed_leaves(feeder, rec, tr.n_leaves, s_q[wv], leaf, first);
        if (first >= 0) {
            ra0 = rec.rec[2 * (int64_t)first];
            ra1 = rec.rec[2 * (int64_t)first + 1];
        }
        if (!__ballot(leaf >= 0)) break;   // no work left (more is false)
        bool done = false;
        if (leaf >= 0) {
            const int nxt = ra1.x;
            const int64_t ray = ra1.y;
            // the next record is loaded while this one is summed
            int4 nx0 = make_int4(0, 0, 0, 0), nx1 = make_int4(-1, 0, 0, 0);
            if (nxt >= 0) {
                nx0 = rec.rec[2 * (int64_t)nxt];
                nx1 = rec.rec[2 * (int64_t)nxt + 1];
            }
            const float4 g = make_float4(__int_as_float(ra0.x), __int_as_float(ra0.y), __int_as_float(ra0.z),
                                         __int_as_float(ra0.w));
            float d[3];
            if constexpr (COMMON_T) {
                d[0] = __int_as_float(ra1.y);
                d[1] = __int_as_float(ra1.z);
                d[2] = __int_as_float(ra1.w);
            } else {
                const f3v dv = load3(ra.d + 3 * ray);
                d[0] = dv.x;
                d[1] = dv.y;
                d[2] = dv.z;
            }
            RaySetup rs;
            float dmax;
            ray_direction<IDENT>(in, d, rs, dmax);
            float h[K];
            if constexpr (COMMON_T) {
                float hall[30];
                hh_assemble(gq, rs.dir[0], rs.dir[1], rs.dir[2], hall);
#pragma unroll
                for (int k = 0; k < K; ++k) h[k] = hall[k];
            } else {
                const float t = ra.t ? ra.t[ray] : ra.t_scalar;
                time_setup(tr, in, t, rs.i0, rs.i1, rs.f);
                float bv[C];
                ray_basis<K, C>(tr, rs, h, bv);
#pragma unroll
                for (int c = 0; c < C; ++c) acc[3 * K + c] = fmaf(g.w, bv[c], acc[3 * K + c]);
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                acc[k] = fmaf(g.x, h[k], acc[k]);
                acc[K + k] = fmaf(g.y, h[k], acc[K + k]);
                acc[2 * K + k] = fmaf(g.z, h[k], acc[2 * K + k]);
            }
            acc[NA] += g.w;
            ra0 = nx0;
            ra1 = nx1;
            done = nxt < 0;
        }
        // finished rows go through kFlushSlots LDS rows at a time (a few lanes
        // finish per iteration)
        uint64_t dm = __ballot(done);
        while (dm) {
            const int r = lane_rank(dm);
            const bool mine = ((dm >> lane) & 1ull) && r < kFlushSlots;
            if (mine) {
                if (grad_basis) {
                    float sw[C];
                    load_leaf<DT, C>(tr.wsig, tr.n_leaves, leaf, tr.layout, sw);
#pragma unroll
                    for (int c = 0; c < C; ++c) s_row[wv][r][NA + 1 + c] = sw[c];
                }
#pragma unroll
                for (int c = 0; c <= NA; ++c) {
                    s_row[wv][r][c] = acc[c];
                    acc[c] = 0.0f;
                }
            }
            uint64_t sm = __ballot(mine);
            __builtin_amdgcn_wave_barrier();
            for (int q = 0; sm; ++q) {
                const int j = __builtin_ctzll(sm);
                sm &= sm - 1;
                const int L = __builtin_amdgcn_readlane(leaf, j);
                const float sgx = s_row[wv][q][NA];
#pragma unroll
                for (int c0 = 0; c0 < R; c0 += kWave) {   // one atomic instruction per 64 values
                    const int c = c0 + lane;
                    if (c < 3 * K || (!COMMON_T && c < R)) {
                        unsafeAtomicAdd(grad_leaf + (int64_t)L * ROW + c, s_row[wv][q][c]);
                    } else if (COMMON_T && c < R) {
                        unsafeAtomicAdd(grad_leaf + (int64_t)L * ROW + c, sgx * s_bc[c - 3 * K]);
                    }
                }
                if (grad_basis && lane < C) bacc = fmaf(sgx, s_row[wv][q][NA + 1 + lane], bacc);
            }
            __builtin_amdgcn_wave_barrier();
            if (mine) leaf = -1;
            dm = __ballot(done && leaf >= 0);
        }
    }
    if (grad_basis) {
        if (lane < C) atomicAdd(&s_gb[lane], bacc);
        __syncthreads();
        if (threadIdx.x < C) {
            int i0, i1;
            float f;
            time_setup(tr, in, ra.t_scalar, i0, i1, f);
            const float v = s_gb[threadIdx.x];
            unsafeAtomicAdd(grad_basis + (int64_t)i0 * C + threadIdx.x, (1.0f - f) * v);
            if (f != 0.0f) unsafeAtomicAdd(grad_basis + (int64_t)i1 * C + threadIdx.x, f * v);
        }
    }
}

template <int K, int C, int DT, bool EDIT, bool TRACE>
static hipError_t fwd_e(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, float t_stop, const RenderOut& o,
                        hipStream_t st) {
    if constexpr (TRACE) {
        // the trace's allocation counters start at zero
        hipLaunchKernelGGL(zero_queue_kernel, dim3(1), dim3(kQueues * kQueueStride), 0, st, o.trace.counter);
    }
    if (in.identity) {
        auto kern = render_fwd_kernel<K, C, DT, true, EDIT, TRACE>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, ra)), dim3(kBlock), 0, st, tr, in, ra, t_stop, o);
    } else {
        auto kern = render_fwd_kernel<K, C, DT, false, EDIT, TRACE>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, ra)), dim3(kBlock), 0, st, tr, in, ra, t_stop, o);
    }
    return hipGetLastError();
}

// Appearance edits are compiled for the K = 16, C = 8 shape only (the C ABI
// rejects trees with edits of other shapes).
template <int K, int C, int DT>
static hipError_t fwd_t(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, float t_stop, const RenderOut& o,
                        hipStream_t st) {
    if constexpr (K == 16 && C == 8) {
        if (o.trace.head)
            return tr.edit ? fwd_e<K, C, DT, true, true>(tr, in, ra, t_stop, o, st)
                           : fwd_e<K, C, DT, false, true>(tr, in, ra, t_stop, o, st);
        return tr.edit ? fwd_e<K, C, DT, true, false>(tr, in, ra, t_stop, o, st)
                       : fwd_e<K, C, DT, false, false>(tr, in, ra, t_stop, o, st);
    } else {
        if (o.trace.head) return fwd_e<K, C, DT, false, true>(tr, in, ra, t_stop, o, st);
        return fwd_e<K, C, DT, false, false>(tr, in, ra, t_stop, o, st);
    }
}

template <int K, int C, int DT, bool REPLAY>
static hipError_t bwd_k(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, const BackwardIO& io,
                        const RecordArgs& rec, hipStream_t st) {
    if (in.identity) {
        auto kern = render_bwd_kernel<K, C, DT, true, REPLAY>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, ra)), dim3(kBlock), 0, st, tr, in, ra, io, rec);
    } else {
        auto kern = render_bwd_kernel<K, C, DT, false, REPLAY>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, ra)), dim3(kBlock), 0, st, tr, in, ra, io, rec);
    }
    return hipGetLastError();
}

template <int K, int C, int DT>
static hipError_t bwd_t(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, const BackwardIO& io,
                        hipStream_t st) {
    // records need int32 ray and record indices
    const int64_t cap =
        ra.n <= (int64_t)INT32_MAX && tr.n_leaves > 0 && tr.n_leaves <= (int64_t)INT32_MAX ? io.record_cap : 0;
    RecordArgs rec{};
    void* mem = nullptr;
    hipError_t e = records_begin(tr, cap, st, rec, mem);
    if (e == hipSuccess) {
        // one cull pass and render adjoint per source of samples: rays that walk,
        // and (traced forward) rays that replay their trace
        auto walk = [&](const RayArgs& r) { return bwd_k<K, C, DT, false>(tr, in, r, io, rec, st); };
        auto replay = [&](const RayArgs& r) { return bwd_k<K, C, DT, true>(tr, in, r, io, rec, st); };
        // the walking adjoint's cull reads whether the forward's traces are all complete
        const RenderOut trace_out{nullptr, nullptr, nullptr, nullptr, nullptr, io.trace};
        if (io.trace.head) {
            if (ra.n > (int64_t)INT32_MAX) e = hipErrorInvalidValue;   // traced calls take candidate lists
            if (e == hipSuccess) e = with_candidates<2>(tr, in, ra, trace_out, io.nsamp, st, walk, io.trace.head);
            if (e == hipSuccess) e = with_candidates<3>(tr, in, ra, RenderOut{}, io.nsamp, st, replay, io.trace.head);
        } else {
            e = with_candidates<1>(tr, in, ra, RenderOut{}, io.nsamp, st, walk);
        }
    }
    if (e == hipSuccess && cap > 0) {
        // persistent: four blocks per CU
        int64_t blocks = (tr.n_leaves + kBlock - 1) / kBlock;
        const int64_t lim = (int64_t)device_cu_count() * 4;
        if (blocks > lim) blocks = lim;
        const dim3 grid((unsigned)blocks);
        if (ra.t == nullptr) {
            if (in.identity)
                hipLaunchKernelGGL((reduce_records_kernel<K, C, DT, true, true>), grid, dim3(kBlock), 0, st, tr, in,
                                   ra, rec, io.grad_leaf, io.grad_basis);
            else
                hipLaunchKernelGGL((reduce_records_kernel<K, C, DT, false, true>), grid, dim3(kBlock), 0, st, tr, in,
                                   ra, rec, io.grad_leaf, io.grad_basis);
        } else {
            if (in.identity)
                hipLaunchKernelGGL((reduce_records_kernel<K, C, DT, true, false>), grid, dim3(kBlock), 0, st, tr, in,
                                   ra, rec, io.grad_leaf, nullptr);
            else
                hipLaunchKernelGGL((reduce_records_kernel<K, C, DT, false, false>), grid, dim3(kBlock), 0, st, tr,
                                   in, ra, rec, io.grad_leaf, nullptr);
        }
        e = hipGetLastError();
    }
    if (mem) {
        const hipError_t f = work_free(mem, st);
        if (e == hipSuccess) e = f;
    }
    return e;
}


// Host launchers of one compiled (K, C) shape of the global-hyperangle form,
// instantiated in a translation unit of their own per shape (render_k*.hip),
// so that the shapes compile in parallel.
template <int K, int C>
hipError_t launch_render_fwd_shape(int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                                   float t_stop, const RenderOut& out, hipStream_t stream, void* ws) {
    auto run = [&](auto dt) {
        return with_candidates<0>(
            tr, in, ra, out, nullptr, stream,
            [&](const RayArgs& r) { return fwd_t<K, C, decltype(dt)::value>(tr, in, r, t_stop, out, stream); },
            nullptr, ws);
    };
    switch (dtype) {
        case 0: return run(std::integral_constant<int, 0>{});
        case 1: return run(std::integral_constant<int, 1>{});
        default: return run(std::integral_constant<int, 2>{});
    }
}

template <int K, int C>
hipError_t launch_render_bwd_shape(int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                                   const BackwardIO& io, hipStream_t stream) {
    switch (dtype) {
        case 0: return bwd_t<K, C, 0>(tr, in, ra, io, stream);
        case 1: return bwd_t<K, C, 1>(tr, in, ra, io, stream);
        default: return bwd_t<K, C, 2>(tr, in, ra, io, stream);
    }
}

// Explicit instantiation of one shape's launchers.
#define NEUVV_RENDER_SHAPE(K, C)                                                                                 \
    template hipError_t launch_render_fwd_shape<K, C>(int, const TreeArgs&, const InstArgs&, const RayArgs&, float, \
                                                      const RenderOut&, hipStream_t, void*);                      \
    template hipError_t launch_render_bwd_shape<K, C>(int, const TreeArgs&, const InstArgs&, const RayArgs&,       \
                                                      const BackwardIO&, hipStream_t);

}  // namespace neuvv
