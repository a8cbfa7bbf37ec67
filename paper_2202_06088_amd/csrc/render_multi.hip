// Exact per-ray rendering of up to 4 placed VOctree instances that may
// interpenetrate or duplicate one another (Sec. 5.1 composition; Alg. 1 is
// exact only for primitives disjoint in depth along a ray).
//
// Every instance k gives a world ray its own local ray with the same
// parameter u, and its leaves give disjoint intervals [a, b) of u with
// constant extinction kappa_k = sigma |d_l,k| per unit u and colour c. A lane
// walks all instances of its ray together: it holds the current segment of
// each, composites the elementary interval from the current position to the
// next boundary of any instance (optical depth sum kappa_k du over the
// instances covering it, colour the kappa-weighted mean of theirs; Eq. 8),
// and fetches the next segment of every instance whose segment ended there.
// Boundaries are compensated ray parameters, so every interval length keeps
// float32 relative accuracy.
//
// Two forms compute this. The two-phase form (below the fused kernel) first
// writes each instance's segments per ray as a list, then merges the lists.
// The fused kernel walks all instances of a ray in one lane: per lane and
// instance, the ray setup, walk state and current segment stay in registers
// (the HH basis is recomputed at each segment fetch). Up to 3 instances it
// runs two wavefronts per SIMD: at 256 registers some of that state spills,
// but the second wavefront hides more memory latency than the spills cost.
// With 4 instances it runs one. It renders the rays whose lists did not fit
// the two-phase form's room. Work distribution is that of render_kernels.h:
// a cull pass lists the candidate rays per XCD part, and persistent
// wavefronts take 64-ray chunks of the lists.
#include <hip/hip_runtime.h>

#include <math.h>

#include "launch.h"
#include "neuvv_device.h"
#include "render_common.h"

namespace neuvv {

struct MSeg {
    df a, b;                  // current segment [a, b) in the ray parameter
    float kap, c0, c1, c2;    // extinction per unit u, colour
    bool has;                 // a segment is held (false: the instance has no more)
};

// Fetches instance k's next segment: walk, then evaluate the leaf (Eq. 4, 5).
template <int DT>
__device__ __forceinline__ void fetch_segment(const TreeArgs& tr, const RaySetup& rs, Walk& w, MSeg& sg) {
    float delta, umid;
    df a, b;
    const int leaf = walk_next(tr, rs, w, delta, umid, a, b);
    if (leaf < 0) {
        sg.has = false;
        return;
    }
    float hall[30];
    const float gam = (1.0f - rs.f) * tr.gamma[rs.i0] + rs.f * tr.gamma[rs.i1];
    hh_all(rs.dir[0], rs.dir[1], rs.dir[2], gam, hall);
    float wv[48], sv[8];
    load_leaf<DT, 48>(tr.hh, tr.n_leaves, leaf, tr.layout, wv);
    load_leaf<DT, 8>(tr.wsig, tr.n_leaves, leaf, tr.layout, sv);
    const float* b0 = tr.basis + (int64_t)rs.i0 * 8;
    const float* b1 = tr.basis + (int64_t)rs.i1 * 8;
    float x = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) x = fmaf(sv[c], (1.0f - rs.f) * b0[c] + rs.f * b1[c], x);
    float z0 = 0.0f, z1 = 0.0f, z2 = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        z0 = fmaf(wv[k], hall[k], z0);
        z1 = fmaf(wv[16 + k], hall[k], z1);
        z2 = fmaf(wv[32 + k], hall[k], z2);
    }
    sg.a = a;
    sg.b = b;
    sg.kap = density_f(x, tr.relu) * rs.len_local;
    sg.c0 = sigmoid_f(z0);
    sg.c1 = sigmoid_f(z1);
    sg.c2 = sigmoid_f(z2);
    sg.has = true;
}

// Coarse test of L placed trees: may the ray hit any of them (the cull pass).
template <int L>
struct AnyTreeHit {
    MultiArgs ma;
    __device__ __forceinline__ bool operator()(const float o[3], const float d[3]) const {
        bool h = false;
#pragma unroll
        for (int k = 0; k < L; ++k) h = h || ray_may_hit<false>(ma.tr[k], ma.in[k], o, d);
        return h;
    }
};

template <int L, int DT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(L <= 3 ? 2 : 1, 8))) void render_multi_kernel(
    MultiArgs ma, RayArgs ra, float t_stop, RenderOut out) {
    if (no_candidates(ra)) return;
    ChunkCursor cc = chunk_cursor();
    bool more = true;

    bool alive = false;
    int64_t ray = -1;
    RaySetup rs[L];
    Walk w[L];
    MSeg sg[L];
    df u = df_from(0.0f);     // current position
    float Tr = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f, wsum = 0.0f, dsum = 0.0f, dlen = 0.0f;
    int ns = 0;

    for (;;) {
        const uint64_t idle = __ballot(!alive);
        const int n_idle = __popcll(idle);
        if (more && (n_idle >= ra.refill_min || n_idle == kWave)) {
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
                            cand = ra.list != nullptr || AnyTreeHit<L>{ma}(o, d);
                            if (!cand) write_miss(out, ray);
                        }
                    }
                }
                cc.pos += take;
            }
            if (cand) {
                Tr = 1.0f; acc0 = acc1 = acc2 = 0.0f; wsum = dsum = 0.0f; ns = 0;
                dlen = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                bool any = false;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    ray_setup<false>(ma.tr[k], ma.in[k], o, d, t, rs[k]);
                    sg[k].has = false;
                    if (rs[k].hit) {
                        walk_begin(ma.tr[k], rs[k], w[k]);
                        fetch_segment<DT>(ma.tr[k], rs[k], w[k], sg[k]);
                        any = any || sg[k].has;
                    }
                }
                if (any) {
                    // start at the first segment's entry
                    bool first = true;
#pragma unroll
                    for (int k = 0; k < L; ++k)
                        if (sg[k].has && (first || df_lt(sg[k].a, u))) { u = sg[k].a; first = false; }
                    alive = true;
                } else {
                    write_miss(out, ray);
                }
            }
            continue;
        }
        if (n_idle == kWave) break;
        if (alive) {
            // next boundary of any instance, and the instances covering [u, nb)
            df nb = df_from(0.0f);
            bool have_nb = false;
            float ksum = 0.0f, kc0 = 0.0f, kc1 = 0.0f, kc2 = 0.0f;
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (!sg[k].has) continue;
                const bool inside = !df_lt(u, sg[k].a);          // a <= u (< b)
                const df e = inside ? sg[k].b : sg[k].a;
                if (!have_nb || df_lt(e, nb)) { nb = e; have_nb = true; }
                if (inside) {
                    ksum += sg[k].kap;
                    kc0 = fmaf(sg[k].kap, sg[k].c0, kc0);
                    kc1 = fmaf(sg[k].kap, sg[k].c1, kc1);
                    kc2 = fmaf(sg[k].kap, sg[k].c2, kc2);
                }
            }
            bool finish = !have_nb;
            if (have_nb && ksum > 0.0f) {
                const float du = df_f(df_sub(nb, u));
                const float od = ksum * du;
                float a, e_od;
                absorb(od, a, e_od);
                const float wt = Tr * a;
                const float inv = 1.0f / ksum;
                acc0 = fmaf(wt, kc0 * inv, acc0);
                acc1 = fmaf(wt, kc1 * inv, acc1);
                acc2 = fmaf(wt, kc2 * inv, acc2);
                wsum += wt;
                dsum = fmaf(wt, 0.5f * (df_f(u) + df_f(nb)) * dlen, dsum);
                Tr *= e_od;
                ++ns;
                finish = t_stop > 0.0f && Tr < t_stop;
            }
            if (!finish) {
                u = nb;
                bool any = false;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    if (sg[k].has && !df_lt(u, sg[k].b))        // this instance's segment ends here
                        fetch_segment<DT>(ma.tr[k], rs[k], w[k], sg[k]);
                    any = any || sg[k].has;
                }
                finish = !any;
            }
            if (finish) {
                if (out.rgb) { out.rgb[3 * ray] = acc0; out.rgb[3 * ray + 1] = acc1; out.rgb[3 * ray + 2] = acc2; }
                if (out.alpha) out.alpha[ray] = 1.0f - Tr;
                if (out.depth) out.depth[ray] = wsum > 0.0f ? dsum / wsum : INFINITY;
                if (out.nsamp) out.nsamp[ray] = ns;
                alive = false;
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Two-phase form, used when the rays' lists fit their room.
//
// Phase 1 (merge_emit_kernel, one launch per instance over the list of one
// cull pass for all instances) walks the rays through
// one instance, as the forward does, and writes that instance's segments
// along each ray as a linked list of 32-byte entries in increasing u:
// {b.hi, b.lo, kappa, c_r} {c_g, c_b, next (-1: last), 0}, where b is the
// compensated end of the entry's interval; an interval starts where the
// previous entry's ends. The stretch before the first segment, and every gap
// between two segments, is an entry of extinction 0, so that a list reads as
// a sequence of abutting intervals. A ray stops once the instance's own
// transmittance falls below kEmitStop * t_stop: the merged transmittance is
// the product of every instance's, so the merge stops at that entry's end at
// the latest (the factor covers the rounding of the two products).
//
// Phase 2 (merge_lists_kernel) holds one entry per instance and ray and
// composites the elementary intervals between consecutive entry ends with the
// arithmetic of the fused kernel above, in the same order (an extinction-0
// entry adds exact zeros), so the two forms give the same result. It keeps no
// walk state, payload or node rows, and runs at full occupancy.
//
// Rays whose list did not fit the room (head -2) are listed by phase 2 and
// rendered afterwards by the fused kernel.

constexpr float kEmitStop = 0.99f;
constexpr int64_t kMergeRoomPerRay = 2;   // list entries per ray and instance

struct MergeLists {
    int32_t* head;                 // [n] first entry of the ray's list; -1: empty, -2: the room ran out
    int4* ent;                     // [cap][2]
    unsigned long long* counter;   // kQueues counters, 128 bytes apart (entries handed out per XCD part)
    int64_t cap;
};

__device__ __forceinline__ void store_entry(int4* ent, int slot, df b, float kap, float c0, float c1, float c2,
                                            int next) {
    int4* e = ent + 2 * (int64_t)slot;
    e[0] = make_int4(__float_as_int(b.hi), __float_as_int(b.lo), __float_as_int(kap), __float_as_int(c0));
    e[1] = make_int4(__float_as_int(c1), __float_as_int(c2), next, 0);
}

template <int DT, bool IDENT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void merge_emit_kernel(
    TreeArgs tr, InstArgs in, RayArgs ra, float t_stop, MergeLists ml) {
    if (no_candidates(ra)) return;
    __shared__ float s_h[kBlock * 16];
    __shared__ float s_b[kBlock * 8];
    ChunkCursor cc = chunk_cursor();
    bool more = true;

    bool alive = false;
    int64_t ray = -1;
    RaySetup rs;
    Walk w;
    float* const hl = s_h + threadIdx.x * 16;
    float* const bl = s_b + threadIdx.x * 8;
    float Tr = 1.0f;
    int first = -1;               // the ray's first entry; -2: the room ran out
    int pslot = -1;               // the last segment's entry, stored once what follows it is known
    df pb = df_from(0.0f);        // that segment's end, extinction and colour
    float pk = 0.0f, pc0 = 0.0f, pc1 = 0.0f, pc2 = 0.0f;
    int tcur = 0, tend = 0;   // what is left of the wavefront's block of entries (wave-uniform)

    for (;;) {
        const uint64_t idle = __ballot(!alive);
        const int n_idle = __popcll(idle);
        if (more && (n_idle >= ra.refill_min || n_idle == kWave)) {
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
                            cand = ray_may_hit<IDENT>(tr, in, o, d);   // (the list holds rays of any instance)
                        }
                    }
                }
                cc.pos += take;
            }
            if (cand) {
                ray_setup<IDENT>(tr, in, o, d, t, rs);
                if (rs.hit) {
                    float hall[30];
                    const float gam = (1.0f - rs.f) * tr.gamma[rs.i0] + rs.f * tr.gamma[rs.i1];
                    hh_all(rs.dir[0], rs.dir[1], rs.dir[2], gam, hall);
#pragma unroll
                    for (int k = 0; k < 16; ++k) hl[k] = hall[k];
                    const float* b0 = tr.basis + (int64_t)rs.i0 * 8;
                    const float* b1 = tr.basis + (int64_t)rs.i1 * 8;
#pragma unroll
                    for (int c = 0; c < 8; ++c) bl[c] = (1.0f - rs.f) * b0[c] + rs.f * b1[c];
                    walk_begin(tr, rs, w);
                    alive = true;
                    Tr = 1.0f;
                    first = -1;
                    pslot = -1;
                }
            }
            continue;
        }
        if (n_idle == kWave) break;
        bool finish = false;
        int leaf = -1;
        float delta = 0.0f, umid = 0.0f;
        df a = df_from(0.0f), b = df_from(0.0f);
        if (alive) {
            leaf = walk_next<kWalkBudget>(tr, rs, w, delta, umid, a, b);
            finish = leaf == -1;
        }
        // this iteration's entries: the segment, after a gap entry when it does
        // not start where the previous one ended (always before the first)
        const bool gap = leaf >= 0 && (pslot < 0 || df_lt(pb, a));
        const uint64_t m1 = __ballot(leaf >= 0), m2 = __ballot(gap);
        const int n_e = __popcll(m1) + __popcll(m2);
        const int at = n_e > 0 ? take_items(ml.counter, ml.cap, cc.home, n_e, tcur, tend) : -1;
        if (leaf >= 0) {
            if (at < 0) {
                first = -2;   // the room ran out: the fused kernel renders this ray
                finish = true;
            } else {
                const int e0 = (int)(at + lane_rank(m1) + lane_rank(m2));
                const int seg = gap ? e0 + 1 : e0;
                float wv[48], sv[8];
                load_leaf<DT, 48>(tr.hh, tr.n_leaves, leaf, tr.layout, wv);
                load_leaf<DT, 8>(tr.wsig, tr.n_leaves, leaf, tr.layout, sv);
                if (pslot >= 0) store_entry(ml.ent, pslot, pb, pk, pc0, pc1, pc2, e0);
                if (gap) store_entry(ml.ent, e0, a, 0.0f, 0.0f, 0.0f, 0.0f, seg);
                if (first == -1) first = e0;
                float x = 0.0f;
#pragma unroll
                for (int c = 0; c < 8; ++c) x = fmaf(sv[c], bl[c], x);
                float z0 = 0.0f, z1 = 0.0f, z2 = 0.0f;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const float hk = hl[k];
                    z0 = fmaf(wv[k], hk, z0);
                    z1 = fmaf(wv[16 + k], hk, z1);
                    z2 = fmaf(wv[32 + k], hk, z2);
                }
                const float sig = density_f(x, tr.relu);
                pslot = seg;
                pb = b;
                pk = sig * rs.len_local;
                pc0 = sigmoid_f(z0);
                pc1 = sigmoid_f(z1);
                pc2 = sigmoid_f(z2);
                float al, e_od;
                absorb(sig * delta, al, e_od);
                Tr *= e_od;
                finish = t_stop > 0.0f && Tr < kEmitStop * t_stop;
            }
        }
        if (alive && finish) {
            if (first >= 0) store_entry(ml.ent, pslot, pb, pk, pc0, pc1, pc2, -1);
            ml.head[ray] = first;
            alive = false;
        }
    }
}

__device__ __forceinline__ void load_entry(const int4* __restrict__ ent, int slot, df& b, float& kap, float& c0,
                                           float& c1, float& c2, int& next) {
    const int4* e = ent + 2 * (int64_t)slot;
    const int4 A = e[0], B = e[1];
    b = df{__int_as_float(A.x), __int_as_float(A.y)};
    kap = __int_as_float(A.z);
    c0 = __int_as_float(A.w);
    c1 = __int_as_float(B.x);
    c2 = __int_as_float(B.y);
    next = B.z;
}

// Cull of phase 2: a ray is worth merging when some instance gave it a list
// (or ran out of room for it); the others get the miss outputs.
template <int L>
struct AnyList {
    const int32_t* head;
    int64_t n;
    __device__ __forceinline__ bool keep(int64_t ray) const {
        bool k = false;
#pragma unroll
        for (int i = 0; i < L; ++i) k = k || head[(int64_t)i * n + ray] != -1;
        return k;
    }
};

template <int L>
__global__ __launch_bounds__(kBlock) void merge_lists_kernel(RayArgs ra, const int32_t* __restrict__ head,
                                                             const int4* __restrict__ ent, float t_stop,
                                                             RenderOut out, int32_t* fb_list,
                                                             unsigned long long* fb_count) {
    ChunkCursor cc = chunk_cursor();
    bool more = true;
    bool alive = false;
    int64_t ray = -1;
    df cb[L];                                     // per instance: the current entry's end,
    float ck[L], cr[L], cg[L], cbl[L];            // extinction, colour
    int nx[L];                                    // and next entry
    bool act[L];                                  // false: the instance's list is done
    df u = df_from(0.0f);
    float Tr = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f, wsum = 0.0f, dsum = 0.0f, dlen = 0.0f;
    int ns = 0;
    const int64_t n = ra.n;

    for (;;) {
        const uint64_t idle = __ballot(!alive);
        const int n_idle = __popcll(idle);
        if (more && (n_idle >= ra.refill_min || n_idle == kWave)) {
            bool cand = false;
            int hd[L];
            for (;;) {
                const uint64_t need = __ballot(!alive && !cand);
                const int n_need = __popcll(need);
                if (n_need < ra.refill_min) break;
                if (cc.pos == kWave && !next_chunk(ra, cc)) {
                    more = false;
                    break;
                }
                const int take = n_need < kWave - cc.pos ? n_need : kWave - cc.pos;
                bool fb = false;
                if (!alive && !cand) {
                    const int r = lane_rank(need);
                    if (r < take) {
                        ray = chunk_ray(ra, cc, cc.pos + r);
                        if (ray >= 0) {
                            bool any = false;
#pragma unroll
                            for (int k = 0; k < L; ++k) {
                                hd[k] = head[(int64_t)k * n + ray];
                                fb = fb || hd[k] == -2;
                                any = any || hd[k] >= 0;
                            }
                            if (!fb) {
                                if (any) cand = true;
                                else write_miss(out, ray);   // (the cull pass has listed only rays with lists)
                            }
                        }
                    }
                }
                const uint64_t fm = __ballot(fb);
                if (fm) {
                    unsigned long long base = 0;
                    if ((threadIdx.x & 63) == 0) base = atomicAdd(fb_count, (unsigned long long)__popcll(fm));
                    const int b0 = __builtin_amdgcn_readfirstlane((int)(uint32_t)base);
                    if (fb) fb_list[b0 + lane_rank(fm)] = (int32_t)ray;
                }
                cc.pos += take;
            }
            if (cand) {
                const f3v dv = load3(ra.d + 3 * ray);
                dlen = sqrtf(dv.x * dv.x + dv.y * dv.y + dv.z * dv.z);
                Tr = 1.0f; acc0 = acc1 = acc2 = 0.0f; wsum = dsum = 0.0f; ns = 0;
                bool first = true;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    act[k] = hd[k] >= 0;
                    if (act[k]) {
                        load_entry(ent, hd[k], cb[k], ck[k], cr[k], cg[k], cbl[k], nx[k]);
                        // a list opens with the gap before its first segment: start at the earliest
                        if (first || df_lt(cb[k], u)) { u = cb[k]; first = false; }
                    }
                }
                alive = true;
            }
            continue;
        }
        if (n_idle == kWave) break;
        if (alive) {
            // every instance whose entry ends here moves to its next entry
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (act[k] && !df_lt(u, cb[k])) {
                    if (nx[k] >= 0) load_entry(ent, nx[k], cb[k], ck[k], cr[k], cg[k], cbl[k], nx[k]);
                    else act[k] = false;
                }
            }
            // the next entry end, and the extinction and colour over [u, nb)
            df nb = df_from(0.0f);
            bool any = false;
            float ksum = 0.0f, kc0 = 0.0f, kc1 = 0.0f, kc2 = 0.0f;
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (!act[k]) continue;
                if (!any || df_lt(cb[k], nb)) nb = cb[k];
                any = true;
                ksum += ck[k];
                kc0 = fmaf(ck[k], cr[k], kc0);
                kc1 = fmaf(ck[k], cg[k], kc1);
                kc2 = fmaf(ck[k], cbl[k], kc2);
            }
            bool finish = !any;
            if (any && ksum > 0.0f) {
                const float du = df_f(df_sub(nb, u));
                const float od = ksum * du;
                float a, e_od;
                absorb(od, a, e_od);
                const float wt = Tr * a;
                const float inv = 1.0f / ksum;
                acc0 = fmaf(wt, kc0 * inv, acc0);
                acc1 = fmaf(wt, kc1 * inv, acc1);
                acc2 = fmaf(wt, kc2 * inv, acc2);
                wsum += wt;
                dsum = fmaf(wt, 0.5f * (df_f(u) + df_f(nb)) * dlen, dsum);
                Tr *= e_od;
                ++ns;
                finish = t_stop > 0.0f && Tr < t_stop;
            }
            if (!finish) u = nb;
            if (finish) {
                if (out.rgb) { out.rgb[3 * ray] = acc0; out.rgb[3 * ray + 1] = acc1; out.rgb[3 * ray + 2] = acc2; }
                if (out.alpha) out.alpha[ray] = 1.0f - Tr;
                if (out.depth) out.depth[ray] = wsum > 0.0f ? dsum / wsum : INFINITY;
                if (out.nsamp) out.nsamp[ray] = ns;
                alive = false;
            }
        }
    }
}

static __global__ void merge_init_kernel(int32_t* head, int64_t n, unsigned long long* hdr, int n_hdr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) head[i] = -1;
    if (i < n_hdr) hdr[i] = 0ull;
}

template <int L, int DT>
static hipError_t multi_lists(const MultiArgs& ma, const RayArgs& ra, float t_stop, const RenderOut& o,
                              hipStream_t st) {
    const int64_t n = ra.n;
    const int64_t cap = kMergeRoomPerRay * L * n;
    // scratch: 8 KiB of counters (entries handed out; 1 KiB unused; the
    // fallback launch's work queue and list counts; a work queue per
    // instance's walk), the heads, the fallback list, the entries (the
    // candidate lists of both phases come from with_list)
    constexpr size_t hdr = 4096 + 4 * 1024;
    const size_t head_b = ((size_t)L * n * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t list_b = ((size_t)((ra.n_slots + 63) >> 6) * 64 * sizeof(int32_t) + 255) & ~(size_t)255;
    void* mem = nullptr;
    hipError_t e = work_alloc(&mem, hdr + head_b + list_b + (size_t)cap * 2 * sizeof(int4), st);
    if (e != hipSuccess) return e;
    char* p = static_cast<char*>(mem);
    auto* counter = reinterpret_cast<unsigned long long*>(p);
    auto* q_fb = reinterpret_cast<unsigned long long*>(p + 2048);
    auto* cnt_fb = reinterpret_cast<unsigned long long*>(p + 3072);
    auto* q_emit = reinterpret_cast<unsigned long long*>(p + 4096);
    auto* head = reinterpret_cast<int32_t*>(p + hdr);
    auto* fb_list = reinterpret_cast<int32_t*>(p + hdr + head_b);
    auto* ent = reinterpret_cast<int4*>(p + hdr + head_b + list_b);
    const int64_t init_n = L * n > (int64_t)(hdr / 8) ? L * n : (int64_t)(hdr / 8);
    hipLaunchKernelGGL(merge_init_kernel, dim3((unsigned)((init_n + 255) / 256)), dim3(256), 0, st, head, L * n,
                       counter, (int)(hdr / 8));
    e = hipGetLastError();
    if (e == hipSuccess) {
        // phase 1: one cull pass lists the rays that may hit any instance; each
        // instance's walk takes that list through a work queue of its own
        e = with_list(
            ra, st,
            [&](int32_t* list, unsigned long long* count) {
                return launch_cull_hit<0>(AnyTreeHit<L>{ma}, ra, RenderOut{}, nullptr, nullptr, list, count, st);
            },
            [&](const RayArgs& r) {
                hipError_t le = hipSuccess;
                for (int k = 0; k < L && le == hipSuccess; ++k) {
                    RayArgs rk = r;
                    rk.queue = q_emit + (size_t)k * 128;
                    const MergeLists ml{head + (int64_t)k * n, ent, counter, cap};
                    if (ma.in[k].identity) {
                        auto kern = merge_emit_kernel<DT, true>;
                        hipLaunchKernelGGL(kern, dim3(grid_for(kern, rk)), dim3(kBlock), 0, st, ma.tr[k], ma.in[k],
                                           rk, t_stop, ml);
                    } else {
                        auto kern = merge_emit_kernel<DT, false>;
                        hipLaunchKernelGGL(kern, dim3(grid_for(kern, rk)), dim3(kBlock), 0, st, ma.tr[k], ma.in[k],
                                           rk, t_stop, ml);
                    }
                    le = hipGetLastError();
                }
                return le;
            });
    }
    if (e == hipSuccess) {
        // phase 2 over the rays with lists (a cull pass lists them and writes the misses)
        e = with_list(
            ra, st,
            [&](int32_t* list, unsigned long long* count) {
                return launch_cull_hit<4>(AnyList<L>{head, n}, ra, o, nullptr, nullptr, list, count, st);
            },
            [&](const RayArgs& rm) {
                auto kern = merge_lists_kernel<L>;
                hipLaunchKernelGGL(kern, dim3(grid_for(kern, rm)), dim3(kBlock), 0, st, rm, head, ent, t_stop, o,
                                   fb_list, cnt_fb);
                return hipGetLastError();
            });
    }
    if (e == hipSuccess) {
        // the rays listed by phase 2 (all in the first part of the list)
        RayArgs rf = ra;
        rf.queue = q_fb;
        rf.count = cnt_fb;
        rf.list = fb_list;
        auto kern = render_multi_kernel<L, DT>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, rf)), dim3(kBlock), 0, st, ma, rf, t_stop, o);
        e = hipGetLastError();
    }
    const hipError_t f = work_free(mem, st);
    return e != hipSuccess ? e : f;
}

template <int L, int DT>
static hipError_t multi_t(const MultiArgs& ma, const RayArgs& ra, float t_stop, const RenderOut& o, hipStream_t st) {
    // two-phase form while list indices fit int32
    if (ra.n <= (int64_t)INT32_MAX / (2 * kMergeRoomPerRay * L)) return multi_lists<L, DT>(ma, ra, t_stop, o, st);
    // cull pass over every instance, then the merge over the listed rays
    return with_list(
        ra, st,
        [&](int32_t* list, unsigned long long* count) {
            return launch_cull_hit<0>(AnyTreeHit<L>{ma}, ra, o, nullptr, nullptr, list, count, st);
        },
        [&](const RayArgs& r) {
            auto kern = render_multi_kernel<L, DT>;
            hipLaunchKernelGGL(kern, dim3(grid_for(kern, r)), dim3(kBlock), 0, st, ma, r, t_stop, o);
            return hipGetLastError();
        });
}

template <int DT>
static hipError_t multi_l(int L, const MultiArgs& ma, const RayArgs& ra, float t_stop, const RenderOut& o,
                          hipStream_t st) {
    switch (L) {
        case 1: return multi_t<1, DT>(ma, ra, t_stop, o, st);
        case 2: return multi_t<2, DT>(ma, ra, t_stop, o, st);
        case 3: return multi_t<3, DT>(ma, ra, t_stop, o, st);
        default: return multi_t<4, DT>(ma, ra, t_stop, o, st);
    }
}

hipError_t launch_render_multi(int L, int dtype, const MultiArgs& ma, const RayArgs& ra, float t_stop,
                               const RenderOut& out, hipStream_t stream) {
    if (ra.n_slots <= 0) return hipSuccess;
    switch (dtype) {
        case 0: return multi_l<0>(L, ma, ra, t_stop, out, stream);
        case 1: return multi_l<1>(L, ma, ra, t_stop, out, stream);
        default: return multi_l<2>(L, ma, ra, t_stop, out, stream);
    }
}

}  // namespace neuvv
