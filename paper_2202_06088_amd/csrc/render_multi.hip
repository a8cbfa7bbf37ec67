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
// Per lane and instance, the ray setup, walk state and current segment stay
// in registers (the HH basis is recomputed at each segment fetch). Up to 3
// instances the kernel runs two wavefronts per SIMD: at 256 registers some of
// that state spills, but the second wavefront hides more memory latency than
// the spills cost. With 4 instances it runs one. Work distribution is that of render_kernels.h: a cull pass
// (here: may the ray hit any instance) lists the candidate rays per XCD
// part, and persistent wavefronts take 64-ray chunks of the lists.
#include <hip/hip_runtime.h>

#include <math.h>

#include "launch.h"
#include "neuvv_device.h"
#include "render_common.h"

namespace neuvv {

constexpr int kLdsNodesMulti = 512;

struct MSeg {
    df a, b;                  // current segment [a, b) in the ray parameter
    float kap, c0, c1, c2;    // extinction per unit u, colour
    bool has;                 // a segment is held (false: the instance has no more)
};

// Fetches instance k's next segment: walk, then evaluate the leaf (Eq. 4, 5).
template <int DT>
__device__ __forceinline__ void fetch_segment(const TreeArgs& tr, const int4* s_nodes, int n_lds, int* path,
                                              const RaySetup& rs, Walk& w, MSeg& sg) {
    float delta, umid;
    df a, b;
    const int leaf = walk_next(tr, s_nodes, n_lds, path, kBlock, rs, w, delta, umid, a, b);
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
    __shared__ int4 s_nodes[L][kLdsNodesMulti];
    __shared__ int s_path[L][kMaxLevels * kBlock];
    int n_lds[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        n_lds[k] = (int)(ma.tr[k].n_nodes < kLdsNodesMulti ? ma.tr[k].n_nodes : kLdsNodesMulti);
        for (int i = threadIdx.x; i < n_lds[k]; i += kBlock) s_nodes[k][i] = ma.tr[k].nodes[i];
    }
    __syncthreads();
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
                        fetch_segment<DT>(ma.tr[k], s_nodes[k], n_lds[k], &s_path[k][threadIdx.x], rs[k], w[k], sg[k]);
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
                        fetch_segment<DT>(ma.tr[k], s_nodes[k], n_lds[k], &s_path[k][threadIdx.x], rs[k], w[k],
                                          sg[k]);
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

template <int L, int DT>
static hipError_t multi_t(const MultiArgs& ma, const RayArgs& ra, float t_stop, const RenderOut& o, hipStream_t st) {
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
