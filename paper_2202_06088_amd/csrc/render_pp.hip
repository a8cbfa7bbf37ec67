// VOctree rendering with the per-point hyperangle (Sec. 4.2, Eq. 6): every
// leaf carries Cg weights on a second learned temporal basis, a sample's
// hyperangle is gamma = pi sigmoid(sum_c wgam_c Bg_c(t)), and its HH basis is
// g_nl(gamma) Y_lm(d) (Eq. 2-4), with the direction factors Y_lm per ray and
// the radial factors g_nl per sample. Compiled for the paper's leaf: K = 14
// HH functions per channel (all n <= 2), C = 31 density weights and Cg = 31
// hyperangle weights, 104 values in all (Sec. 1, Tables 2-3); forward and
// adjoint (Sec. 4.3 "Optimization"), whose chain rule gains the hyperangle
// path dL/dgamma -> dL/dwgam and dL/dBg.
//
// Work distribution, traversal and compositing are those of render_kernels.h. The
// interpolated basis rows are common to all rays when the time is one scalar
// and are then staged once per block in LDS; with a time per ray they are
// read per sample from the basis tables, which stay in cache. A traced
// forward also records every sample, with the three dz/dgamma its colour
// logits need, so that the adjoint of the same call replays the samples
// without walking the tree or reading the payload.
#include <hip/hip_runtime.h>

#include <math.h>

#include "launch.h"
#include "neuvv_device.h"
#include "render_common.h"

namespace neuvv {

namespace pp {
constexpr int K = 14;
constexpr int C = 31;
constexpr int CG = 31;
constexpr int ROW = ((3 * K + C + CG + 63) / 64) * 64;   // 128
// cells per walk call in the adjoint (as in the forward: the basis gradients'
// wavefront-wide butterfly, which made longer strides pay, only runs for
// samples without a record)
constexpr int kWalkBudgetBwd = kWalkBudget;
constexpr float kPi = 3.14159265358979323846f;
}  // namespace pp

// sum_c w[c] * ((1 - f) B[i0][c] + f B[i1][c]); s_row holds that interpolated
// row when every ray shares it (nullptr otherwise).
template <int N>
__device__ __forceinline__ float basis_dot(const float (&w)[N], const float* s_row, const float* B, int i0, int i1,
                                           float f) {
    float x = 0.0f;
    if (s_row) {
#pragma unroll
        for (int c = 0; c < N; ++c) x = fmaf(w[c], s_row[c], x);
    } else {
        const float* b0 = B + (int64_t)i0 * N;
        const float* b1 = B + (int64_t)i1 * N;
#pragma unroll
        for (int c = 0; c < N; ++c) x = fmaf(w[c], (1.0f - f) * b0[c] + f * b1[c], x);
    }
    return x;
}

// Value e of the R-value row of leaf `slot` (layouts as in load_leaf).
template <int DT, int R>
__device__ __forceinline__ float leaf_elem(const void* base, int64_t N, int64_t slot, int e, int layout) {
    constexpr int V = StoreTraits<DT>::V;
    constexpr int NG = (R + V - 1) / V;
    const int g = e / V, r = e - (e / V) * V;
    const int64_t vec = layout ? slot * NG + g : (int64_t)g * N + slot;
    if constexpr (DT == 0) {
        return reinterpret_cast<const float*>(base)[vec * 4 + r];
    } else {
        const uint16_t u = reinterpret_cast<const uint16_t*>(base)[vec * 8 + r];
        if constexpr (DT == 1) return (float)__builtin_bit_cast(_Float16, u);
        else return __uint_as_float((uint32_t)u << 16);
    }
}

// Stages the interpolated basis rows shared by every ray (scalar time) in
// LDS; the caller's barrier makes them visible.
__device__ __forceinline__ void stage_common_rows(const TreeArgs& tr, const InstArgs& in, float t, float* s_b,
                                                  float* s_bg) {
    using namespace pp;
    if (threadIdx.x < C + CG) {
        int i0, i1;
        float f;
        time_setup(tr, in, t, i0, i1, f);
        if (threadIdx.x < C) {
            const int c = threadIdx.x;
            s_b[c] = (1.0f - f) * tr.basis[(int64_t)i0 * C + c] + f * tr.basis[(int64_t)i1 * C + c];
        } else {
            const int c = threadIdx.x - C;
            s_bg[c] = (1.0f - f) * tr.basis_g[(int64_t)i0 * CG + c] + f * tr.basis_g[(int64_t)i1 * CG + c];
        }
    }
}

// One sample's per-point quantities: density logit x, hyperangle logit y,
// radial factors g (and dg / dgamma) and colour logits z.
template <int DT>
struct PPSample {
    float wv[3 * pp::K], sv[pp::C], gv[pp::CG];
    float x, y, g[6], dg[6], h[pp::K], z0, z1, z2;
};

template <int DT>
__device__ __forceinline__ void pp_load(const TreeArgs& tr, int leaf, PPSample<DT>& p) {
    using namespace pp;
    load_leaf<DT, 3 * K>(tr.hh, tr.n_leaves, leaf, tr.layout, p.wv);
    load_leaf<DT, C>(tr.wsig, tr.n_leaves, leaf, tr.layout, p.sv);
    load_leaf<DT, CG>(tr.wgam, tr.n_leaves, leaf, tr.layout, p.gv);
}

// The sample's logits x, y, hyperangle factors g, g' and basis h, and the
// colour logits z (Eq. 2-6), from the payload pp_load fetched.
template <int DT>
__device__ __forceinline__ void pp_compute(const TreeArgs& tr, const RaySetup& rs, const float (&Y)[8],
                                           const float* s_b, const float* s_bg, PPSample<DT>& p) {
    using namespace pp;
    p.x = basis_dot<C>(p.sv, s_b, tr.basis, rs.i0, rs.i1, rs.f);
    p.y = basis_dot<CG>(p.gv, s_bg, tr.basis_g, rs.i0, rs.i1, rs.f);
    const float gam = kPi * sigmoid_f(p.y);
    float sn, cs;
    sincosf(gam, &sn, &cs);
    radial_n2(sn, cs, p.g, p.dg);
    hh14(p.g, Y, p.h);
    p.z0 = p.z1 = p.z2 = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        p.z0 = fmaf(p.wv[k], p.h[k], p.z0);
        p.z1 = fmaf(p.wv[K + k], p.h[k], p.z1);
        p.z2 = fmaf(p.wv[2 * K + k], p.h[k], p.z2);
    }
}

// dz_ch/dgamma = sum_k W_ch,k g'_nl(gamma) Y_k for the three colour channels.
template <int DT>
__device__ __forceinline__ void pp_dz_dgamma(const PPSample<DT>& p, const float (&Y)[8], float& q0, float& q1,
                                             float& q2) {
    using namespace pp;
    float dh[K];
    hh14(p.dg, Y, dh);
    q0 = q1 = q2 = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        q0 = fmaf(p.wv[k], dh[k], q0);
        q1 = fmaf(p.wv[K + k], dh[k], q1);
        q2 = fmaf(p.wv[2 * K + k], dh[k], q2);
    }
}

// A per-point trace entry is 64 bytes (two entries of the trace's room):
// {leaf, delta, x, y} {c_r, c_g, c_b, next} {dz_r/dgamma, dz_g/dgamma,
// dz_b/dgamma, -}, the fourth 16 bytes unused.
constexpr int kPPTraceInt4 = 4;

// ----------------------------------------------------------------------------
// forward

// TRACE: every sample is also written to out.trace (leaf, segment length,
// logits x and y, colours, dz/dgamma; linked in ray order) for the adjoint of
// the same call, as in render_kernels.h: entries of one iteration at consecutive
// slots in lane order, a sample's entry stored one sample later (when the
// slot it links to is known) right after the next sample's payload loads,
// the last one when the ray finishes; a ray whose samples do not all fit
// gets head -1. The room in samples is half the trace's room in 32-byte
// entries.
template <int DT, bool IDENT, bool TRACE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void render_pp_fwd_kernel(
    TreeArgs tr, InstArgs in, RayArgs ra, float t_stop, RenderOut out) {
    if (no_candidates(ra)) return;
    using namespace pp;
    __shared__ float s_brow[C], s_bgrow[CG];
    const bool common_t = ra.t == nullptr;
    if (common_t) stage_common_rows(tr, in, ra.t_scalar, s_brow, s_bgrow);
    __syncthreads();
    const float* s_b = common_t ? s_brow : nullptr;
    const float* s_bg = common_t ? s_bgrow : nullptr;
    ChunkCursor cc = chunk_cursor();
    bool more = true;

    bool alive = false;
    int64_t ray = -1;
    RaySetup rs;
    Walk w;
    float Y[8];
    float Tr = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f, wsum = 0.0f, dsum = 0.0f;
    int ns = 0;
    int t_first = -1;                // trace: the ray's first entry; -2: incomplete
    int tcur = 0, tend = 0;      // trace: what is left of the wavefront's block (wave-uniform)
    const int64_t t_room = out.trace.cap / 2;
    // trace: the previous sample, stored once the slot of the next is known
    int pslot = -1, pleaf = 0;
    float pdelta = 0.0f, px = 0.0f, py = 0.0f, pc0 = 0.0f, pc1 = 0.0f, pc2 = 0.0f, pq0 = 0.0f, pq1 = 0.0f,
          pq2 = 0.0f;

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
                    sh_deg2(rs.dir[0], rs.dir[1], rs.dir[2], Y);
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
        bool finish = false;
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
            const int at = n_s > 0 ? take_items(out.trace.counter, t_room, cc.home, n_s, tcur, tend) : -1;
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
            PPSample<DT> p;
            pp_load<DT>(tr, leaf, p);
            if constexpr (TRACE) {
                // the previous sample's entry, linked to this one; a ray's first
                // sample stores a placeholder into its own slot (overwritten by this
                // lane later), an incomplete trace into its last slot or the spare
                // half of the trace header
                const int tgt = pslot >= 0 ? pslot : cur;
                int4* dst = tgt >= 0 ? out.trace.smp + kPPTraceInt4 * (int64_t)tgt
                                     : reinterpret_cast<int4*>(reinterpret_cast<char*>(out.trace.counter) + 1024) +
                                           kPPTraceInt4 * (threadIdx.x & 15);
                dst[0] = make_int4(pleaf, __float_as_int(pdelta), __float_as_int(px), __float_as_int(py));
                dst[1] = make_int4(__float_as_int(pc0), __float_as_int(pc1), __float_as_int(pc2), cur);
                dst[2] = make_int4(__float_as_int(pq0), __float_as_int(pq1), __float_as_int(pq2), 0);
            }
            pp_compute<DT>(tr, rs, Y, s_b, s_bg, p);
            const float sig = density_f(p.x, tr.relu);
            const float od = sig * delta;
            float a, e_od;
            absorb(od, a, e_od);
            const float wt = Tr * a;
            const float c0 = sigmoid_f(p.z0), c1 = sigmoid_f(p.z1), c2 = sigmoid_f(p.z2);
            acc0 = fmaf(wt, c0, acc0);
            acc1 = fmaf(wt, c1, acc1);
            acc2 = fmaf(wt, c2, acc2);
            wsum += wt;
            dsum = fmaf(wt, umid * rs.len_world, dsum);
            Tr *= e_od;
            ++ns;
            finish = t_stop > 0.0f && Tr < t_stop;
            if constexpr (TRACE) {
                if (cur >= 0) pslot = cur;
                pleaf = leaf; pdelta = delta; px = p.x; py = p.y; pc0 = c0; pc1 = c1; pc2 = c2;
                pp_dz_dgamma<DT>(p, Y, pq0, pq1, pq2);
            }
        }
        if (alive && finish) {
            out.rgb[3 * ray] = acc0; out.rgb[3 * ray + 1] = acc1; out.rgb[3 * ray + 2] = acc2;
            out.alpha[ray] = 1.0f - Tr;
            if (out.depth) out.depth[ray] = wsum > 0.0f ? dsum / wsum : INFINITY;
            out.nsamp[ray] = ns;
            if constexpr (TRACE) {
                if (t_first >= 0) {
                    int4* dst = out.trace.smp + kPPTraceInt4 * (int64_t)pslot;
                    dst[0] = make_int4(pleaf, __float_as_int(pdelta), __float_as_int(px), __float_as_int(py));
                    dst[1] = make_int4(__float_as_int(pc0), __float_as_int(pc1), __float_as_int(pc2), -1);
                    dst[2] = make_int4(__float_as_int(pq0), __float_as_int(pq1), __float_as_int(pq2), 0);
                }
                out.trace.head[ray] = t_first >= 0 ? t_first : -1;
            }
            alive = false;
        }
    }
}

// ----------------------------------------------------------------------------
// adjoint
//
// A sample's gradient row has 3K + C + CG = 104 values (two 64-lane atomics):
// lane component c < 42 is d/dhh = gz_ch h_k, 42 <= c < 73 d/dwsig = gx b,
// 73 <= c < 104 d/dwgam = gy bg, with gy = dL/dgamma * pi sigmoid'(y) and
// dL/dgamma = sum_ch gz_ch sum_k W_ch,k g'_nl(gamma) Y_k. The sample's h is
// passed to the other lanes through LDS; the basis gradients are summed by
// the lanes that own the density and hyperangle components, each reading the
// source leaf's weight from cache (it was loaded just before).

// Component of lane slot j (0, 1) of the gradient row.
__device__ __forceinline__ int pp_component(int j, int lane) { return j * kWave + lane; }

// REPLAY: every ray of the launch has a trace in io.trace (the forward's
// samples) and replays it without walking the tree or reading the leaf
// payload: dL/dgamma = sum_ch gz_ch dz_ch/dgamma comes from the traced
// derivatives, and h is recomputed from y only for samples without a record.
template <int DT, bool IDENT, bool REPLAY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(REPLAY ? 3 : 2, 8))) void render_pp_bwd_kernel(
    TreeArgs tr, InstArgs in, RayArgs ra, BackwardIO io, RecordArgs rec) {
    if (no_candidates(ra)) return;
    using namespace pp;
    __shared__ float s_h[kBlock * K];
    __shared__ float s_brow[C], s_bgrow[CG];
    __shared__ float s_acc[2 * kWave];   // block sum of the lanes' basis-gradient components
    const bool common_t = ra.t == nullptr;
    if (common_t) stage_common_rows(tr, in, ra.t_scalar, s_brow, s_bgrow);
    if (threadIdx.x < 2 * kWave) s_acc[threadIdx.x] = 0.0f;
    __syncthreads();
    const float* s_b = common_t ? s_brow : nullptr;
    const float* s_bg = common_t ? s_bgrow : nullptr;
    ChunkCursor cc = chunk_cursor();
    bool more = true;
    const int64_t N = tr.n_leaves;
    int tnext = -1;   // replay: the ray's next sample
    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x - lane;

    bool alive = false;
    int64_t ray = -1;
    RaySetup rs;
    Walk w;
    float Y[8];
    float Tr = 1.0f, Tfin = 0.0f, p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, F0 = 0.0f, F1 = 0.0f, F2 = 0.0f;
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, ga = 0.0f;
    int ns = 0, ns_fwd = 0;
    // scalar time: lane c < C holds component c of the density-basis gradient
    // (bacc[0]) and, c < CG, of the hyperangle-basis gradient (bacc[1])
    float bacc[2] = {0.0f, 0.0f};
    // records (scalar time only): [wrec, wend) is what is left of the
    // wavefront's current block of records (wave-uniform)
    int wrec = 0, wend = 0;

    for (;;) {
        const uint64_t idle = __ballot(!alive);
        const int n_idle = __popcll(idle);
        if (more && (n_idle >= ra.refill_min || n_idle == kWave)) {
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
                const float t = ra.t ? ra.t[ray] : ra.t_scalar;
                ray_setup<IDENT>(tr, in, o, d, t, rs);
                if (rs.hit) {
                    sh_deg2(rs.dir[0], rs.dir[1], rs.dir[2], Y);
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
                    alive = true;
                }
            }
            continue;
        }
        if (n_idle == kWave) break;
        bool has = false;
        int leaf = -1, my_rec = -1;
        float gz0 = 0.0f, gz1 = 0.0f, gz2 = 0.0f, gx = 0.0f, gy = 0.0f, y = 0.0f;
        if (alive) {
            float delta = 0.0f, x = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, q0 = 0.0f, q1 = 0.0f, q2 = 0.0f;
            bool finish;
            if constexpr (REPLAY) {
                // replay the forward's sample
                if (tnext >= 0) {
                    const int4* e = io.trace.smp + kPPTraceInt4 * (int64_t)tnext;
                    const int4 A = e[0], B = e[1], Q = e[2];
                    leaf = A.x;
                    delta = __int_as_float(A.y);
                    x = __int_as_float(A.z);
                    y = __int_as_float(A.w);
                    c0 = __int_as_float(B.x);
                    c1 = __int_as_float(B.y);
                    c2 = __int_as_float(B.z);
                    tnext = B.w;
                    q0 = __int_as_float(Q.x);
                    q1 = __int_as_float(Q.y);
                    q2 = __int_as_float(Q.z);
                }
                finish = leaf < 0;
            } else {
                float umid;
                leaf = walk_next<kWalkBudgetBwd>(tr, rs, w, delta, umid);
                finish = leaf == -1;
                if (leaf >= 0) {
                    PPSample<DT> p;
                    pp_load<DT>(tr, leaf, p);
                    pp_compute<DT>(tr, rs, Y, s_b, s_bg, p);
                    x = p.x;
                    y = p.y;
                    c0 = sigmoid_f(p.z0);
                    c1 = sigmoid_f(p.z1);
                    c2 = sigmoid_f(p.z2);
                    pp_dz_dgamma<DT>(p, Y, q0, q1, q2);
#pragma unroll
                    for (int k = 0; k < K; ++k) s_h[threadIdx.x * K + k] = p.h[k];
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
                const float gsig = delta * (Tn * gdotc - gsuf) + ga * delta * Tfin;
                gx = gsig * density_dx(x, tr.relu);
                gz0 = g0 * wt * c0 * (1.0f - c0);
                gz1 = g1 * wt * c1 * (1.0f - c1);
                gz2 = g2 * wt * c2 * (1.0f - c2);
                // dL/dgamma through every h_k = g_nl(gamma) Y_k
                const float ggam = gz0 * q0 + gz1 * q1 + gz2 * q2;
                const float sg = sigmoid_f(y);
                gy = ggam * kPi * sg * (1.0f - sg);
                has = true;
                Tr = Tn;
                ++ns;
                finish = ns >= ns_fwd;
            }
            if (finish) alive = false;
        }
        if (rec.head) {
            // records: this iteration's samples take consecutive records in lane
            // order; their leaf rows and basis gradients are summed per leaf later
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
                    rec.rec[2 * (int64_t)my_rec + 1] = make_int4(nxt, (int)ray, __float_as_int(gy), 0);
                }
            }
        }
        // samples without a record: basis gradients and the atomic row scatter
        has = has && my_rec < 0;
        if constexpr (REPLAY) {
            if (has) {
                // the sample's basis h, for the scatter below (Eq. 2-4, 6)
                float g[6], dg[6], h[K], sn, cs;
                sincosf(kPi * sigmoid_f(y), &sn, &cs);
                radial_n2(sn, cs, g, dg);
                hh14(g, Y, h);
#pragma unroll
                for (int k = 0; k < K; ++k) s_h[threadIdx.x * K + k] = h[k];
            }
        }
        uint64_t m = __ballot(has);
        if (common_t && m) {
            // basis gradients of this step: sum over the wavefront's samples of
            // gx wsig_c and gy wgam_c (butterfly), lane c keeping component c;
            // the weights are read again here (from cache) rather than held
            float sv[C], gv[CG];
            if (has) {
                load_leaf<DT, C>(tr.wsig, N, leaf, tr.layout, sv);
                load_leaf<DT, CG>(tr.wgam, N, leaf, tr.layout, gv);
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c) sv[c] = 0.0f;
#pragma unroll
                for (int c = 0; c < CG; ++c) gv[c] = 0.0f;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float v = gx * sv[c];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                if (lane == c) bacc[0] += v;
            }
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                float v = gy * gv[c];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                if (lane == c) bacc[1] += v;
            }
        }
        __builtin_amdgcn_wave_barrier();
        while (m) {
            const int src = __builtin_ctzll(m);
            m &= m - 1;
            const int L = __builtin_amdgcn_readlane(leaf, src);
            const float a0 = readlane_f(gz0, src), a1 = readlane_f(gz1, src), a2 = readlane_f(gz2, src);
            const float ax = readlane_f(gx, src), ay = readlane_f(gy, src);
            int i0 = 0, i1 = 0;
            float f = 0.0f;
            if (!common_t) {
                i0 = __builtin_amdgcn_readlane(rs.i0, src);
                i1 = __builtin_amdgcn_readlane(rs.i1, src);
                f = readlane_f(rs.f, src);
            }
            float* row = io.grad_leaf + (int64_t)L * ROW;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int c = pp_component(j, lane);
                if (c < 3 * K) {
                    const int ch = c / K;
                    const float gzc = ch == 0 ? a0 : (ch == 1 ? a1 : a2);
                    unsafeAtomicAdd(row + c, gzc * s_h[(wbase + src) * K + (c - ch * K)]);
                } else if (c < 3 * K + C + CG) {
                    const bool dens = c < 3 * K + C;
                    const int e = dens ? c - 3 * K : c - 3 * K - C;
                    const float gsrc = dens ? ax : ay;
                    const float* B = dens ? tr.basis : tr.basis_g;
                    const int R = dens ? C : CG;
                    const float be = common_t ? (dens ? s_brow[e] : s_bgrow[e])
                                              : (1.0f - f) * B[(int64_t)i0 * R + e] + f * B[(int64_t)i1 * R + e];
                    unsafeAtomicAdd(row + c, gsrc * be);
                    float* gB = dens ? io.grad_basis : io.grad_basis_g;
                    if (!common_t && gB) {
                        // a time per ray: this sample's rows of the basis gradient
                        const float wl = dens ? leaf_elem<DT, C>(tr.wsig, N, L, e, tr.layout)
                                              : leaf_elem<DT, CG>(tr.wgam, N, L, e, tr.layout);
                        const float v = gsrc * wl;
                        unsafeAtomicAdd(gB + (int64_t)i0 * R + e, (1.0f - f) * v);
                        if (f != 0.0f) unsafeAtomicAdd(gB + (int64_t)i1 * R + e, f * v);
                    }
                }
            }
        }
    }
    // one shared time: sum the wavefronts' components over the block, then
    // spread them over the two interpolated rows
    if (common_t) {
        if (lane < C) atomicAdd(&s_acc[lane], bacc[0]);
        if (lane < CG) atomicAdd(&s_acc[kWave + lane], bacc[1]);
        __syncthreads();
        const int c = threadIdx.x;
        const bool dens = c < C;
        const bool gam = c >= kWave && c < kWave + CG;
        float* gB = dens ? io.grad_basis : io.grad_basis_g;
        if ((dens || gam) && gB) {
            const int e = dens ? c : c - kWave;
            const int R = dens ? C : CG;
            int i0, i1;
            float f;
            time_setup(tr, in, ra.t_scalar, i0, i1, f);
            const float v = s_acc[c];
            unsafeAtomicAdd(gB + (int64_t)i0 * R + e, (1.0f - f) * v);
            if (f != 0.0f) unsafeAtomicAdd(gB + (int64_t)i1 * R + e, f * v);
        }
    }
}

// ----------------------------------------------------------------------------
// second pass of the two-phase adjoint (scalar time)
//
// One lane per leaf, with lane refill as in the global form. With one time
// for every ray the leaf's hyperangle gamma, hence its radial factors g, are
// the same for all its samples: they are computed once when the lane takes
// the leaf. Per record the lane redoes the ray's direction and its degree-2
// harmonics Y (the adjoint's functions and inputs), forms h = hh14(g, Y) and
// adds gz_ch h_k; the density and hyperangle parts of the row are
// (sum gx) B(tau) and (sum gy) B^gamma(tau), and the basis gradients
// (sum gx) w^sigma and (sum gy) w^gamma, so only the 42 HH sums and the two
// scalar sums are held.

template <int DT, bool IDENT>
__global__ __launch_bounds__(kBlock) void reduce_pp_records_kernel(TreeArgs tr, InstArgs in, RayArgs ra,
                                                                   RecordArgs rec, BackwardIO io) {
    using namespace pp;
    constexpr int R = 3 * K + 2;   // HH sums, sum gx, sum gy
    // a finished leaf's slot: its sums, then its w^sigma and w^gamma rows
    __shared__ float s_row[kBlock / kWave][kFlushSlots][R + C + CG + 1];
    __shared__ float s_brow[C], s_bgrow[CG];
    __shared__ float s_acc[2 * kWave];
    stage_common_rows(tr, in, ra.t_scalar, s_brow, s_bgrow);
    if (threadIdx.x < 2 * kWave) s_acc[threadIdx.x] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    int leaf = -1;
    int4 ra0 = make_int4(0, 0, 0, 0), ra1 = make_int4(-1, 0, 0, 0);
    float g[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) g[q] = 0.0f;
    float acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = 0.0f;
    float bacc[2] = {0.0f, 0.0f};   // lane c: components c of the two basis gradients
    LeafFeeder feeder = leaf_feeder(wv);
    __shared__ int2 s_q[kBlock / kWave][kWave];

    for (;;) {
        // hand leaves with records to idle lanes; a lane that got one loads its
        // first record and computes the leaf's radial factors
        int first = -1;
        feed_leaves(feeder, rec, tr.n_leaves, s_q[wv], leaf, first);
        if (first >= 0) {
            ra0 = rec.rec[2 * (int64_t)first];
            ra1 = rec.rec[2 * (int64_t)first + 1];
            float gv[CG];
            load_leaf<DT, CG>(tr.wgam, tr.n_leaves, leaf, tr.layout, gv);
            float y = 0.0f;
#pragma unroll
            for (int c = 0; c < CG; ++c) y = fmaf(gv[c], s_bgrow[c], y);
            const float gam = kPi * sigmoid_f(y);
            float sn, cs, dg[6];
            sincosf(gam, &sn, &cs);
            radial_n2(sn, cs, g, dg);
        }
        if (!__ballot(leaf >= 0)) break;
        bool done = false;
        if (leaf >= 0) {
            const int nxt = ra1.x;
            const int64_t ray = ra1.y;
            int4 nx0 = make_int4(0, 0, 0, 0), nx1 = make_int4(-1, 0, 0, 0);
            if (nxt >= 0) {
                nx0 = rec.rec[2 * (int64_t)nxt];
                nx1 = rec.rec[2 * (int64_t)nxt + 1];
            }
            const float gz0 = __int_as_float(ra0.x), gz1 = __int_as_float(ra0.y), gz2 = __int_as_float(ra0.z);
            const f3v dv = load3(ra.d + 3 * ray);
            const float d[3] = {dv.x, dv.y, dv.z};
            RaySetup rs;
            float dmax;
            ray_direction<IDENT>(in, d, rs, dmax);
            float Y[8], h[K];
            sh_deg2(rs.dir[0], rs.dir[1], rs.dir[2], Y);
            hh14(g, Y, h);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                acc[k] = fmaf(gz0, h[k], acc[k]);
                acc[K + k] = fmaf(gz1, h[k], acc[K + k]);
                acc[2 * K + k] = fmaf(gz2, h[k], acc[2 * K + k]);
            }
            acc[3 * K] += __int_as_float(ra0.w);
            acc[3 * K + 1] += __int_as_float(ra1.z);
            ra0 = nx0;
            ra1 = nx1;
            done = nxt < 0;
        }
        uint64_t dm = __ballot(done);
        while (dm) {
            const int r = lane_rank(dm);
            const bool mine = ((dm >> lane) & 1ull) && r < kFlushSlots;
            if (mine) {
                // the weights for the basis gradients, loaded by all finishing
                // lanes at once rather than one leaf at a time below
                float sv[C], gv[CG];
                load_leaf<DT, C>(tr.wsig, tr.n_leaves, leaf, tr.layout, sv);
                load_leaf<DT, CG>(tr.wgam, tr.n_leaves, leaf, tr.layout, gv);
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    s_row[wv][r][c] = acc[c];
                    acc[c] = 0.0f;
                }
#pragma unroll
                for (int c = 0; c < C; ++c) s_row[wv][r][R + c] = sv[c];
#pragma unroll
                for (int c = 0; c < CG; ++c) s_row[wv][r][R + C + c] = gv[c];
            }
            uint64_t sm = __ballot(mine);
            __builtin_amdgcn_wave_barrier();
            for (int q = 0; sm; ++q) {
                const int j = __builtin_ctzll(sm);
                sm &= sm - 1;
                const int L = __builtin_amdgcn_readlane(leaf, j);
                const float sgx = s_row[wv][q][3 * K], sgy = s_row[wv][q][3 * K + 1];
                float* row = io.grad_leaf + (int64_t)L * ROW;
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) {
                    const int c = pp_component(jj, lane);
                    if (c < 3 * K) unsafeAtomicAdd(row + c, s_row[wv][q][c]);
                    else if (c < 3 * K + C) unsafeAtomicAdd(row + c, sgx * s_brow[c - 3 * K]);
                    else if (c < 3 * K + C + CG) unsafeAtomicAdd(row + c, sgy * s_bgrow[c - 3 * K - C]);
                }
                if (lane < C) bacc[0] = fmaf(sgx, s_row[wv][q][R + lane], bacc[0]);
                if (lane < CG) bacc[1] = fmaf(sgy, s_row[wv][q][R + C + lane], bacc[1]);
            }
            __builtin_amdgcn_wave_barrier();
            if (mine) leaf = -1;
            dm = __ballot(done && leaf >= 0);
        }
    }
    // basis gradients: sum over the block, spread over the two interpolated rows
    if (lane < C) atomicAdd(&s_acc[lane], bacc[0]);
    if (lane < CG) atomicAdd(&s_acc[kWave + lane], bacc[1]);
    __syncthreads();
    const int c = threadIdx.x;
    const bool dens = c < C;
    const bool gam = c >= kWave && c < kWave + CG;
    float* gB = dens ? io.grad_basis : io.grad_basis_g;
    if ((dens || gam) && gB) {
        const int e = dens ? c : c - kWave;
        const int Rb = dens ? C : CG;
        int i0, i1;
        float f;
        time_setup(tr, in, ra.t_scalar, i0, i1, f);
        const float v = s_acc[c];
        unsafeAtomicAdd(gB + (int64_t)i0 * Rb + e, (1.0f - f) * v);
        if (f != 0.0f) unsafeAtomicAdd(gB + (int64_t)i1 * Rb + e, f * v);
    }
}

// ----------------------------------------------------------------------------
// launchers

template <int DT, bool TRACE>
static hipError_t pp_fwd_e(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, float t_stop,
                           const RenderOut& o, hipStream_t st) {
    if constexpr (TRACE) {
        // the trace's allocation counters start at zero
        hipLaunchKernelGGL(zero_queue_kernel, dim3(1), dim3(kQueues * kQueueStride), 0, st, o.trace.counter);
    }
    if (in.identity) {
        auto kern = render_pp_fwd_kernel<DT, true, TRACE>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, ra)), dim3(kBlock), 0, st, tr, in, ra, t_stop, o);
    } else {
        auto kern = render_pp_fwd_kernel<DT, false, TRACE>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, ra)), dim3(kBlock), 0, st, tr, in, ra, t_stop, o);
    }
    return hipGetLastError();
}

template <int DT>
static hipError_t pp_fwd_t(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, float t_stop,
                           const RenderOut& o, hipStream_t st) {
    return o.trace.head ? pp_fwd_e<DT, true>(tr, in, ra, t_stop, o, st) : pp_fwd_e<DT, false>(tr, in, ra, t_stop, o, st);
}

template <int DT, bool REPLAY>
static hipError_t pp_bwd_k(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, const BackwardIO& io,
                           const RecordArgs& rec, hipStream_t st) {
    if (in.identity) {
        auto kern = render_pp_bwd_kernel<DT, true, REPLAY>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, ra)), dim3(kBlock), 0, st, tr, in, ra, io, rec);
    } else {
        auto kern = render_pp_bwd_kernel<DT, false, REPLAY>;
        hipLaunchKernelGGL(kern, dim3(grid_for(kern, ra)), dim3(kBlock), 0, st, tr, in, ra, io, rec);
    }
    return hipGetLastError();
}

template <int DT>
static hipError_t pp_bwd_t(const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, const BackwardIO& io,
                           hipStream_t st) {
    // records with one time for every ray (the per-leaf sums rely on it)
    const int64_t cap = ra.t == nullptr && ra.n <= (int64_t)INT32_MAX && tr.n_leaves > 0 &&
                                tr.n_leaves <= (int64_t)INT32_MAX
                            ? io.record_cap
                            : 0;
    RecordArgs rec{};
    void* mem = nullptr;
    hipError_t e = records_begin(tr, cap, st, rec, mem);
    if (e == hipSuccess) {
        // one cull pass and adjoint per source of samples: rays that walk, and
        // (traced forward) rays that replay their trace
        auto walk = [&](const RayArgs& r) { return pp_bwd_k<DT, false>(tr, in, r, io, rec, st); };
        auto replay = [&](const RayArgs& r) { return pp_bwd_k<DT, true>(tr, in, r, io, rec, st); };
        // the walking adjoint's cull reads whether the forward's traces are all complete
        TraceArgs room = io.trace;
        room.cap = io.trace.cap / 2;   // two entries per sample
        const RenderOut trace_out{nullptr, nullptr, nullptr, nullptr, nullptr, room};
        if (io.trace.head) {
            if (ra.n > (int64_t)INT32_MAX) e = hipErrorInvalidValue;   // traced calls take candidate lists
            if (e == hipSuccess) e = with_candidates<2>(tr, in, ra, trace_out, io.nsamp, st, walk, io.trace.head);
            if (e == hipSuccess) e = with_candidates<3>(tr, in, ra, RenderOut{}, io.nsamp, st, replay, io.trace.head);
        } else {
            e = with_candidates<1>(tr, in, ra, RenderOut{}, io.nsamp, st, walk);
        }
    }
    if (e == hipSuccess && cap > 0) {
        int64_t blocks = (tr.n_leaves + kBlock - 1) / kBlock;
        const int64_t lim = (int64_t)device_cu_count() * 4;
        if (blocks > lim) blocks = lim;
        if (in.identity)
            hipLaunchKernelGGL((reduce_pp_records_kernel<DT, true>), dim3((unsigned)blocks), dim3(kBlock), 0, st, tr,
                               in, ra, rec, io);
        else
            hipLaunchKernelGGL((reduce_pp_records_kernel<DT, false>), dim3((unsigned)blocks), dim3(kBlock), 0, st,
                               tr, in, ra, rec, io);
        e = hipGetLastError();
    }
    if (mem) {
        const hipError_t f = work_free(mem, st);
        if (e == hipSuccess) e = f;
    }
    return e;
}

hipError_t launch_render_pp_fwd(int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra, float t_stop,
                                const RenderOut& out, hipStream_t stream, void* ws) {
    if (ra.n_slots <= 0) return hipSuccess;
    switch (dtype) {
        case 0: return with_candidates<0>(tr, in, ra, out, nullptr, stream, [&](const RayArgs& r) { return pp_fwd_t<0>(tr, in, r, t_stop, out, stream); }, nullptr, ws);
        case 1: return with_candidates<0>(tr, in, ra, out, nullptr, stream, [&](const RayArgs& r) { return pp_fwd_t<1>(tr, in, r, t_stop, out, stream); }, nullptr, ws);
        default: return with_candidates<0>(tr, in, ra, out, nullptr, stream, [&](const RayArgs& r) { return pp_fwd_t<2>(tr, in, r, t_stop, out, stream); }, nullptr, ws);
    }
}

hipError_t launch_render_pp_bwd(int dtype, const TreeArgs& tr, const InstArgs& in, const RayArgs& ra,
                                const BackwardIO& io, hipStream_t stream) {
    if (ra.n_slots <= 0) return hipSuccess;
    switch (dtype) {
        case 0: return pp_bwd_t<0>(tr, in, ra, io, stream);
        case 1: return pp_bwd_t<1>(tr, in, ra, io, stream);
        default: return pp_bwd_t<2>(tr, in, ra, io, stream);
    }
}

}  // namespace neuvv
