// Device-side building blocks of the VOctree renderer (gfx950).
//
//  * df:        compensated float32 pairs (hi + lo, about 48 significant bits)
//               used for all ray geometry, so that segment lengths inside
//               leaves keep float32 relative accuracy even when the ray
//               parameter is thousands of leaf units large;
//  * hh_all:    the first 30 real 4-D hyperspherical harmonics (Sec. 4.1,
//               Eq. 2-3, Appendix A.2) as closed-form polynomials;
//  * RaySetup:  instance transform and re-timing of one ray (Eq. 13), clip to
//               the tree box, per-ray HH basis and density-basis row (Eq. 4, 5);
//  * walk_next: the next occupied leaf along the ray (Sec. 4.3 "Rendering"),
//               skipping whole empty octree cubes; the octree is stored two
//               levels per node (64-bit occupancy mask + base index), a
//               directory maps each 4^3 region of leaf cells to its
//               last-level node (a "brick") or to the largest empty cube
//               around it, and the current brick's node is kept in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace neuvv {

constexpr int kMaxDepth = 12;
constexpr int kWave = 64;

// ----------------------------------------------------------------------------
// compensated float arithmetic (error-free transformations); contraction is
// switched off inside so that no a*b+c is fused behind the algorithm's back.

struct df {
    float hi, lo;
};

__device__ __forceinline__ df df_two_sum(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ df df_quick(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float e = b - (s - a);
    return {s, e};
}
__device__ __forceinline__ df df_two_prod(float a, float b) {
#pragma clang fp contract(off)
    float p = a * b;
    float e = __builtin_fmaf(a, b, -p);
    return {p, e};
}
__device__ __forceinline__ df df_from(float a) { return {a, 0.0f}; }
__device__ __forceinline__ df df_neg(df a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ df df_add(df a, df b) {
#pragma clang fp contract(off)
    df s = df_two_sum(a.hi, b.hi);
    df t = df_two_sum(a.lo, b.lo);
    float lo = s.lo + t.hi;
    df u = df_quick(s.hi, lo);
    lo = t.lo + u.lo;
    return df_quick(u.hi, lo);
}
__device__ __forceinline__ df df_sub(df a, df b) { return df_add(a, df_neg(b)); }
__device__ __forceinline__ df df_mul(df a, df b) {
#pragma clang fp contract(off)
    df p = df_two_prod(a.hi, b.hi);
    float cross = __builtin_fmaf(a.hi, b.lo, a.lo * b.hi);
    return df_quick(p.hi, p.lo + cross);
}
__device__ __forceinline__ df df_mul_f(df a, float b) {
#pragma clang fp contract(off)
    df p = df_two_prod(a.hi, b);
    return df_quick(p.hi, __builtin_fmaf(a.lo, b, p.lo));
}
__device__ __forceinline__ df df_div(df a, df b) {
#pragma clang fp contract(off)
    float q1 = a.hi / b.hi;
    df r = df_sub(a, df_mul_f(b, q1));
    float q2 = r.hi / b.hi;
    r = df_sub(r, df_mul_f(b, q2));
    float q3 = r.hi / b.hi;
    return df_add(df_quick(q1, q2), df_from(q3));
}
// 1/d: hardware reciprocal refined by one compensated Newton step (~46 bits).
__device__ __forceinline__ df df_rcp(df d) {
#pragma clang fp contract(off)
    const float r = __builtin_amdgcn_rcpf(d.hi);
    const float e = __builtin_fmaf(-d.hi, r, 1.0f) - d.lo * r;
    return df_quick(r, r * e);
}
__device__ __forceinline__ bool df_lt(df a, df b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ float df_f(df a) { return a.hi + a.lo; }

// floor of the value hi + lo (|lo| <= ulp(hi)/2).
__device__ __forceinline__ int df_floor(df a) {
    float f = floorf(a.hi);
    if (f == a.hi && a.lo < 0.0f) f -= 1.0f;
    return (int)f;
}
// Index of the half-open unit cell a ray occupies just after passing x along
// a direction of the given sign: floor(x) moving up (or still), ceil(x)-1 down.
__device__ __forceinline__ int df_cell(df a, int sign) {
    if (sign >= 0) return df_floor(a);
    float c = ceilf(a.hi);
    if (c == a.hi && a.lo > 0.0f) c += 1.0f;
    return (int)c - 1;
}

// ----------------------------------------------------------------------------
// Real 4-D hyperspherical harmonics H_nlm(d, gamma) = g_nl(gamma) Y_lm(d)
// with g_nl = A_nl sin^l(gamma) C^{l+1}_{n-l}(cos gamma), A_nl =
// (2l)!! sqrt(2 (n+1) (n-l)! / (pi (n+l+1)!)), and Y_lm the orthonormal real
// spherical harmonic of the unit direction d = (x, y, z), polar axis z, no
// Condon-Shortley phase (cos m phi for m > 0, sin |m| phi for m < 0). Order:
// n = 0.., l = 0..n, m = -l..l. Constants are the closed forms evaluated.
// Radial factors g_nl of the hyperangle gamma, n + l <= 3 (order g00, g10, g11,
// g20, g21, g22, g30, g31, g32, g33).
__device__ __forceinline__ void hh_radial(float gam, float (&g)[10]) {
    float s, c;
    sincosf(gam, &s, &c);
    const float c2 = c * c, s2 = s * s;
    g[0] = 0.7978845608028654f;                        // sqrt(2/pi)
    g[1] = 1.5957691216057308f * c;                    // 2 sqrt(2/pi) cos
    g[2] = 0.9213177319235613f * s;                    // 2 sqrt(2/(3pi)) sin
    g[3] = 0.7978845608028654f * (4.0f * c2 - 1.0f);   // sqrt(2/pi) U_2
    g[4] = 2.256758334191025f * s * c;                 // (1/sqrt(pi)) sin * 4 cos
    g[5] = 1.009253008808064f * s2;                    // 8/sqrt(20 pi) sin^2
    g[6] = 0.7978845608028654f * c * (8.0f * c2 - 4.0f);    // sqrt(2/pi) U_3
    g[7] = 0.41202581549140227f * s * (12.0f * c2 - 2.0f);  // 2 sqrt(2/(15pi)) sin C^2_2
    g[8] = 2.854598585844434f * c * s2;                // 8/sqrt(90 pi) sin^2 * 6 cos
    g[9] = 1.0789368501515768f * s2 * s;               // 48/sqrt(630 pi) sin^3
}

// The 30 HH values from the radial factors and the unit direction (x, y, z):
// h = g_nl Y_lm with real spherical harmonics up to degree 3.
__device__ __forceinline__ void hh_assemble(const float (&g)[10], float x, float y, float z, float (&h)[30]) {
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float Y00 = 0.28209479177387814f;
    const float k1 = 0.4886025119029199f;
    const float Y1n1 = k1 * y, Y10 = k1 * z, Y11 = k1 * x;
    const float k2 = 1.0925484305920792f;
    const float Y2n2 = k2 * x * y, Y2n1 = k2 * y * z, Y20 = 0.31539156525252005f * (3.0f * z2 - 1.0f);
    const float Y21 = k2 * x * z, Y22 = 0.5462742152960396f * (x2 - y2);
    const float k33 = 0.5900435899266435f, k31 = 0.4570457994644658f;
    const float Y3n3 = k33 * y * (3.0f * x2 - y2), Y3n2 = 2.890611442640554f * x * y * z;
    const float Y3n1 = k31 * y * (5.0f * z2 - 1.0f), Y30 = 0.3731763325901154f * z * (5.0f * z2 - 3.0f);
    const float Y31 = k31 * x * (5.0f * z2 - 1.0f), Y32 = 1.445305721320277f * z * (x2 - y2);
    const float Y33 = k33 * x * (x2 - 3.0f * y2);
    h[0] = g[0] * Y00;
    h[1] = g[1] * Y00;
    h[2] = g[2] * Y1n1; h[3] = g[2] * Y10; h[4] = g[2] * Y11;
    h[5] = g[3] * Y00;
    h[6] = g[4] * Y1n1; h[7] = g[4] * Y10; h[8] = g[4] * Y11;
    h[9] = g[5] * Y2n2; h[10] = g[5] * Y2n1; h[11] = g[5] * Y20; h[12] = g[5] * Y21; h[13] = g[5] * Y22;
    h[14] = g[6] * Y00;
    h[15] = g[7] * Y1n1; h[16] = g[7] * Y10; h[17] = g[7] * Y11;
    h[18] = g[8] * Y2n2; h[19] = g[8] * Y2n1; h[20] = g[8] * Y20; h[21] = g[8] * Y21; h[22] = g[8] * Y22;
    h[23] = g[9] * Y3n3; h[24] = g[9] * Y3n2; h[25] = g[9] * Y3n1; h[26] = g[9] * Y30;
    h[27] = g[9] * Y31; h[28] = g[9] * Y32; h[29] = g[9] * Y33;
}

__device__ __forceinline__ void hh_all(float x, float y, float z, float gam, float (&h)[30]) {
    float g[10];
    hh_radial(gam, g);
    hh_assemble(g, x, y, z, h);
}

// Per-point hyperangle form (Eq. 6), first 14 functions (all n <= 2): the
// direction factors are per ray, the radial factors per sample.
// Y = (Y1-1, Y10, Y11, Y2-2, Y2-1, Y20, Y21, Y22) of the unit direction; Y00 is
// the constant 1 / (2 sqrt(pi)).
constexpr float kY00 = 0.28209479177387814f;
__device__ __forceinline__ void sh_deg2(float x, float y, float z, float (&Y)[8]) {
    const float k1 = 0.4886025119029199f, k2 = 1.0925484305920792f;
    Y[0] = k1 * y; Y[1] = k1 * z; Y[2] = k1 * x;
    Y[3] = k2 * x * y; Y[4] = k2 * y * z; Y[5] = 0.31539156525252005f * (3.0f * z * z - 1.0f);
    Y[6] = k2 * x * z; Y[7] = 0.5462742152960396f * (x * x - y * y);
}
// g = (g00, g10, g11, g20, g21, g22)(gamma) and their derivatives in gamma,
// from s = sin(gamma), c = cos(gamma); same closed forms as hh_all.
__device__ __forceinline__ void radial_n2(float s, float c, float (&g)[6], float (&dg)[6]) {
    const float a0 = 0.7978845608028654f, a1 = 1.5957691216057308f, b1 = 0.9213177319235613f;
    const float d1 = 2.256758334191025f, e2 = 1.009253008808064f;
    g[0] = a0;                         dg[0] = 0.0f;
    g[1] = a1 * c;                     dg[1] = -a1 * s;
    g[2] = b1 * s;                     dg[2] = b1 * c;
    g[3] = a0 * (4.0f * c * c - 1.0f); dg[3] = -8.0f * a0 * c * s;
    g[4] = d1 * s * c;                 dg[4] = d1 * (c * c - s * s);
    g[5] = e2 * s * s;                 dg[5] = 2.0f * e2 * s * c;
}
// h_k = g_{n(k) l(k)} Y_{l(k) m(k)} in the canonical order of the first 14.
__device__ __forceinline__ void hh14(const float (&g)[6], const float (&Y)[8], float (&h)[14]) {
    h[0] = g[0] * kY00;
    h[1] = g[1] * kY00;
    h[2] = g[2] * Y[0]; h[3] = g[2] * Y[1]; h[4] = g[2] * Y[2];
    h[5] = g[3] * kY00;
    h[6] = g[4] * Y[0]; h[7] = g[4] * Y[1]; h[8] = g[4] * Y[2];
    h[9] = g[5] * Y[3]; h[10] = g[5] * Y[4]; h[11] = g[5] * Y[5]; h[12] = g[5] * Y[6]; h[13] = g[5] * Y[7];
}

// ----------------------------------------------------------------------------
// kernel-side descriptions of the tree, instance and rays

struct TreeArgs {
    const int4* nodes;   // [n_nodes] {mask lo, mask hi, first child, 0}
    const void* hh;
    const void* wsig;
    const float* basis;
    const float* gamma;
    int64_t n_nodes;
    int64_t n_leaves;
    int32_t depth;
    int32_t T;
    int32_t box_lo[3];   // occupied-cell bounds: rays are clipped to [lo, hi)
    int32_t box_hi[3];
    int32_t layout;      // 0: vectors structure-of-arrays, 1: leaf-major rows of vectors
    int32_t Cg;          // per-point hyperangle weights per leaf (0: the global table gamma)
    const void* wgam;    // [N] rows of Cg weights, storage dtype and layout of wsig
    const float* basis_g;   // [T][Cg] hyperangle basis
    const float4* edit;     // nullptr, or [N][2] rows {r, g, b, sigma_d}, {t_d, owner, 0, 0} (appearance edits)
    int32_t relu;           // density activation of Eq. 5: 0 softplus, 1 ReLU
    const int32_t* dir;     // brick directory (directory_entries(depth) entries; see walk_next)
};

struct InstArgs {
    float rot[9];
    float trans[3];
    float scale;
    float time_offset;
    int32_t wrap;
    int32_t identity;
};

struct RayArgs {
    const float* o;
    const float* d;
    const float* t;      // nullptr: t_scalar for every ray
    float t_scalar;
    int32_t img_w;       // > 0: rays form a row-major image of this width
    int32_t tiles_x;
    int64_t n;
    int64_t n_slots;     // work slots (64 per 8x8 tile when img_w > 0, else n)
    int32_t refill_min;  // idle lanes that trigger a refill of the wavefront
    unsigned long long* queue;   // work-queue counters of the launch (set by the launcher)
    // candidate form (set by the launcher): the rays a cull pass kept, listed in
    // the slot range of their XCD part, with the per-part counts; nullptr: the
    // work items are the slots themselves
    const int32_t* list;
    const unsigned long long* count;
};

// Work slot -> ray index, -1 when the slot is padding of a ragged tile.
__device__ __forceinline__ int64_t slot_to_ray(const RayArgs& ra, int64_t slot) {
    if (ra.img_w <= 0) return slot < ra.n ? slot : -1;
    int64_t tile = slot >> 6;
    int within = (int)(slot & 63);
    int64_t ty = tile / ra.tiles_x, tx = tile - ty * ra.tiles_x;
    int64_t px = tx * 8 + (within & 7), py = ty * 8 + (within >> 3);
    if (px >= ra.img_w) return -1;
    int64_t r = py * ra.img_w + px;
    return r < ra.n ? r : -1;
}

// Per-ray constants: local ray x_l(u) = O + u D with the world parameter u,
// reciprocal direction, box interval [u_in, u_out), frame interpolation.
struct RaySetup {
    df O[3], D[3], inv[3];
    int sgn[3];
    df u_in, u_out;
    float len_local;   // |D|: leaf units per unit of u
    float len_world;   // |d|: world distance per unit of u
    float dir[3];      // unit local direction
    int i0, i1;
    float f;
    float tau;         // local time after re-timing (appearance edits are gated on it)
    bool hit;
};

// Re-timing (Eq. 13): tau = t + offset, wrapped into [0, T) or clamped into
// [0, T-1]; frames i0 = floor(tau), i1 = min(i0 + 1, T - 1), weight f = tau - i0
// (0 on the held last frame). tau is kept compensated so f is accurate.
__device__ __forceinline__ void time_setup(const TreeArgs& tr, const InstArgs& in, float t, int& i0_out,
                                           int& i1_out, float& f_out, float* tau_out = nullptr) {
    const int T = tr.T;
    const float Tf = (float)T;
    df tau = df_two_sum(t, in.time_offset);
    if (in.wrap) {
        float k = floorf(tau.hi / Tf);
        tau = df_sub(tau, df_two_prod(k, Tf));
        if (df_lt(tau, df_from(0.0f))) tau = df_add(tau, df_from(Tf));
        if (!df_lt(tau, df_from(Tf))) tau = df_sub(tau, df_from(Tf));
        if (df_lt(tau, df_from(0.0f))) tau = df_from(0.0f);
    } else {
        if (df_lt(tau, df_from(0.0f))) tau = df_from(0.0f);
        if (df_lt(df_from(Tf - 1.0f), tau)) tau = df_from(Tf - 1.0f);
    }
    int i0 = df_floor(tau);
    i0 = i0 < 0 ? 0 : (i0 > T - 1 ? T - 1 : i0);
    float f = df_f(df_sub(tau, df_from((float)i0)));
    if (i0 == T - 1) f = 0.0f;
    i0_out = i0;
    i1_out = i0 + 1 < T ? i0 + 1 : T - 1;
    f_out = f;
    if (tau_out) *tau_out = df_f(tau);
}

// IDENT: the instance is the identity (known at compile time), so the local
// ray is the world ray and the low parts of O and D are constant zeros.
// Coarse reject in plain float against the occupied box grown by one leaf on
// every side: float rounding of the clip is far below that margin for any
// local coordinate below ~1e5, so a ray rejected here misses the exact box.
// Returns false only for such rays.
template <bool IDENT>
__device__ __forceinline__ bool ray_may_hit(const TreeArgs& tr, const InstArgs& in, const float o[3],
                                            const float d[3]) {
    float of[3], dfl[3];
    if constexpr (IDENT) {
#pragma unroll
        for (int a = 0; a < 3; ++a) { of[a] = o[a]; dfl[a] = d[a]; }
    } else {
        const float is = 1.0f / in.scale;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            of[a] = ((o[0] - in.trans[0]) * in.rot[a] + (o[1] - in.trans[1]) * in.rot[3 + a] +
                     (o[2] - in.trans[2]) * in.rot[6 + a]) * is;
            dfl[a] = (d[0] * in.rot[a] + d[1] * in.rot[3 + a] + d[2] * in.rot[6 + a]) * is;
        }
    }
    float tn = 0.0f, tf = INFINITY;
    bool pass = true, small = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        small = small && fabsf(of[a]) < 1.0e5f;
        const float lo = (float)tr.box_lo[a] - 1.0f, hi = (float)tr.box_hi[a] + 1.0f;
        if (dfl[a] == 0.0f) {
            pass = pass && of[a] >= lo && of[a] < hi;
        } else {
            const float iv = __builtin_amdgcn_rcpf(dfl[a]);   // 1 ulp: far inside the margin
            const float t0 = (lo - of[a]) * iv, t1 = (hi - of[a]) * iv;
            tn = fmaxf(tn, fminf(t0, t1));
            tf = fminf(tf, fmaxf(t0, t1));
        }
    }
    return !small || (pass && tn < tf);
}

// Local direction of a ray (compensated D = R^T d / s), |D| (leaf units per
// unit of the ray parameter), |d| and the unit local direction; dmax = the
// largest |D| component.
template <bool IDENT>
__device__ __forceinline__ void ray_direction(const InstArgs& in, const float d[3], RaySetup& rs, float& dmax) {
    if constexpr (IDENT) {
#pragma unroll
        for (int a = 0; a < 3; ++a) rs.D[a] = df_from(d[a]);
    } else {
        df s = df_from(in.scale);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            df ad = df_two_prod(d[0], in.rot[a]);
            ad = df_add(ad, df_two_prod(d[1], in.rot[3 + a]));
            ad = df_add(ad, df_two_prod(d[2], in.rot[6 + a]));
            rs.D[a] = df_div(ad, s);
        }
    }
    float dl2 = 0.0f, dw2 = 0.0f;
    dmax = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float v = df_f(rs.D[a]);
        dl2 += v * v;
        dw2 += d[a] * d[a];
        dmax = fmaxf(dmax, fabsf(v));
    }
    rs.len_local = sqrtf(dl2);
    rs.len_world = sqrtf(dw2);
    const float inv_len = rs.len_local > 0.0f ? 1.0f / rs.len_local : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) rs.dir[a] = df_f(rs.D[a]) * inv_len;
    if (!(rs.len_local > 0.0f)) rs.dir[2] = 1.0f;
}

// Exact per-ray setup (compensated geometry); call for rays ray_may_hit accepts.
template <bool IDENT>
__device__ __forceinline__ void ray_setup(const TreeArgs& tr, const InstArgs& in, const float o[3],
                                          const float d[3], float t, RaySetup& rs) {
    float dmax;
    ray_direction<IDENT>(in, d, rs, dmax);
    if constexpr (IDENT) {
#pragma unroll
        for (int a = 0; a < 3; ++a) rs.O[a] = df_from(o[a]);
    } else {
        df diff[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) diff[b] = df_two_sum(o[b], -in.trans[b]);
        df s = df_from(in.scale);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            df ao = df_mul_f(diff[0], in.rot[a]);
            ao = df_add(ao, df_mul_f(diff[1], in.rot[3 + a]));
            ao = df_add(ao, df_mul_f(diff[2], in.rot[6 + a]));
            rs.O[a] = df_div(ao, s);
        }
    }
    bool hit = rs.len_local > 0.0f;
    // clip to the occupied-cell box [lo, hi) (no occupied cell lies outside it).
    // Direction components below 1e-20 of the largest are treated as zero: their
    // plane crossings lie beyond any representable ray parameter.
    df u_in = df_from(0.0f), u_out = df_from(0.0f);
    bool have_out = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool zero = fabsf(rs.D[a].hi) <= 1.0e-20f * dmax;
        rs.sgn[a] = zero ? 0 : (rs.D[a].hi > 0.0f ? 1 : -1);
        const float lo_p = (float)tr.box_lo[a], hi_p = (float)tr.box_hi[a];
        if (rs.sgn[a] == 0) {
            if (df_lt(rs.O[a], df_from(lo_p)) || !df_lt(rs.O[a], df_from(hi_p))) hit = false;
            rs.inv[a] = df_from(0.0f);
            continue;
        }
        rs.inv[a] = df_rcp(rs.D[a]);
        df t0 = df_mul(df_sub(df_from(lo_p), rs.O[a]), rs.inv[a]);
        df t1 = df_mul(df_sub(df_from(hi_p), rs.O[a]), rs.inv[a]);
        df lo = rs.sgn[a] > 0 ? t0 : t1, hi = rs.sgn[a] > 0 ? t1 : t0;
        if (df_lt(u_in, lo)) u_in = lo;
        if (!have_out || df_lt(hi, u_out)) { u_out = hi; have_out = true; }
    }
    if (!have_out || !df_lt(u_in, u_out)) hit = false;
    rs.u_in = u_in;
    rs.u_out = u_out;
    rs.hit = hit;
    time_setup(tr, in, t, rs.i0, rs.i1, rs.f, &rs.tau);
}

// ----------------------------------------------------------------------------
// octree walk

struct Walk {
    int cell[3];     // leaf-level cell containing the ray just after the entry point
    int steps;
    int entry_axis;  // the entry point is the crossing of plane entry_plane on this axis; -1: u_in
    int entry_plane;
    df u_entry;      // the exact entry parameter when u_entry_ok (the previous step computed it)
    bool u_entry_ok;
    bool done;
    int brick;       // directory entry of the brick whose node is held below, -1: none
    uint32_t bm_lo, bm_hi;
    int bbase;
};

// Node levels of a depth-D tree: L = ceil(D/2); level w is a cube of edge
// 2^node_edge(D, w) split into child cells of edge 2^(node_edge - node_bits).
__device__ __forceinline__ int node_bits(int D, int w) { return (w == 0 && (D & 1)) ? 1 : 2; }
__device__ __forceinline__ int node_edge(int D, int w) { return w == 0 ? D : D - (D & 1 ? 1 : 2) - 2 * (w - 1); }
// The brick directory: one int32 per 4^3 region of leaf cells, E^3 entries
// with E = 2^(D-2) (E = 1 for D <= 2, where the root is the only node),
// entry (k E + j) E + i for the region with corner (4i, 4j, 4k): the row of
// the region's last-level node when the region holds a leaf, else -(1 + s)
// where 2^s is the edge of the largest aligned cube around the region that
// holds no leaf, the cube at which a descent from the root would stop.
__host__ __device__ __forceinline__ int64_t directory_edge(int D) { return D <= 2 ? 1 : (int64_t)1 << (D - 2); }
__host__ __device__ __forceinline__ int64_t directory_entries(int D) {
    const int64_t e = directory_edge(D);
    return e * e * e;
}

__device__ __forceinline__ void walk_begin(const TreeArgs& tr, const RaySetup& rs, Walk& w) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        df p = df_add(rs.O[a], df_mul(rs.u_in, rs.D[a]));
        int c = df_cell(p, rs.sgn[a]);
        w.cell[a] = c < tr.box_lo[a] ? tr.box_lo[a] : (c > tr.box_hi[a] - 1 ? tr.box_hi[a] - 1 : c);
    }
    w.steps = 0;
    w.entry_axis = -1;
    w.entry_plane = 0;
    w.u_entry = rs.u_in;
    w.u_entry_ok = true;
    w.done = !rs.hit;
    w.brick = -1;
    w.bm_lo = w.bm_hi = 0u;
    w.bbase = 0;
}

// v[i] for a runtime i in [0, 3) without indexing a local array (which would
// place it in scratch memory).
#define NEUVV_SEL3(v, i) ((i) == 0 ? +(v)[0] : ((i) == 1 ? +(v)[1] : +(v)[2]))

// Exact (compensated) parameter at which the ray crosses the plane x_a = p.
__device__ __forceinline__ df crossing(const RaySetup& rs, int a, int p) {
    // branches over constant members (no address arithmetic), so rs stays in registers
    float oh, ol, ih, il;
    if (a == 0) {
        oh = rs.O[0].hi; ol = rs.O[0].lo; ih = rs.inv[0].hi; il = rs.inv[0].lo;
    } else if (a == 1) {
        oh = rs.O[1].hi; ol = rs.O[1].lo; ih = rs.inv[1].hi; il = rs.inv[1].lo;
    } else {
        oh = rs.O[2].hi; ol = rs.O[2].lo; ih = rs.inv[2].hi; il = rs.inv[2].lo;
    }
    return df_mul(df_sub(df_from((float)p), df{oh, ol}), df{ih, il});
}

__device__ __forceinline__ df entry_param(const RaySetup& rs, const Walk& w) {
    return w.entry_axis < 0 ? rs.u_in : crossing(rs, w.entry_axis, w.entry_plane);
}

// Advances to the next occupied leaf segment of positive length. Returns its
// slot and writes delta (leaf units), umid (ray parameter of the segment
// midpoint) and the segment's compensated bounds [seg_a, seg_b) in the ray
// parameter; returns -1 when the ray has left the box. With kBudget > 0 at
// most kBudget cells are visited per call, and -2 says that the budget ran out
// before a segment was found (the next call resumes the walk): lanes of a
// wavefront in long empty stretches then stop holding back the lanes that
// have a sample to evaluate.
//
// A cell visit reads nothing while the walk stays in the brick whose node it
// holds. Entering another 4^3 region, it reads the region's directory entry
// and, when the region holds a leaf, the brick's node row: at most two
// dependent loads, where a descent from the deepest common ancestor took up
// to one per node level (and a wavefront as many loop iterations as its
// deepest lane).
//
// Every decision of the walk (which face a node is left through, which cell
// the ray enters, whether it leaves the box) is taken on float estimates
// whose rounding error is bounded; only when an estimate falls within that
// bound of the decision threshold is it redone in compensated arithmetic.
// Segment lengths of leaves always come from compensated entry and exit
// parameters. The sequence of cells is therefore that of the exact walk.
template <int kBudget = 0>
__device__ __forceinline__ int walk_next(const TreeArgs& tr, const RaySetup& rs, Walk& w, float& delta,
                                         float& umid, df& seg_a, df& seg_b) {
    const int Dp = tr.depth;
    const int G = 1 << Dp;
    const int E = (int)directory_edge(Dp);
    const int max_steps = 3 * G + 16;
    constexpr float kRel = 1.0e-6f;   // bound on the relative error of a float estimate (~16 ulp)
    int budget = kBudget;
    while (!w.done) {
        if (kBudget > 0 && budget-- == 0) return -2;
        if (++w.steps > max_steps) { w.done = true; break; }
        // the cell's brick, or the empty cube around its region; sh = log2 of the
        // edge of the empty cube or cell reached (0 for a leaf)
        int leaf = -1;
        int sh = 0;
        {
            const int bid = ((w.cell[2] >> 2) * E + (w.cell[1] >> 2)) * E + (w.cell[0] >> 2);
            bool held = bid == w.brick;
            if (!held) {
                const int e = tr.dir[bid];
                if (e >= 0) {
                    const int4 v = tr.nodes[e];
                    w.brick = bid;
                    w.bm_lo = (uint32_t)v.x;
                    w.bm_hi = (uint32_t)v.y;
                    w.bbase = v.z;
                    held = true;
                } else {
                    sh = -e - 1;
                }
            }
            if (held) {
                // child q of the brick node: bit 0 of x, y, z, then bit 1 of x, y, z
                const int x = w.cell[0], y = w.cell[1], z = w.cell[2];
                const int q = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((x & 2) << 2) | ((y & 2) << 3) | ((z & 2) << 4);
                const uint64_t m = ((uint64_t)w.bm_hi << 32) | w.bm_lo;
                if ((m >> q) & 1ull)
                    leaf = w.bbase + (int)__builtin_popcountll(m & ((1ull << q) - 1ull));
                else   // an empty cell; its 2^3 group (one byte of the mask) may be empty as a whole
                    sh = ((m >> (q & 56)) & 0xffull) == 0ull ? 1 : 0;
            }
        }
        const int S = 1 << sh;
        // Exit face of the cell (or empty node) of edge S: per axis the float
        // estimate of the crossing of its far plane and the bound on its error,
        // computed for every axis without branches (zero direction components
        // never exit); the smallest estimate wins, and the decision is redone in
        // compensated arithmetic only when another axis is within the bounds.
        int corner[3], plane[3];
        float est[3], tol[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            corner[a] = w.cell[a] & ~(S - 1);
            plane[a] = corner[a] + (rs.sgn[a] > 0 ? S : 0);
            const float pf = (float)plane[a], of = rs.O[a].hi, iv = rs.inv[a].hi;
            const float e = (pf - of) * iv;
            const float t = kRel * (fabsf(pf) + fabsf(of)) * fabsf(iv) + 1.0e-30f;
            est[a] = rs.sgn[a] != 0 ? e : INFINITY;
            tol[a] = rs.sgn[a] != 0 ? t : 0.0f;
        }
        int am = 0;
        float e_am = est[0], t_am = tol[0];
        if (est[1] < e_am) { am = 1; e_am = est[1]; t_am = tol[1]; }
        if (est[2] < e_am) { am = 2; e_am = est[2]; t_am = tol[2]; }
        bool exact_ue = false;
        df ue = df_from(0.0f);
        const bool near = (am != 0 && rs.sgn[0] != 0 && est[0] - e_am <= tol[0] + t_am) ||
                          (am != 1 && rs.sgn[1] != 0 && est[1] - e_am <= tol[1] + t_am) ||
                          (am != 2 && rs.sgn[2] != 0 && est[2] - e_am <= tol[2] + t_am);
        if (near) {
            // exact: the smallest crossing among the axes within the bounds (first axis on a tie)
            int best = -1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (rs.sgn[a] == 0 || est[a] - e_am > tol[a] + t_am) continue;
                const df ua = crossing(rs, a, plane[a]);
                if (best < 0 || df_lt(ua, ue)) { ue = ua; best = a; }
            }
            am = best;
            exact_ue = true;
        }
        const int p_am = NEUVV_SEL3(plane, am);
        const int c_am = NEUVV_SEL3(corner, am);
        float ue_est = exact_ue ? df_f(ue) : e_am;
        const float ue_tol = exact_ue ? 0.0f : t_am;
        // leaving the box?
        const float uo = df_f(rs.u_out);
        bool last;
        if (ue_est - ue_tol > uo + kRel * fabsf(uo)) {
            last = true;
        } else if (ue_est + ue_tol < uo - kRel * fabsf(uo)) {
            last = false;
        } else {
            if (!exact_ue) { ue = crossing(rs, am, p_am); exact_ue = true; }
            last = !df_lt(ue, rs.u_out);
        }
        bool produced = false;
        if (leaf >= 0) {
            df ux;
            if (last) ux = rs.u_out;
            else if (exact_ue) ux = ue;
            else ux = crossing(rs, am, p_am);
            const df u0 = w.u_entry_ok ? w.u_entry : entry_param(rs, w);
            if (df_lt(u0, ux)) {
                delta = df_f(df_sub(ux, u0)) * rs.len_local;
                umid = 0.5f * (df_f(u0) + df_f(ux));
                seg_a = u0;
                seg_b = ux;
                produced = delta > 0.0f;
            }
            if (!exact_ue && !last) { ue = ux; exact_ue = true; }
        }
        if (last) {
            w.done = true;
        } else {
            // The next cell: across the exit plane on the exit axis; on the other
            // axes the cell of the float position at the estimated exit, unless
            // that position is within its error bound of a cell face, where the
            // exact position decides.
            int nc[3];
            bool amb[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float of = rs.O[b].hi, dfb = rs.D[b].hi;
                const float pf = __builtin_fmaf(ue_est, dfb, of);
                const float err = ue_tol * fabsf(dfb) + kRel * (fabsf(of) + fabsf(ue_est * dfb)) + 1.0e-30f;
                const float r = rintf(pf);
                const int cf = rs.sgn[b] > 0 ? (int)floorf(pf) : (int)ceilf(pf) - 1;
                const bool free_axis = b != am && rs.sgn[b] != 0;
                amb[b] = free_axis && !(fabsf(pf - r) > err);
                nc[b] = b == am ? (rs.sgn[b] > 0 ? corner[b] + S : corner[b] - 1) : (rs.sgn[b] == 0 ? w.cell[b] : cf);
            }
            if (amb[0] || amb[1] || amb[2]) {
                if (!exact_ue) { ue = crossing(rs, am, p_am); exact_ue = true; }
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    if (amb[b]) nc[b] = df_cell(df_add(rs.O[b], df_mul(ue, rs.D[b])), rs.sgn[b]);
            }
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (b != am && rs.sgn[b] != 0)
                    nc[b] = nc[b] < corner[b] ? corner[b] : (nc[b] > corner[b] + S - 1 ? corner[b] + S - 1 : nc[b]);
            const int n_am = NEUVV_SEL3(rs.sgn, am) > 0 ? c_am + S : c_am - 1;
            if (n_am < 0 || n_am >= G) {
                w.done = true;
            } else {
                w.cell[0] = nc[0];
                w.cell[1] = nc[1];
                w.cell[2] = nc[2];
                w.entry_axis = am;
                w.entry_plane = p_am;
                // the next step's entry parameter is this exit, when it was computed exactly
                w.u_entry = ue;
                w.u_entry_ok = exact_ue;
            }
        }
        if (produced) return leaf;
    }
    return -1;
}

// The same without the segment's compensated bounds [seg_a, seg_b).
template <int kBudget = 0>
__device__ __forceinline__ int walk_next(const TreeArgs& tr, const RaySetup& rs, Walk& w, float& delta,
                                         float& umid) {
    df a, b;
    return walk_next<kBudget>(tr, rs, w, delta, umid, a, b);
}

}  // namespace neuvv
