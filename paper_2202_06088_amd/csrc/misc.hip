// Elementwise kernels around the renderer:
//  * compose_fwd / compose_bwd: depth-aware alpha blending of L layers
//    (Alg. 1), read as a per-pixel depth sort then premultiplied "over";
//  * pinhole: camera rays, compensated arithmetic rounded once;
//  * eval_hh: the per-ray HH basis on its own (Eq. 2-4), a test hook;
//  * pack: leaf coefficients into the 16-byte-vector structure-of-arrays
//    storage layout, with round-to-nearest-even for 16-bit storage;
//  * directory: the brick directory of a node table (one descent per 4^3
//    region of leaf cells, done once per tree).
// All are memory-bound streaming kernels: one thread per pixel / ray / leaf,
// grid-stride loops over a grid sized to the device.
#include <hip/hip_runtime.h>

#include <math.h>

#include "launch.h"
#include "neuvv_device.h"

namespace neuvv {

constexpr int kEwBlock = 256;

static int ew_grid(int64_t n) {
    const int64_t want = (n + kEwBlock - 1) / kEwBlock;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    const int64_t g = want < cap ? want : cap;
    return (int)(g > 0 ? g : 1);
}

// ----------------------------------------------------------------------------
// compose. Front-to-back position of layer i: the number of layers j with
// depth_j < depth_i, or depth_j == depth_i and j > i (the later layer is in
// front on ties). Ranks are a permutation, so the sorted arrays are built by
// fully unrolled selection and everything stays in registers.

template <int L>
__device__ __forceinline__ void layer_ranks(const float (&dep)[L], int (&rank)[L]) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
        int r = 0;
#pragma unroll
        for (int j = 0; j < L; ++j)
            if (j != i) r += (dep[j] < dep[i] || (dep[j] == dep[i] && j > i)) ? 1 : 0;
        rank[i] = r;
    }
}

template <int L>
__global__ __launch_bounds__(kEwBlock) void compose_fwd_kernel(int64_t n, const float* __restrict__ rgb,
                                                               const float* __restrict__ alpha,
                                                               const float* __restrict__ depth,
                                                               float* __restrict__ out_rgb,
                                                               float* __restrict__ out_alpha,
                                                               float* __restrict__ out_depth) {
    for (int64_t p = blockIdx.x * (int64_t)kEwBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kEwBlock) {
        float dep[L], A[L], P[L][3];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            dep[i] = depth[(int64_t)i * n + p];
            A[i] = alpha[(int64_t)i * n + p];
            const float* q = rgb + ((int64_t)i * n + p) * 3;
            P[i][0] = q[0]; P[i][1] = q[1]; P[i][2] = q[2];
        }
        int rank[L];
        layer_ranks<L>(dep, rank);
        float sA[L], sP[L][3], front = INFINITY;
#pragma unroll
        for (int r = 0; r < L; ++r) {
            sA[r] = 0.0f; sP[r][0] = sP[r][1] = sP[r][2] = 0.0f;
#pragma unroll
            for (int i = 0; i < L; ++i)
                if (rank[i] == r) {
                    sA[r] = A[i]; sP[r][0] = P[i][0]; sP[r][1] = P[i][1]; sP[r][2] = P[i][2];
                    if (r == 0) front = dep[i];
                }
        }
        float M = 1.0f, o0 = 0.0f, o1 = 0.0f, o2 = 0.0f;
#pragma unroll
        for (int r = 0; r < L; ++r) {
            o0 = fmaf(M, sP[r][0], o0);
            o1 = fmaf(M, sP[r][1], o1);
            o2 = fmaf(M, sP[r][2], o2);
            M *= 1.0f - sA[r];
        }
        out_rgb[3 * p] = o0; out_rgb[3 * p + 1] = o1; out_rgb[3 * p + 2] = o2;
        out_alpha[p] = 1.0f - M;
        if (out_depth) out_depth[p] = front;
    }
}

// d out_rgb / d P_k = M_k; d out_rgb / d A_k = -M_k S_{k+1}; d out_alpha / d A_k = M_k Q_{k+1},
// with M_k the transmittance in front of sorted layer k, S_{k+1} the "over" of
// the layers behind it and Q_{k+1} their joint transmittance.
template <int L>
__global__ __launch_bounds__(kEwBlock) void compose_bwd_kernel(int64_t n, const float* __restrict__ rgb,
                                                               const float* __restrict__ alpha,
                                                               const float* __restrict__ depth,
                                                               const float* __restrict__ g_rgb,
                                                               const float* __restrict__ g_alpha,
                                                               float* __restrict__ grad_rgb,
                                                               float* __restrict__ grad_alpha) {
    for (int64_t p = blockIdx.x * (int64_t)kEwBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kEwBlock) {
        float dep[L], A[L], P[L][3];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            dep[i] = depth[(int64_t)i * n + p];
            A[i] = alpha[(int64_t)i * n + p];
            const float* q = rgb + ((int64_t)i * n + p) * 3;
            P[i][0] = q[0]; P[i][1] = q[1]; P[i][2] = q[2];
        }
        int rank[L];
        layer_ranks<L>(dep, rank);
        float sA[L], sP[L][3];
#pragma unroll
        for (int r = 0; r < L; ++r) {
            sA[r] = 0.0f; sP[r][0] = sP[r][1] = sP[r][2] = 0.0f;
#pragma unroll
            for (int i = 0; i < L; ++i)
                if (rank[i] == r) { sA[r] = A[i]; sP[r][0] = P[i][0]; sP[r][1] = P[i][1]; sP[r][2] = P[i][2]; }
        }
        const float gp0 = g_rgb[3 * p], gp1 = g_rgb[3 * p + 1], gp2 = g_rgb[3 * p + 2];
        const float ga = g_alpha ? g_alpha[p] : 0.0f;
        float M[L];
        float m = 1.0f;
#pragma unroll
        for (int r = 0; r < L; ++r) { M[r] = m; m *= 1.0f - sA[r]; }
        float gsA[L];
        float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f, Q = 1.0f;   // of the layers behind r
#pragma unroll
        for (int r = L - 1; r >= 0; --r) {
            gsA[r] = -M[r] * (gp0 * S0 + gp1 * S1 + gp2 * S2) + ga * M[r] * Q;
            const float t = 1.0f - sA[r];
            S0 = fmaf(t, S0, sP[r][0]);
            S1 = fmaf(t, S1, sP[r][1]);
            S2 = fmaf(t, S2, sP[r][2]);
            Q *= t;
        }
#pragma unroll
        for (int i = 0; i < L; ++i) {
            float Mi = 0.0f, gAi = 0.0f;
#pragma unroll
            for (int r = 0; r < L; ++r)
                if (rank[i] == r) { Mi = M[r]; gAi = gsA[r]; }
            float* q = grad_rgb + ((int64_t)i * n + p) * 3;
            q[0] = Mi * gp0; q[1] = Mi * gp1; q[2] = Mi * gp2;
            grad_alpha[(int64_t)i * n + p] = gAi;
        }
    }
}

template <int L>
static hipError_t compose_fwd_t(int64_t n, const float* rgb, const float* alpha, const float* depth, float* o_rgb,
                                float* o_alpha, float* o_depth, hipStream_t st) {
    hipLaunchKernelGGL(compose_fwd_kernel<L>, dim3(ew_grid(n)), dim3(kEwBlock), 0, st, n, rgb, alpha, depth, o_rgb,
                       o_alpha, o_depth);
    return hipGetLastError();
}

template <int L>
static hipError_t compose_bwd_t(int64_t n, const float* rgb, const float* alpha, const float* depth,
                                const float* g_rgb, const float* g_alpha, float* grad_rgb, float* grad_alpha,
                                hipStream_t st) {
    hipLaunchKernelGGL(compose_bwd_kernel<L>, dim3(ew_grid(n)), dim3(kEwBlock), 0, st, n, rgb, alpha, depth, g_rgb,
                       g_alpha, grad_rgb, grad_alpha);
    return hipGetLastError();
}

#define NEUVV_L_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_compose_fwd(int L, int64_t n, const float* rgb, const float* alpha, const float* depth,
                              float* out_rgb, float* out_alpha, float* out_depth, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    switch (L) {
#define NEUVV_CASE(l) \
    case l: return compose_fwd_t<l>(n, rgb, alpha, depth, out_rgb, out_alpha, out_depth, stream);
        NEUVV_L_CASES(NEUVV_CASE)
#undef NEUVV_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_compose_bwd(int L, int64_t n, const float* rgb, const float* alpha, const float* depth,
                              const float* g_rgb, const float* g_alpha, float* grad_rgb, float* grad_alpha,
                              hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    switch (L) {
#define NEUVV_CASE(l) \
    case l: return compose_bwd_t<l>(n, rgb, alpha, depth, g_rgb, g_alpha, grad_rgb, grad_alpha, stream);
        NEUVV_L_CASES(NEUVV_CASE)
#undef NEUVV_CASE
        default: return hipErrorInvalidValue;
    }
}

// ----------------------------------------------------------------------------
// pinhole rays

struct CamArgs {
    float intr[4];
    float c2w[12];
    int32_t W, H;
};

__global__ __launch_bounds__(kEwBlock) void pinhole_kernel(CamArgs cam, int64_t n, const int32_t* __restrict__ pix,
                                                           float* __restrict__ ray_o, float* __restrict__ ray_d) {
    for (int64_t i = blockIdx.x * (int64_t)kEwBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kEwBlock) {
        const int64_t p = pix ? (int64_t)pix[i] : i;
        const int64_t v = p / cam.W, u = p - v * cam.W;
        // x_c = (u + 0.5 - cx) / fx, y_c = (v + 0.5 - cy) / fy: u + 0.5 is exact below 2^23
        const df xc = df_div(df_two_sum((float)u + 0.5f, -cam.intr[2]), df_from(cam.intr[0]));
        const df yc = df_div(df_two_sum((float)v + 0.5f, -cam.intr[3]), df_from(cam.intr[1]));
        df dv[3];
        df n2 = df_from(0.0f);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            df s = df_add(df_mul_f(xc, cam.c2w[4 * a]), df_mul_f(yc, cam.c2w[4 * a + 1]));
            dv[a] = df_add(s, df_from(cam.c2w[4 * a + 2]));
            n2 = df_add(n2, df_mul(dv[a], dv[a]));
        }
        // 1/sqrt(n2): float estimate refined by two compensated Newton steps r += r (1 - n2 r^2) / 2
        df r = df_from(1.0f / sqrtf(n2.hi));
        for (int it = 0; it < 2; ++it) {
            const df e = df_sub(df_from(1.0f), df_mul(n2, df_mul(r, r)));
            r = df_add(r, df_mul_f(df_mul(r, e), 0.5f));
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ray_d[3 * i + a] = df_f(df_mul(dv[a], r));
            ray_o[3 * i + a] = cam.c2w[4 * a + 3];
        }
    }
}

hipError_t launch_pinhole(int W, int H, const float intr[4], const float c2w[12], int64_t n, const int32_t* pix,
                          float* ray_o, float* ray_d, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    CamArgs cam;
    for (int i = 0; i < 4; ++i) cam.intr[i] = intr[i];
    for (int i = 0; i < 12; ++i) cam.c2w[i] = c2w[i];
    cam.W = W;
    cam.H = H;
    hipLaunchKernelGGL(pinhole_kernel, dim3(ew_grid(n)), dim3(kEwBlock), 0, stream, cam, n, pix, ray_o, ray_d);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// HH basis test hook

__global__ __launch_bounds__(kEwBlock) void eval_hh_kernel(int K, int64_t n, const float* __restrict__ dirs,
                                                           const float* __restrict__ gam, float* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)kEwBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kEwBlock) {
        float h[30];
        hh_all(dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], gam[i], h);
#pragma unroll
        for (int k = 0; k < 30; ++k)
            if (k < K) out[i * K + k] = h[k];
    }
}

hipError_t launch_eval_hh(int K, int64_t n, const float* dirs, const float* gam, float* out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_hh_kernel, dim3(ew_grid(n)), dim3(kEwBlock), 0, stream, K, n, dirs, gam, out);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// payload packing

__device__ __forceinline__ uint16_t f32_to_f16_rne(float x) {
    return __builtin_bit_cast(uint16_t, (_Float16)x);   // v_cvt_f16_f32 rounds to nearest even
}
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One thread per (leaf, vector): reads the V values of the vector, converts
// and writes 16 bytes.
template <int DT>
__global__ __launch_bounds__(kEwBlock) void pack_kernel(int R, int NG, int layout, int64_t n,
                                                        const float* __restrict__ in,
                                                        const int64_t* __restrict__ slot_of_input,
                                                        uint4* __restrict__ out) {
    constexpr int V = DT == 0 ? 4 : 8;
    const int64_t total = n * NG;
    for (int64_t t = blockIdx.x * (int64_t)kEwBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kEwBlock) {
        const int64_t i = t / NG;
        const int g = (int)(t - i * NG);
        const int64_t s = slot_of_input ? slot_of_input[i] : i;
        float v[8];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int r = g * V + e;
            v[e] = r < R ? in[i * R + r] : 0.0f;
        }
        uint4 w;
        if constexpr (DT == 0) {
            w.x = __float_as_uint(v[0]); w.y = __float_as_uint(v[1]);
            w.z = __float_as_uint(v[2]); w.w = __float_as_uint(v[3]);
        } else {
            uint32_t q[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint16_t lo = DT == 1 ? f32_to_f16_rne(v[2 * k]) : f32_to_bf16_rne(v[2 * k]);
                const uint16_t hi = DT == 1 ? f32_to_f16_rne(v[2 * k + 1]) : f32_to_bf16_rne(v[2 * k + 1]);
                q[k] = (uint32_t)lo | ((uint32_t)hi << 16);
            }
            w.x = q[0]; w.y = q[1]; w.z = q[2]; w.w = q[3];
        }
        out[layout ? s * NG + g : (int64_t)g * n + s] = w;
    }
}

template <int DT>
static hipError_t pack_t(int R, int layout, int64_t n, const float* in, const int64_t* slots, void* out,
                         hipStream_t st) {
    constexpr int V = DT == 0 ? 4 : 8;
    const int NG = (R + V - 1) / V;
    hipLaunchKernelGGL(pack_kernel<DT>, dim3(ew_grid(n * NG)), dim3(kEwBlock), 0, st, R, NG, layout, n, in, slots,
                       reinterpret_cast<uint4*>(out));
    return hipGetLastError();
}

hipError_t launch_pack_rows(int R, int dtype, int layout, int64_t n, const float* in, const int64_t* slot_of_input,
                            void* out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    switch (dtype) {
        case 0: return pack_t<0>(R, layout, n, in, slot_of_input, out, stream);
        case 1: return pack_t<1>(R, layout, n, in, slot_of_input, out, stream);
        default: return pack_t<2>(R, layout, n, in, slot_of_input, out, stream);
    }
}

hipError_t launch_pack(int K, int C, int dtype, int layout, int64_t n, const float* hh_in, const float* wsig_in,
                       const int64_t* slot_of_input, void* hh_out, void* wsig_out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipError_t e;
    switch (dtype) {
        case 0:
            e = pack_t<0>(3 * K, layout, n, hh_in, slot_of_input, hh_out, stream);
            return e != hipSuccess ? e : pack_t<0>(C, layout, n, wsig_in, slot_of_input, wsig_out, stream);
        case 1:
            e = pack_t<1>(3 * K, layout, n, hh_in, slot_of_input, hh_out, stream);
            return e != hipSuccess ? e : pack_t<1>(C, layout, n, wsig_in, slot_of_input, wsig_out, stream);
        default:
            e = pack_t<2>(3 * K, layout, n, hh_in, slot_of_input, hh_out, stream);
            return e != hipSuccess ? e : pack_t<2>(C, layout, n, wsig_in, slot_of_input, wsig_out, stream);
    }
}

}  // namespace neuvv

namespace neuvv {

// ----------------------------------------------------------------------------
// brick directory: entry (k E + j) E + i for the 4^3 region with corner
// (4i, 4j, 4k) descends from the root through the node levels above the last
// one. It stops at the first child cell (edge 2^cs) that holds no leaf and
// records -(1 + s), s = cs + 1 when the child's 2^3 group (one byte of a
// 2-bit node's mask) is empty as well, else s = cs: the cube at which a walk
// descending to any cell of the region would stop. A region that holds a
// leaf gets the row of its last-level node. With D <= 2 the root is that node.

__global__ __launch_bounds__(kEwBlock) void directory_kernel(const int4* __restrict__ nodes, int D, int64_t n,
                                                             int32_t* __restrict__ dir) {
    const int64_t E = directory_edge(D);
    const int last = (D + 1) / 2 - 1;
    for (int64_t i = (int64_t)blockIdx.x * kEwBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kEwBlock) {
        const int x = (int)(i % E) << 2, y = (int)((i / E) % E) << 2, z = (int)(i / (E * E)) << 2;
        int node = 0;
        int entry = 0;
        bool empty = false;
        for (int w = 0; w < last && !empty; ++w) {
            const int bits = node_bits(D, w);
            const int cs = node_edge(D, w) - bits;
            const int xs = x >> cs, ys = y >> cs, zs = z >> cs;
            int q = (xs & 1) | ((ys & 1) << 1) | ((zs & 1) << 2);
            if (bits == 2) q |= ((xs & 2) << 2) | ((ys & 2) << 3) | ((zs & 2) << 4);
            const int4 v = nodes[node];
            const uint64_t m = ((uint64_t)(uint32_t)v.y << 32) | (uint32_t)v.x;
            if ((m >> q) & 1ull) {
                node = v.z + (int)__builtin_popcountll(m & ((1ull << q) - 1ull));
            } else {
                const int s = (bits == 2 && ((m >> (q & 56)) & 0xffull) == 0ull) ? cs + 1 : cs;
                entry = -(1 + s);
                empty = true;
            }
        }
        dir[i] = empty ? entry : node;
    }
}

hipError_t launch_build_directory(const int4* nodes, int depth, int32_t* dir, hipStream_t stream) {
    const int64_t n = directory_entries(depth);
    hipLaunchKernelGGL(directory_kernel, dim3(ew_grid(n)), dim3(kEwBlock), 0, stream, nodes, depth, n, dir);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// appearance edits (Sec. 5.2 "Appearance editing"): every ray that ended in a
// leaf claims it, the lowest ray index wins, and the winner writes its target
// colour, density and first frame into the leaf's edit row {r, g, b, sigma_d,
// t_d, owner, 0, 0}. Three passes: reset the owners of the leaves involved,
// claim with atomicMin, write.

__global__ __launch_bounds__(kEwBlock) void paint_reset_kernel(int64_t n, const int32_t* __restrict__ last_leaf,
                                                               int64_t n_leaves, int32_t* __restrict__ words) {
    for (int64_t r = blockIdx.x * (int64_t)kEwBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kEwBlock) {
        const int32_t L = last_leaf[r];
        if (L >= 0 && L < n_leaves) words[8 * (int64_t)L + 5] = 0x7fffffff;
    }
}

__global__ __launch_bounds__(kEwBlock) void paint_claim_kernel(int64_t n, const int32_t* __restrict__ last_leaf,
                                                               int64_t n_leaves, int32_t* __restrict__ words) {
    for (int64_t r = blockIdx.x * (int64_t)kEwBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kEwBlock) {
        const int32_t L = last_leaf[r];
        if (L >= 0 && L < n_leaves) atomicMin(words + 8 * (int64_t)L + 5, (int32_t)r);
    }
}

__global__ __launch_bounds__(kEwBlock) void paint_write_kernel(int64_t n, const int32_t* __restrict__ last_leaf,
                                                               int64_t n_leaves, const float* __restrict__ colours,
                                                               float sigma_d, float t_d, float* __restrict__ edit) {
    int32_t* words = reinterpret_cast<int32_t*>(edit);
    for (int64_t r = blockIdx.x * (int64_t)kEwBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kEwBlock) {
        const int32_t L = last_leaf[r];
        if (L < 0 || L >= n_leaves || words[8 * (int64_t)L + 5] != (int32_t)r) continue;
        float* row = edit + 8 * (int64_t)L;
        row[0] = colours[3 * r];
        row[1] = colours[3 * r + 1];
        row[2] = colours[3 * r + 2];
        row[3] = sigma_d;
        row[4] = t_d;
    }
}

hipError_t launch_paint(int64_t n, const int32_t* last_leaf, const float* colours, float sigma_d, float t_d,
                        int64_t n_leaves, float* edit, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int32_t* words = reinterpret_cast<int32_t*>(edit);
    const int g = ew_grid(n);
    hipLaunchKernelGGL(paint_reset_kernel, dim3(g), dim3(kEwBlock), 0, stream, n, last_leaf, n_leaves, words);
    hipLaunchKernelGGL(paint_claim_kernel, dim3(g), dim3(kEwBlock), 0, stream, n, last_leaf, n_leaves, words);
    hipLaunchKernelGGL(paint_write_kernel, dim3(g), dim3(kEwBlock), 0, stream, n, last_leaf, n_leaves, colours,
                       sigma_d, t_d, edit);
    return hipGetLastError();
}

}  // namespace neuvv
