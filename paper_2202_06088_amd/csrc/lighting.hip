// Spotlight shadow and distance-falloff lighting (Sec. 5.2 "Spotlight
// Lighting", Sec. 6 "Lighting") on top of rendered maps:
//  * blur: the Gaussian low-pass of the light's alpha map (shadow map),
//    taps w_i ~ exp(-i^2 / (2 sigma^2)), |i| <= round(3 sigma), normalised,
//    borders clamped to the edge; the 2-D sum of the separable kernel is
//    evaluated per output pixel (light maps are small);
//  * shade: per viewer pixel, the ground plane z = ground_z is met at q, q is
//    projected into the light camera and the shadow map sampled bilinearly
//    there (0 outside the image or behind the light); the ground colour is
//    scaled by 1 - k A; the performer's premultiplied colour is scaled by
//    (r0 / max(r, r0))^2, r the distance from the light to its expected
//    surface point; the performer is composited over the ground unless the
//    ground is met first. Memory-bound streaming kernels.
#include <hip/hip_runtime.h>

#include <math.h>

#include "launch.h"

namespace neuvv {

constexpr int kLightBlock = 256;

static int light_grid(int64_t n) {
    const int64_t want = (n + kLightBlock - 1) / kLightBlock;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    const int64_t g = want < cap ? want : cap;
    return (int)(g > 0 ? g : 1);
}

__global__ __launch_bounds__(kLightBlock) void blur_kernel(int H, int W, const float* __restrict__ in, BlurTaps taps,
                                                           float* __restrict__ out) {
    const int64_t n = (int64_t)H * W;
    const int r = taps.radius;
    for (int64_t p = blockIdx.x * (int64_t)kLightBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kLightBlock) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        float acc = 0.0f;
        for (int i = -r; i <= r; ++i) {
            int yy = y + i;
            yy = yy < 0 ? 0 : (yy > H - 1 ? H - 1 : yy);
            const float* row = in + (int64_t)yy * W;
            float rs = 0.0f;
            for (int j = -r; j <= r; ++j) {
                int xx = x + j;
                xx = xx < 0 ? 0 : (xx > W - 1 ? W - 1 : xx);
                rs = fmaf(taps.w[j + r], row[xx], rs);
            }
            acc = fmaf(taps.w[i + r], rs, acc);
        }
        out[p] = acc;
    }
}

// Bilinear sample at image coordinates (u, v) (pixel centres at +1/2),
// edge-clamped inside [0, W] x [0, H], 0 outside.
__device__ __forceinline__ float sample_map(const float* __restrict__ m, int W, int H, float u, float v) {
    if (!(u >= 0.0f && u <= (float)W && v >= 0.0f && v <= (float)H)) return 0.0f;
    const float x = u - 0.5f, y = v - 0.5f;
    const float x0 = floorf(x), y0 = floorf(y);
    const float fx = x - x0, fy = y - y0;
    const int xi0 = x0 < 0.0f ? 0 : (int)x0, yi0 = y0 < 0.0f ? 0 : (int)y0;
    const int xa = xi0 > W - 1 ? W - 1 : xi0, ya = yi0 > H - 1 ? H - 1 : yi0;
    const int xb = (int)x0 + 1 > W - 1 ? W - 1 : ((int)x0 + 1 < 0 ? 0 : (int)x0 + 1);
    const int yb = (int)y0 + 1 > H - 1 ? H - 1 : ((int)y0 + 1 < 0 ? 0 : (int)y0 + 1);
    const float a = m[(int64_t)ya * W + xa], b = m[(int64_t)ya * W + xb];
    const float c = m[(int64_t)yb * W + xa], d = m[(int64_t)yb * W + xb];
    return (1.0f - fy) * ((1.0f - fx) * a + fx * b) + fy * ((1.0f - fx) * c + fx * d);
}

__global__ __launch_bounds__(kLightBlock) void shade_kernel(LightArgs L, const float* __restrict__ shadow_map,
                                                            int64_t n, const float* __restrict__ ray_o,
                                                            const float* __restrict__ ray_d,
                                                            const float* __restrict__ rgb,
                                                            const float* __restrict__ alpha,
                                                            const float* __restrict__ depth,
                                                            float* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)kLightBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLightBlock) {
        const float o0 = ray_o[3 * i], o1 = ray_o[3 * i + 1], o2 = ray_o[3 * i + 2];
        const float d0 = ray_d[3 * i], d1 = ray_d[3 * i + 1], d2 = ray_d[3 * i + 2];
        const float dn = sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
        const float dep = depth[i];
        // falloff of the performer's colour
        float F = 1.0f;
        if (L.r0 > 0.0f && isfinite(dep) && dn > 0.0f) {
            const float s = dep / dn;
            const float p0 = fmaf(s, d0, o0) - L.C[0], p1 = fmaf(s, d1, o1) - L.C[1], p2 = fmaf(s, d2, o2) - L.C[2];
            const float r = sqrtf(p0 * p0 + p1 * p1 + p2 * p2);
            const float q = L.r0 / fmaxf(r, L.r0);
            F = q * q;
        }
        // ground
        float g0 = L.bg[0], g1 = L.bg[1], g2 = L.bg[2];
        bool ground_first = false;
        if (d2 != 0.0f) {
            const float t = (L.ground_z - o2) / d2;
            if (t > 0.0f) {
                float S = 0.0f;
                if (shadow_map) {
                    const float q0 = fmaf(t, d0, o0) - L.C[0], q1 = fmaf(t, d1, o1) - L.C[1];
                    const float q2 = L.ground_z - L.C[2];
                    // light-camera frame: x = R^T (q - C), R row-major
                    const float x = L.R[0] * q0 + L.R[3] * q1 + L.R[6] * q2;
                    const float y = L.R[1] * q0 + L.R[4] * q1 + L.R[7] * q2;
                    const float z = L.R[2] * q0 + L.R[5] * q1 + L.R[8] * q2;
                    if (z > 0.0f) S = sample_map(shadow_map, L.W, L.H, L.fx * x / z + L.cx, L.fy * y / z + L.cy);
                }
                const float sh = 1.0f - L.k * S;
                g0 = L.ground[0] * sh; g1 = L.ground[1] * sh; g2 = L.ground[2] * sh;
                ground_first = t * dn < dep;
            }
        }
        if (ground_first) {
            out[3 * i] = g0; out[3 * i + 1] = g1; out[3 * i + 2] = g2;
        } else {
            const float ta = 1.0f - alpha[i];
            out[3 * i] = fmaf(ta, g0, rgb[3 * i] * F);
            out[3 * i + 1] = fmaf(ta, g1, rgb[3 * i + 1] * F);
            out[3 * i + 2] = fmaf(ta, g2, rgb[3 * i + 2] * F);
        }
    }
}

hipError_t launch_blur(int H, int W, const float* in, const BlurTaps& taps, float* out, hipStream_t stream) {
    const int64_t n = (int64_t)H * W;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(blur_kernel, dim3(light_grid(n)), dim3(kLightBlock), 0, stream, H, W, in, taps, out);
    return hipGetLastError();
}

hipError_t launch_shade(const LightArgs& L, const float* shadow_map, int64_t n, const float* ray_o, const float* ray_d,
                        const float* rgb, const float* alpha, const float* depth, float* out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(shade_kernel, dim3(light_grid(n)), dim3(kLightBlock), 0, stream, L, shadow_map, n, ray_o, ray_d,
                       rgb, alpha, depth, out);
    return hipGetLastError();
}

}  // namespace neuvv
