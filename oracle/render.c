/*
 * FP64 oracle renderer for VOctree volume rendering (NeuVV, arXiv 2202.06088).
 *
 * TEST INFRASTRUCTURE ONLY: built by the test/bench tooling, called through
 * ctypes from oracle/core.py. The product library never links or calls it.
 * It shares no code with the GPU path.
 *
 * What it computes, per ray, in double precision (Sec. 4.3 "Rendering",
 * Eq. 4, 5, 8, 9, 13):
 *   1. instance transform (Eq. 13): local point x_l = R^T (x - trans) / s for
 *      every point of the world ray x(u) = o + u d, so the local ray is
 *      o_l + u d_l with o_l = R^T (o - trans)/s, d_l = R^T d / s and the same
 *      parameter u; re-timing tau = t + offset, wrapped into [0,T) or clamped
 *      into [0,T-1];
 *   2. the voxels on the ray and the lengths of the line segments inside them
 *      (Sec. 4.3): an exact leaf-level DDA over the grid [0,2^D)^3 with
 *      half-open cells [i,i+1), each occupied cell looked up in a hash set
 *      of the leaf coordinates. Segments of zero length are not samples;
 *   3. per ray, the basis h = first K real HH at the unit local view
 *      direction and gamma = lerp of the hyperangle table at tau (Eq. 2-4),
 *      and b = lerp of the density basis rows at tau (Eq. 5);
 *   4. per occupied segment, in order of increasing u:
 *        sigma = softplus(sum_c wsig_c b_c)          (Eq. 5, softplus reading;
 *                or relu(...), the activation Eq. 5 prints, with density_act = 1)
 *        c_ch  = sigmoid(sum_k hh_ch,k h_k)            (Eq. 4 + sigmoid)
 *        delta = segment length in leaf units
 *        alpha_i = 1 - exp(-sigma delta), w = T alpha_i, T *= exp(-sigma delta)
 *        C += w c, A += w, D += w * (world distance of the segment midpoint)
 *      stopping after the first sample that leaves T < t_stop (Eq. 8);
 *   5. outputs: premultiplied colour C, alpha A = sum of weights (Eq. 9),
 *      depth D / A (+inf when A = 0), the sample count and the final
 *      transmittance exp(-sum sigma delta) recomputed from the optical depth.
 *   6. optionally the gradient of L = <g_C, C> + g_A * A with respect to the
 *      HH coefficients, density weights and density basis rows, by the chain
 *      rule through steps 3-4 (Sec. 4.3 "Optimization").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* real 4-D hyperspherical harmonics (Sec. 4.1 Eq. 2-3, Appendix A.2) */

static double fact(int k) { double r = 1.0; for (int i = 2; i <= k; ++i) r *= i; return r; }
static double dfact(int k) { double r = 1.0; for (; k > 1; k -= 2) r *= k; return r; }
static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

/* Gegenbauer C^lam_k(x) as the explicit finite sum. */
static double gegenbauer(int k, double lam, double x) {
    double acc = 0.0;
    for (int j = 0; j <= k / 2; ++j) {
        double coef = ((j & 1) ? -1.0 : 1.0) * tgamma(k - j + lam) /
                      (tgamma(lam) * fact(j) * fact(k - 2 * j));
        acc += coef * pow(2.0 * x, k - 2 * j);
    }
    return acc;
}

/* sqrt((l-m)!/(l+m)!) sum_k B_{k,lm} z^(l-2k-m), m >= 0. */
static double legendre_part(int l, int m, double z) {
    double acc = 0.0;
    for (int k = 0; k <= (l - m) / 2; ++k) {
        double b = ((k & 1) ? -1.0 : 1.0) * pow(2.0, -l) * binom(l, k) * binom(2 * l - 2 * k, l) *
                   fact(l - 2 * k) / fact(l - 2 * k - m);
        acc += b * pow(z, l - 2 * k - m);
    }
    return sqrt(fact(l - m) / fact(l + m)) * acc;
}

/* Orthonormal real SH at a unit direction, polar axis z, no Condon-Shortley phase. */
static double real_sh(int l, int m, double x, double y, double z) {
    int am = m < 0 ? -m : m;
    double pref = sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
    double poly = legendre_part(l, am, z);
    if (m == 0) return pref * poly;
    double re = 0.0, im = 0.0;  /* Re, Im of (x + i y)^|m| by the binomial sum */
    for (int p = 0; p <= am; ++p) {
        double term = binom(am, p) * pow(x, p) * pow(y, am - p);
        re += term * cos((am - p) * M_PI / 2.0);
        im += term * sin((am - p) * M_PI / 2.0);
    }
    return sqrt(2.0) * pref * poly * (m > 0 ? re : im);
}

/* first K functions in the order n, l, m: h[k] = A_nl sin^l g C^{l+1}_{n-l}(cos g) Y_lm(d) */
static void hh_basis(int K, const double d[3], double gam, double* h) {
    int k = 0;
    for (int n = 0; k < K; ++n)
        for (int l = 0; l <= n && k < K; ++l) {
            double A = dfact(2 * l) * sqrt(2.0 * (n + 1) * fact(n - l) / (M_PI * fact(n + l + 1)));
            double g = A * pow(sin(gam), l) * gegenbauer(n - l, l + 1.0, cos(gam));
            for (int m = -l; m <= l && k < K; ++m) h[k++] = g * real_sh(l, m, d[0], d[1], d[2]);
        }
}

/* Direction factors Y_k and the (n, l) of each of the first K functions. */
static void hh_dir_factors(int K, const double d[3], double* Y, int* nk, int* lk) {
    int k = 0;
    for (int n = 0; k < K; ++n)
        for (int l = 0; l <= n && k < K; ++l)
            for (int m = -l; m <= l && k < K; ++m) {
                Y[k] = real_sh(l, m, d[0], d[1], d[2]);
                nk[k] = n; lk[k] = l; ++k;
            }
}

/* g_nl(gamma) = A_nl sin^l(g) C^{l+1}_{n-l}(cos g) and its derivative in gamma, using
   d/dx C^lam_k(x) = 2 lam C^{lam+1}_{k-1}(x). */
static void hh_radial(int n, int l, double gam, double* g, double* dg) {
    double A = dfact(2 * l) * sqrt(2.0 * (n + 1) * fact(n - l) / (M_PI * fact(n + l + 1)));
    double s = sin(gam), c = cos(gam);
    double C0 = gegenbauer(n - l, l + 1.0, c);
    double C1 = n - l >= 1 ? 2.0 * (l + 1.0) * gegenbauer(n - l - 1, l + 2.0, c) : 0.0;
    double sl = pow(s, l);
    *g = A * sl * C0;
    double dsl = l >= 1 ? l * pow(s, l - 1) * c : 0.0;
    *dg = A * (dsl * C0 - sl * s * C1);
}

void oracle_hh_basis(int K, int64_t n, const double* dirs, const double* gam, double* out) {
    for (int64_t i = 0; i < n; ++i) hh_basis(K, dirs + 3 * i, gam[i], out + i * K);
}

/* ------------------------------------------------------------------ */
/* occupancy: open-addressing hash set of leaf cells -> input leaf index */

typedef struct { uint64_t* keys; int64_t* vals; uint64_t mask; } hashset;

static uint64_t cell_key(int64_t i, int64_t j, int64_t k) {
    return ((uint64_t)i) | ((uint64_t)j << 21) | ((uint64_t)k << 42);
}
static uint64_t mix(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33;
    return x;
}
static int hs_build(hashset* h, int64_t n, const int32_t* ijk) {
    uint64_t cap = 16;
    while (cap < (uint64_t)(2 * n + 16)) cap <<= 1;
    h->keys = (uint64_t*)malloc(cap * sizeof(uint64_t));
    h->vals = (int64_t*)malloc(cap * sizeof(int64_t));
    if (!h->keys || !h->vals) return -1;
    h->mask = cap - 1;
    for (uint64_t s = 0; s < cap; ++s) h->keys[s] = ~0ULL;
    for (int64_t q = 0; q < n; ++q) {
        uint64_t key = cell_key(ijk[3 * q], ijk[3 * q + 1], ijk[3 * q + 2]);
        uint64_t s = mix(key) & h->mask;
        while (h->keys[s] != ~0ULL && h->keys[s] != key) s = (s + 1) & h->mask;
        if (h->keys[s] == key) return -2; /* duplicate leaf */
        h->keys[s] = key; h->vals[s] = q;
    }
    return 0;
}
static int64_t hs_find(const hashset* h, int64_t i, int64_t j, int64_t k) {
    uint64_t key = cell_key(i, j, k);
    uint64_t s = mix(key) & h->mask;
    while (h->keys[s] != ~0ULL) {
        if (h->keys[s] == key) return h->vals[s];
        s = (s + 1) & h->mask;
    }
    return -1;
}

/* ------------------------------------------------------------------ */

static double softplus(double x) { return (x > 0 ? x : 0.0) + log1p(exp(-fabs(x))); }
/* density activation of Eq. 5 and its derivative: 0 softplus, 1 relu (derivative 0 at x = 0) */
static double density_of(double x, int act) { return act ? (x > 0 ? x : 0.0) : softplus(x); }
static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

typedef struct { int64_t leaf; double delta, smid, x, sig, z[3], c[3], Tin, alpha, yg, gam, ua, ub; } sample_t;

/* Time re-mapping (Eq. 13): tau = t + off; wrap into [0,T) or clamp into [0,T-1];
   i0 = floor(tau), f = tau - i0, i1 = min(i0+1, T-1); the last frame is held on [T-1,T). */
static void time_lerp(double t, double off, int wrap, int T, int* i0, int* i1, double* f, double* tau_out) {
    double tau = t + off;
    if (wrap) { tau = tau - T * floor(tau / T); if (tau >= T) tau -= T; if (tau < 0) tau = 0; }
    else { if (tau < 0) tau = 0; if (tau > T - 1) tau = T - 1; }
    *tau_out = tau;
    int a = (int)floor(tau);
    if (a > T - 1) a = T - 1;
    if (a < 0) a = 0;
    double fr = tau - a;
    if (a == T - 1) fr = 0.0;
    *i0 = a; *i1 = a + 1 < T ? a + 1 : T - 1; *f = fr;
}

/* Returns 0 on success, -1 allocation failure, -2 duplicate leaf, -3 bad argument, -4 seg_cap too small. */
int oracle_render(int depth, int64_t n_leaves, const int32_t* leaf_ijk,
                  int K, int C, const double* hh /*[N][3][K]*/, const double* wsig /*[N][C]*/,
                  int T, const double* basis /*[T][C]*/, const double* gamma /*[T]*/,
                  int Cg, const double* wgam /* NULL or [N][Cg] */, const double* basis_g /* [T][Cg] */,
                  double* grad_wgam /* NULL or [N][Cg] */, double* grad_basis_g /* NULL or [T][Cg] */,
                  const double* inst /* NULL or rot[9] row-major, trans[3], scale, time_offset, wrap */,
                  int64_t n_rays, const float* ray_o, const float* ray_d, const float* ray_t,
                  double t_scalar, double t_stop,
                  const double* g_rgb /* NULL or [n][3] */, const double* g_alpha /* NULL or [n] */,
                  double* rgb, double* alpha, double* depth_out, int32_t* nsamp, double* tfinal,
                  double* margin /* NULL or [n][2]: min sampled delta, min |T - t_stop|/t_stop */,
                  double* grad_hh, double* grad_wsig, double* grad_basis,
                  const double* edit /* NULL or [N][5]: target rgb, target density (< 0: keep), first frame */,
                  int64_t* last_leaf /* NULL or [n]: leaf of the last sample of a ray that stopped, else -1 */,
                  int seg_cap, double* seg_out /* NULL or [n][seg_cap][6]: every sample's ray interval
                                                   [u_in, u_out), density (per leaf unit), colour */,
                  double* len_out /* NULL or [n]: leaf units per unit of the ray parameter */,
                  int density_act /* 0: sigma = softplus(x), 1: sigma = relu(x) */,
                  int n_threads) {
    if (depth < 1 || depth > 20 || K < 1 || K > 64 || C < 1 || C > 64 || T < 1) return -3;
    if (wgam && (Cg < 1 || Cg > 64 || !basis_g)) return -3;
    hashset hs;
    int rc = hs_build(&hs, n_leaves, leaf_ijk);
    if (rc) { free(hs.keys); free(hs.vals); return rc; }
    const double G = (double)(1LL << depth);
    const int64_t Gi = 1LL << depth;
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, tr[3] = {0, 0, 0}, sc = 1.0, toff = 0.0;
    int wrap = 0;
    if (inst) {
        memcpy(R, inst, 9 * sizeof(double)); memcpy(tr, inst + 9, 3 * sizeof(double));
        sc = inst[12]; toff = inst[13]; wrap = inst[14] != 0.0;
    }
    const int want_grad = g_rgb != NULL && grad_hh != NULL;
    if (want_grad && edit) return -3;   /* edits are a render-time appearance change: no adjoint */
    int err = 0;
    if (n_threads < 1) n_threads = 1;

#pragma omp parallel num_threads(n_threads)
    {
        int64_t cap = 3 * Gi + 8;
        sample_t* S = (sample_t*)malloc(cap * sizeof(sample_t));
        if (!S) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rays; ++r) {
            if (!S) continue;
            double o[3], d[3], ol[3], dl[3];
            for (int a = 0; a < 3; ++a) { o[a] = ray_o[3 * r + a]; d[a] = ray_d[3 * r + a]; }
            for (int a = 0; a < 3; ++a) {
                double ao = 0.0, ad = 0.0;
                for (int b = 0; b < 3; ++b) { ao += R[3 * b + a] * (o[b] - tr[b]); ad += R[3 * b + a] * d[b]; }
                ol[a] = ao / sc; dl[a] = ad / sc;
            }
            double dlen = sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
            double dwlen = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double t = ray_t ? (double)ray_t[r] : t_scalar;
            int i0, i1; double f, tau;
            time_lerp(t, toff, wrap, T, &i0, &i1, &f, &tau);
            double b[64], h[64], dirn[3] = {0.0, 0.0, 1.0};
            if (dlen > 0.0) for (int a = 0; a < 3; ++a) dirn[a] = dl[a] / dlen;
            for (int c = 0; c < C; ++c) b[c] = (1.0 - f) * basis[i0 * C + c] + f * basis[i1 * C + c];
            double gam = (1.0 - f) * gamma[i0] + f * gamma[i1];
            hh_basis(K, dirn, gam, h);
            /* per-point hyperangle (Eq. 6): gamma = pi sigmoid(sum_c wgam_c bg_c), h per sample */
            double bg[64], Yd[64];
            int nk[64], lk[64];
            if (wgam) {
                for (int c = 0; c < Cg; ++c) bg[c] = (1.0 - f) * basis_g[i0 * Cg + c] + f * basis_g[i1 * Cg + c];
                hh_dir_factors(K, dirn, Yd, nk, lk);
            }

            /* clip to the box [0,G]^3 */
            double u_in = 0.0, u_out = INFINITY;
            int miss = !(dlen > 0.0); /* a zero direction sees nothing */
            for (int a = 0; a < 3; ++a) {
                if (dl[a] == 0.0) { if (!(ol[a] >= 0.0 && ol[a] < G)) miss = 1; continue; }
                double t0 = (0.0 - ol[a]) / dl[a], t1 = (G - ol[a]) / dl[a];
                double lo = t0 < t1 ? t0 : t1, hi = t0 < t1 ? t1 : t0;
                if (lo > u_in) u_in = lo;
                if (hi < u_out) u_out = hi;
            }
            if (!(u_in < u_out)) miss = 1;
            int ns = 0;
            double Tr = 1.0, col[3] = {0, 0, 0}, wsum = 0.0, dsum = 0.0, optical = 0.0;
            if (last_leaf) last_leaf[r] = -1;
            double min_delta = INFINITY, min_stop = INFINITY;
            if (!miss) {
                int64_t cell[3];
                for (int a = 0; a < 3; ++a) {
                    double p = ol[a] + u_in * dl[a];
                    int64_t ci = dl[a] < 0.0 ? (int64_t)ceil(p) - 1 : (int64_t)floor(p);
                    if (ci < 0) ci = 0;
                    if (ci > Gi - 1) ci = Gi - 1;
                    cell[a] = ci;
                }
                double u = u_in;
                for (;;) {
                    double tmax[3];
                    int amin = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (dl[a] > 0.0) tmax[a] = ((double)(cell[a] + 1) - ol[a]) / dl[a];
                        else if (dl[a] < 0.0) tmax[a] = ((double)cell[a] - ol[a]) / dl[a];
                        else tmax[a] = INFINITY;
                        if (tmax[a] < tmax[amin]) amin = a;
                    }
                    double un = tmax[amin] < u_out ? tmax[amin] : u_out;
                    if (un > u) {
                        int64_t q = hs_find(&hs, cell[0], cell[1], cell[2]);
                        if (q >= 0) {
                            sample_t* s = &S[ns];
                            s->leaf = q;
                            s->ua = u; s->ub = un;
                            s->delta = (un - u) * dlen;
                            s->smid = 0.5 * (u + un) * dwlen;
                            double x = 0.0;
                            for (int c = 0; c < C; ++c) x += wsig[q * C + c] * b[c];
                            s->x = x; s->sig = density_of(x, density_act);
                            double hs[64];
                            const double* hk = h;
                            if (wgam) {
                                double y = 0.0;
                                for (int c = 0; c < Cg; ++c) y += wgam[q * Cg + c] * bg[c];
                                s->yg = y;
                                s->gam = M_PI * sigmoid(y);
                                for (int k = 0; k < K; ++k) {
                                    double g, dg;
                                    hh_radial(nk[k], lk[k], s->gam, &g, &dg);
                                    hs[k] = g * Yd[k];
                                }
                                hk = hs;
                            }
                            for (int ch = 0; ch < 3; ++ch) {
                                double z = 0.0;
                                for (int k = 0; k < K; ++k) z += hh[(q * 3 + ch) * K + k] * hk[k];
                                s->z[ch] = z; s->c[ch] = sigmoid(z);
                            }
                            /* appearance edit (Sec. 5.2): from frame t_d on, the target colour and,
                               when given (>= 0), the target density replace the leaf's own */
                            if (edit && tau >= edit[q * 5 + 4]) {
                                for (int ch = 0; ch < 3; ++ch) s->c[ch] = edit[q * 5 + ch];
                                if (edit[q * 5 + 3] >= 0.0) s->sig = edit[q * 5 + 3];
                            }
                            double e = exp(-s->sig * s->delta);
                            s->alpha = -expm1(-s->sig * s->delta);
                            s->Tin = Tr;
                            double w = Tr * s->alpha;
                            for (int ch = 0; ch < 3; ++ch) col[ch] += w * s->c[ch];
                            wsum += w;
                            dsum += w * s->smid;
                            Tr *= e;
                            optical += s->sig * s->delta;
                            if (s->delta < min_delta) min_delta = s->delta;
                            ++ns;
                            if (t_stop > 0.0) {
                                double mrg = fabs(Tr - t_stop) / t_stop;
                                if (mrg < min_stop) min_stop = mrg;
                                if (Tr < t_stop) {
                                    if (last_leaf) last_leaf[r] = q;
                                    break;
                                }
                            }
                        }
                        u = un;
                    }
                    if (un >= u_out) break;
                    cell[amin] += dl[amin] > 0.0 ? 1 : -1;
                    if (cell[amin] < 0 || cell[amin] >= Gi) break;
                }
            }
            if (len_out) len_out[r] = dlen;
            if (seg_out) {
                if (ns > seg_cap) {
#pragma omp atomic write
                    err = -4;
                } else {
                    for (int k = 0; k < ns; ++k) {
                        double* o6 = seg_out + ((int64_t)r * seg_cap + k) * 6;
                        o6[0] = S[k].ua; o6[1] = S[k].ub; o6[2] = S[k].sig;
                        o6[3] = S[k].c[0]; o6[4] = S[k].c[1]; o6[5] = S[k].c[2];
                    }
                }
            }
            for (int ch = 0; ch < 3; ++ch) rgb[3 * r + ch] = col[ch];
            alpha[r] = wsum;
            depth_out[r] = wsum > 0.0 ? dsum / wsum : INFINITY;
            nsamp[r] = ns;
            if (tfinal) tfinal[r] = exp(-optical);
            if (margin) { margin[2 * r] = min_delta; margin[2 * r + 1] = min_stop; }

            if (want_grad && ns > 0) {
                double gC[3] = {g_rgb[3 * r], g_rgb[3 * r + 1], g_rgb[3 * r + 2]};
                double gA = g_alpha ? g_alpha[r] : 0.0;
                double Tfin = Tr, prefix[3] = {0, 0, 0}, gb[64], gbg[64];
                for (int c = 0; c < C; ++c) gb[c] = 0.0;
                if (wgam) for (int c = 0; c < Cg; ++c) gbg[c] = 0.0;
                for (int k = 0; k < ns; ++k) {
                    const sample_t* s = &S[k];
                    double w = s->Tin * s->alpha, Tnext = s->Tin * (1.0 - s->alpha);
                    double gdotc = 0.0, gdotsuf = 0.0;
                    for (int ch = 0; ch < 3; ++ch) {
                        prefix[ch] += w * s->c[ch];
                        gdotc += gC[ch] * s->c[ch];
                        gdotsuf += gC[ch] * (col[ch] - prefix[ch]);
                    }
                    /* dC/dsigma_k = delta_k (T_{k+1} c_k - sum_{i>k} w_i c_i); dA/dsigma_k = delta_k T_final */
                    double gsig = s->delta * (Tnext * gdotc - gdotsuf) + gA * s->delta * Tfin;
                    double gx = gsig * (density_act ? (s->x > 0 ? 1.0 : 0.0) : sigmoid(s->x));
                    double hs[64], dhs[64];
                    const double* hk = h;
                    if (wgam) {
                        for (int k = 0; k < K; ++k) {
                            double g, dg;
                            hh_radial(nk[k], lk[k], s->gam, &g, &dg);
                            hs[k] = g * Yd[k];
                            dhs[k] = dg * Yd[k];
                        }
                        hk = hs;
                    }
                    double ggam = 0.0;   /* dL/dgamma of this sample */
                    for (int ch = 0; ch < 3; ++ch) {
                        double gz = gC[ch] * w * s->c[ch] * (1.0 - s->c[ch]);
                        for (int kk = 0; kk < K; ++kk) {
#pragma omp atomic
                            grad_hh[(s->leaf * 3 + ch) * K + kk] += gz * hk[kk];
                            if (wgam) ggam += gz * hh[(s->leaf * 3 + ch) * K + kk] * dhs[kk];
                        }
                    }
                    if (wgam) {
                        double sg = sigmoid(s->yg);
                        double gy = ggam * M_PI * sg * (1.0 - sg);
                        for (int c = 0; c < Cg; ++c) {
                            if (grad_wgam) {
#pragma omp atomic
                                grad_wgam[s->leaf * Cg + c] += gy * bg[c];
                            }
                            gbg[c] += gy * wgam[s->leaf * Cg + c];
                        }
                    }
                    for (int c = 0; c < C; ++c) {
#pragma omp atomic
                        grad_wsig[s->leaf * C + c] += gx * b[c];
                        gb[c] += gx * wsig[s->leaf * C + c];
                    }
                }
                if (grad_basis)
                    for (int c = 0; c < C; ++c) {
#pragma omp atomic
                        grad_basis[i0 * C + c] += (1.0 - f) * gb[c];
#pragma omp atomic
                        grad_basis[i1 * C + c] += f * gb[c];
                    }
                if (wgam && grad_basis_g)
                    for (int c = 0; c < Cg; ++c) {
#pragma omp atomic
                        grad_basis_g[i0 * Cg + c] += (1.0 - f) * gbg[c];
#pragma omp atomic
                        grad_basis_g[i1 * Cg + c] += f * gbg[c];
                    }
            }
        }
        free(S);
    }
    free(hs.keys); free(hs.vals);
    return err;
}

/* Pinhole rays (OpenCV convention: x right, y down, z forward; pixel centres at
   +0.5). Camera: fx, fy, cx, cy and a 3x4 row-major camera-to-world matrix.
   Direction = normalize(R (x_c, y_c, 1)), origin = camera centre; both rounded
   once to float. pix = NULL means all W*H pixels in row-major order. */
void oracle_pinhole_rays(int W, int H, const double* intr /*fx,fy,cx,cy*/, const double* c2w /*[12]*/,
                         int64_t n, const int32_t* pix, float* ray_o, float* ray_d) {
    (void)H;
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = pix ? pix[i] : i;
        int64_t u = p % W, v = p / W;
        double xc = ((double)u + 0.5 - intr[2]) / intr[0];
        double yc = ((double)v + 0.5 - intr[3]) / intr[1];
        double dv[3], nn = 0.0;
        for (int a = 0; a < 3; ++a) {
            dv[a] = c2w[4 * a] * xc + c2w[4 * a + 1] * yc + c2w[4 * a + 2];
            nn += dv[a] * dv[a];
        }
        nn = sqrt(nn);
        for (int a = 0; a < 3; ++a) {
            ray_d[3 * i + a] = (float)(dv[a] / nn);
            ray_o[3 * i + a] = (float)c2w[4 * a + 3];
        }
    }
}
