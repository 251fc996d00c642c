/*
 * fcs_oracle.c -- plain, single-threaded CPU oracle of parameterized
 * calorimeter hit simulation (arXiv 2103.14737).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP implementation; the two
 * are written independently from the same numeric contract.
 *
 * What it follows in the paper:
 *   - CUDA Implementation section, Listing 1 (hit-simulation function): per
 *     (particle, layer) draw the number of hits, give every hit the energy
 *     E_layer / nhit, then run the hit chain on each hit.
 *   - same section: a hit's cell is decided from the particle position and a
 *     random lateral parametrization; 3 random numbers per hit; the energy is
 *     accumulated per cell; the hit cells are gathered as {cell_id, E}.
 *   - Kokkos section, Listing 2 (HitCellMapping): look up the cell containing
 *     (layer, eta, phi) and add the hit energy to it.
 *   - Validation section: bit-level CPU/GPU comparison is made possible by
 *     feeding both sides the same random numbers; here both sides evaluate
 *     the same counter-based generator (Philox4x32-10, Salmon et al. SC'11).
 *
 * Readings where the paper is silent (per-layer energy split, hit-count law,
 * lateral histogram layout, (r, alpha) -> (eta, phi), elementary-function
 * evaluation) are listed in the design notes; each is marked below where it
 * is used.  Accumulation is FP64; per-hit placement is FP32 (the paper's GPU
 * arithmetic) so that cell indices are comparable bit for bit.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Input structures (oracle-private)                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_cells;
    int32_t n_layers;
    int32_t n_regions;
    const float *reg_eta_lo, *reg_eta_hi, *reg_inv_deta, *reg_inv_dphi, *reg_phi_lo;
    const int32_t *reg_neta, *reg_nphi, *reg_offset;
    const float *layer_inv_r;
} og_geom;

typedef struct {
    int32_t n_types, n_ebins, n_etabins, n_layers;
    float r_max;
    const float *e_edges;   /* [n_ebins + 1]   */
    const float *eta_edges; /* [n_etabins + 1] */
    const float *alpha;     /* [n_types * n_layers] Dirichlet concentrations */
    const float *cum;       /* [n_sets * n_layers * 256] cumulative histograms */
} og_param;

typedef struct {
    int32_t pdg;
    float e;
    float eta;
    float phi;
} og_particle;

typedef struct {
    uint64_t seed;
    uint64_t event_index_base;
    float hit_energy_scale;     /* MeV of layer energy per expected hit */
    int32_t nhit_cap;
    double min_layer_energy;    /* layers below this energy get no hits */
    const float *elayer_override; /* [N * L] or NULL */
    int32_t placement_fp64;     /* 1: place hits in FP64 (chain variant) */
    int32_t hit_energy_fluct;   /* 1: per-hit energy factor (chain variant) */
} og_opts;

typedef struct {
    /* per (particle, layer) task, [N * L]; any may be NULL */
    int32_t *n_hits;
    double *elayer;
    float *ehit;
    int32_t *set;
    /* per-event sparse cell list (ascending dense cell index) */
    int64_t cell_cap;
    int64_t *ev_cell_off;   /* [n_events + 1] */
    int32_t *cell_idx;
    double *cell_e;
    int32_t *cell_cnt;
    /* optional hit list in (event, particle, layer, hit) order */
    int64_t hit_cap;
    float *hit_eta, *hit_phi, *hit_e;
    int32_t *hit_cell, *hit_bin;
    /* statistics */
    int64_t n_hits_total, n_out_of_acc, n_cells_nonzero;
} og_out;

enum { OG_OK = 0, OG_E_ARG = -1, OG_E_CAPACITY = -3, OG_E_NOMEM = -6 };

#define NBINS 256
#define TAG_GAMMA 1u
#define TAG_POISSON 2u
#define TAG_HIT 3u
#define TAG_PERTURB 4u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                        */
/* ------------------------------------------------------------------------ */
void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {w0, w1, w2, w3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    oracle_philox(ctr, key, out);
}

/* uniform in (0,1) for the FP64 per-task draws */
static double u64(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }
/* uniform in [0, 1 - 2^-24] for the FP32 per-hit draws (exact conversion) */
static float u24(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

/* ------------------------------------------------------------------------ */
/* Elementary functions of the numeric contract (FP64, +,-,*,/,sqrt only)  */
/* ------------------------------------------------------------------------ */
static const double LN2_HI = 6.93147180369123816490e-01; /* low 32 bits zero */
static const double LN2_LO = 1.90821492927058770002e-10;
static const double INV_LN2 = 1.44269504088896338700e+00;
static const double SQRT_HALF = 0.70710678118654752440;
static const double TWO_PI = 6.28318530717958647692;
static const double HALF_LOG_2PI = 0.91893853320467274178;

/* Each Horner step of the series in oracle_log, oracle_exp and
 * oracle_cos_turns is one fused multiply-add (C fma: a single rounding).
 *
 * natural log for finite x > 0 (normal numbers): x = m 2^e, m in
 * [sqrt(1/2), sqrt(2)), log m = 2 atanh(s), s = (m-1)/(m+1), series to s^21 */
double oracle_log(double x)
{
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e = (int)((bits >> 52) & 0x7ff) - 1022;
    bits = (bits & 0x000fffffffffffffull) | 0x3fe0000000000000ull;
    double m;
    memcpy(&m, &bits, sizeof m);
    if (m < SQRT_HALF) {
        m = m * 2.0;
        e = e - 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double s2 = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    p = fma(p, s2, 1.0);
    double lm = (2.0 * s) * p;
    double k = (double)e;
    return k * LN2_HI + (k * LN2_LO + lm);
}

/* exp: x = k ln2 + r, |r| <= ln2/2, Taylor to r^13, scaled by 2^k */
double oracle_exp(double x)
{
    if (x < -708.0) return 0.0;
    if (x > 709.0) return INFINITY;
    double kd = floor(x * INV_LN2 + 0.5);
    double r = (x - kd * LN2_HI) - kd * LN2_LO;
    double p = 1.0 / 6227020800.0;       /* 1/13! */
    p = fma(p, r, 1.0 / 479001600.0);  /* 1/12! */
    p = fma(p, r, 1.0 / 39916800.0);  /* 1/11! */
    p = fma(p, r, 1.0 / 3628800.0);  /* 1/10! */
    p = fma(p, r, 1.0 / 362880.0);  /* 1/9! */
    p = fma(p, r, 1.0 / 40320.0);  /* 1/8! */
    p = fma(p, r, 1.0 / 5040.0);  /* 1/7! */
    p = fma(p, r, 1.0 / 720.0);  /* 1/6! */
    p = fma(p, r, 1.0 / 120.0);  /* 1/5! */
    p = fma(p, r, 1.0 / 24.0);  /* 1/4! */
    p = fma(p, r, 1.0 / 6.0);  /* 1/3! */
    p = fma(p, r, 0.5);  /* 1/2! */
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    int k = (int)kd;
    double scale;
    if (k < -1000) {
        uint64_t b1 = (uint64_t)(k + 1000 + 1023) << 52;
        memcpy(&scale, &b1, sizeof scale);
        return (p * scale) * 0x1p-1000;
    }
    uint64_t b = (uint64_t)(k + 1023) << 52;
    memcpy(&scale, &b, sizeof scale);
    return p * scale;
}

/* cos(2 pi u): exact reduction in quarter turns to |t| <= pi/4, then Taylor
 * series of cos (to t^16) or sin (to t^17); u in (0,1) for the normal draws,
 * u in [-1/4, 1) for the FP64 placement (the quadrant of a negative multiple
 * of a quarter turn is taken modulo 4). */
double oracle_cos_turns(double u)
{
    double q = floor(4.0 * u + 0.5);
    double f = u - 0.25 * q;
    double t = f * TWO_PI;
    double t2 = t * t;
    int qi = ((int)q) & 3;
    if (qi == 0 || qi == 2) {
        double c = 1.0 / 20922789888000.0;        /* 1/16! */
        c = fma(c, t2, -(1.0 / 87178291200.0));  /* 1/14! */
        c = fma(c, t2, 1.0 / 479001600.0);  /* 1/12! */
        c = fma(c, t2, -(1.0 / 3628800.0));  /* 1/10! */
        c = fma(c, t2, 1.0 / 40320.0);  /* 1/8! */
        c = fma(c, t2, -(1.0 / 720.0));  /* 1/6! */
        c = fma(c, t2, 1.0 / 24.0);  /* 1/4! */
        c = fma(c, t2, -(0.5));  /* 1/2! */
        c = fma(c, t2, 1.0);
        return qi == 0 ? c : -c;
    }
    double s = 1.0 / 355687428096000.0;            /* 1/17! */
    s = fma(s, t2, -(1.0 / 1307674368000.0));  /* 1/15! */
    s = fma(s, t2, 1.0 / 6227020800.0);  /* 1/13! */
    s = fma(s, t2, -(1.0 / 39916800.0));  /* 1/11! */
    s = fma(s, t2, 1.0 / 362880.0);  /* 1/9! */
    s = fma(s, t2, -(1.0 / 5040.0));  /* 1/7! */
    s = fma(s, t2, 1.0 / 120.0);  /* 1/5! */
    s = fma(s, t2, -(1.0 / 6.0));  /* 1/3! */
    s = fma(s, t2, 1.0);
    s = t * s;
    return qi == 1 ? -s : s;
}

/* log(k!) : exact factorials for k < 10, Stirling series beyond */
double oracle_lnfact(int64_t k)
{
    if (k < 10) {
        double f = 1.0;
        for (int64_t j = 2; j <= k; ++j) f = f * (double)j;
        return oracle_log(f);
    }
    double x = (double)k + 1.0;
    double ix = 1.0 / x;
    double ix2 = ix * ix;
    double series = ix * (1.0 / 12.0 - ix2 * (1.0 / 360.0 - ix2 * (1.0 / 1260.0)));
    return (((x - 0.5) * oracle_log(x)) - x) + HALF_LOG_2PI + series;
}

/* ------------------------------------------------------------------------ */
/* Per-(particle, layer) draws                                              */
/* ------------------------------------------------------------------------ */

/* Gamma(alpha, 1) by Marsaglia & Tsang (2000); alpha < 1 via the
 * u^(1/alpha) boost.  Attempt j uses counter (j, layer | 1<<8, p, event). */
double oracle_gamma(double alpha, uint64_t seed, uint32_t layer, uint32_t p, uint32_t ev)
{
    double a = alpha < 1.0 ? alpha + 1.0 : alpha;
    double d = a - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (uint32_t j = 0; j < 64; ++j) {
        uint32_t x[4];
        draw(seed, j, layer | (TAG_GAMMA << 8), p, ev, x);
        double ua = u64(x[0]), ub = u64(x[1]), uc = u64(x[2]), ud = u64(x[3]);
        double z = sqrt(-2.0 * oracle_log(ua)) * oracle_cos_turns(ub);
        double t = 1.0 + c * z;
        if (!(t > 0.0)) continue;
        double v = (t * t) * t;
        double lhs = oracle_log(uc);
        double rhs = ((((0.5 * z) * z) + d) - d * v) + d * oracle_log(v);
        if (lhs < rhs) {
            double g = d * v;
            if (alpha < 1.0) g = g * oracle_exp(oracle_log(ud) / alpha);
            return g;
        }
    }
    return d;
}

/* Poisson(mu): sequential inversion for mu < 10, otherwise the transformed
 * rejection method PTRS (Hoermann 1993), two attempts per Philox call.
 * Call j uses counter (j, layer | 2<<8, p, event). */
int64_t oracle_poisson(double mu, uint64_t seed, uint32_t layer, uint32_t p, uint32_t ev)
{
    uint32_t x[4];
    if (mu < 10.0) {
        draw(seed, 0, layer | (TAG_POISSON << 8), p, ev, x);
        double u = u64(x[0]);
        double pk = oracle_exp(-mu);
        double F = pk;
        int64_t k = 0;
        while (u > F && k < 200) {
            k = k + 1;
            pk = (pk * mu) / (double)k;
            F = F + pk;
        }
        return k;
    }
    double slam = sqrt(mu);
    double loglam = oracle_log(mu);
    double b = 0.931 + 2.53 * slam;
    double a = -0.059 + 0.02483 * b;
    double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (uint32_t j = 0; j < 32; ++j) {
        draw(seed, j, layer | (TAG_POISSON << 8), p, ev, x);
        for (int h = 0; h < 2; ++h) {
            double U = u64(x[2 * h]) - 0.5;
            double V = u64(x[2 * h + 1]);
            double us = 0.5 - fabs(U);
            double kd = floor((((2.0 * a) / us + b) * U + mu) + 0.43);
            if (us >= 0.07 && V <= vr) return (int64_t)kd;
            if (kd < 0.0 || (us < 0.013 && V > us)) continue;
            double lhs = (oracle_log(V) + oracle_log(invalpha)) - oracle_log(a / (us * us) + b);
            double rhs = (-mu + kd * loglam) - oracle_lnfact((int64_t)kd);
            if (lhs <= rhs) return (int64_t)kd;
        }
    }
    return (int64_t)floor(mu);
}

/* ------------------------------------------------------------------------ */
/* Parametrization selection (Introduction: by type, energy and location)  */
/* ------------------------------------------------------------------------ */
int32_t oracle_select_set(const og_param *P, int32_t pdg, float e, float eta)
{
    int32_t apdg = pdg < 0 ? -pdg : pdg;
    int32_t t;
    if (apdg == 11) t = 0;
    else if (apdg == 22) t = 1;
    else if (apdg == 211) t = 2;
    else return -1;
    int32_t ie = 0;
    for (int32_t k = 1; k < P->n_ebins; ++k)
        if (e >= P->e_edges[k]) ie = ie + 1;
    float aeta = fabsf(eta);
    int32_t ih = 0;
    for (int32_t k = 1; k < P->n_etabins; ++k)
        if (aeta >= P->eta_edges[k]) ih = ih + 1;
    return (t * P->n_ebins + ie) * P->n_etabins + ih;
}

/* ------------------------------------------------------------------------ */
/* Lateral histogram: cumulative table and inverse-CDF bin choice          */
/* ------------------------------------------------------------------------ */
/* per histogram: FP64 running sum left to right, divided by the FP64 total,
 * rounded to FP32; the last entry is exactly 1.  Returns -1 on a negative or
 * non-finite weight or an all-zero histogram. */
int oracle_build_cum(const float *w, int64_t n_hist, float *cum)
{
    for (int64_t h = 0; h < n_hist; ++h) {
        const float *wh = w + h * NBINS;
        double W = 0.0;
        for (int b = 0; b < NBINS; ++b) {
            if (!(wh[b] >= 0.0f) || !isfinite(wh[b])) return -1;
            W = W + (double)wh[b];
        }
        if (!(W > 0.0)) return -1;
        double acc = 0.0;
        for (int b = 0; b < NBINS; ++b) {
            acc = acc + (double)wh[b];
            cum[h * NBINS + b] = (float)(acc / W);
        }
        cum[h * NBINS + NBINS - 1] = 1.0f;
    }
    return 0;
}

/* the first bin whose cumulative value exceeds u (plain linear scan) */
int32_t oracle_find_bin(const float *cum, float u)
{
    for (int32_t b = 0; b < NBINS; ++b)
        if (cum[b] > u) return b;
    return NBINS - 1;
}

/* cos and sin of alpha = (ia + u) * pi/4, the angle at fraction u of alpha
 * bin ia: a Taylor polynomial on the offset from the nearest multiple of pi/2
 * (offset in [0, pi/4]), evaluated in Horner form with one fused
 * multiply-add (single rounding, fmaf) per step, and an exact quadrant swap. */
void oracle_sincos_bin(int32_t ia, float u, float *cs, float *sn)
{
    const float Q = (float)(0.78539816339744830962);
    float d;
    int32_t m;
    if ((ia & 1) == 0) {
        d = u * Q;
        m = ia >> 1;
    } else {
        d = (1.0f - u) * Q;
        m = (ia + 1) >> 1;
    }
    float d2 = d * d;
    float sp = (float)(1.0 / 362880.0);
    sp = fmaf(sp, d2, (float)(-1.0 / 5040.0));
    sp = fmaf(sp, d2, (float)(1.0 / 120.0));
    sp = fmaf(sp, d2, (float)(-1.0 / 6.0));
    sp = fmaf(sp, d2, 1.0f);
    float s0 = d * sp;
    float cp = (float)(-1.0 / 3628800.0);
    cp = fmaf(cp, d2, (float)(1.0 / 40320.0));
    cp = fmaf(cp, d2, (float)(-1.0 / 720.0));
    cp = fmaf(cp, d2, (float)(1.0 / 24.0));
    cp = fmaf(cp, d2, -0.5f);
    cp = fmaf(cp, d2, 1.0f);
    float c0 = cp;
    float c, s;
    if ((ia & 1) == 0) { /* alpha = m pi/2 + d */
        switch (m & 3) {
        case 0: c = c0; s = s0; break;
        case 1: c = -s0; s = c0; break;
        case 2: c = -c0; s = -s0; break;
        default: c = s0; s = -c0; break;
        }
    } else {             /* alpha = m pi/2 - d */
        switch (m & 3) {
        case 1: c = s0; s = c0; break;
        case 2: c = -c0; s = s0; break;
        case 3: c = -s0; s = -c0; break;
        default: c = c0; s = -s0; break;
        }
    }
    *cs = c;
    *sn = s;
}

/* ------------------------------------------------------------------------ */
/* Cell lookup (Listing 2, getDDE): region by eta, then a uniform grid     */
/* ------------------------------------------------------------------------ */
int32_t oracle_lookup(const og_geom *G, int32_t layer, float eta, float phi)
{
    const int32_t R = G->n_regions;
    const int32_t base = layer * R;
    if (!(eta >= G->reg_eta_lo[base]) || !(eta < G->reg_eta_hi[base + R - 1])) return -1;
    int32_t k = 0;
    for (int32_t j = 1; j < R; ++j)
        if (eta >= G->reg_eta_lo[base + j]) k = k + 1;
    const int32_t r = base + k;
    int32_t ie = (int32_t)floorf((eta - G->reg_eta_lo[r]) * G->reg_inv_deta[r]);
    int32_t ip = (int32_t)floorf((phi - G->reg_phi_lo[r]) * G->reg_inv_dphi[r]);
    if (ie < 0) ie = 0;
    if (ie > G->reg_neta[r] - 1) ie = G->reg_neta[r] - 1;
    if (ip < 0) ip = 0;
    if (ip > G->reg_nphi[r] - 1) ip = G->reg_nphi[r] - 1;
    return G->reg_offset[r] + ie * G->reg_nphi[r] + ip;
}

/* ------------------------------------------------------------------------ */
/* One hit: three uniforms -> bin -> (r, alpha) -> (eta, phi) -> cell       */
/* ------------------------------------------------------------------------ */
typedef struct {
    float eta, phi;
    int32_t bin, cell;
    uint32_t w4; /* the draw's fourth word */
} og_hit;

static og_hit one_hit(const og_geom *G, const float *cum, float r_max, uint64_t seed,
                      uint32_t i, uint32_t layer, uint32_t p, uint32_t ev,
                      float eta_p, float phi_p)
{
    const float PI_F = 3.14159265358979323846f;
    const float TWO_PI_F = 6.28318530717958647692f;
    uint32_t x[4];
    draw(seed, i, layer | (TAG_HIT << 8), p, ev, x);
    float u0 = u24(x[0]), u1 = u24(x[1]), u2 = u24(x[2]);
    og_hit h;
    h.w4 = x[3];
    h.bin = oracle_find_bin(cum, u0);
    int32_t ir = h.bin >> 3, ia = h.bin & 7;
    float dr = r_max / 32.0f;
    /* radius uniform in the bin: lower edge ir * dr plus u1 * dr, one fused
     * multiply-add */
    float r = fmaf(u1, dr, (float)ir * dr);
    float c, s;
    oracle_sincos_bin(ia, u2, &c, &s);
    float inv_r = G->layer_inv_r[layer];
    float deta = (r * c) * inv_r;
    float dphi = (r * s) * inv_r;
    float eta = eta_p + deta;
    float phi = phi_p + dphi;
    if (phi >= PI_F) phi = phi - TWO_PI_F;
    else if (phi < -PI_F) phi = phi + TWO_PI_F;
    h.eta = eta;
    h.phi = phi;
    h.cell = oracle_lookup(G, (int32_t)layer, eta, phi);
    return h;
}

/* ------------------------------------------------------------------------ */
/* FP64 placement (a chain variant of the same hit; Validation section: the  */
/* rounding of the placement decides the cell of a few hits)                */
/* ------------------------------------------------------------------------ */
/* The cell lookup of oracle_lookup with the position and every product in
 * FP64, the FP32 geometry values promoted. */
static int32_t lookup_f64(const og_geom *G, int32_t layer, double eta, double phi)
{
    const int32_t R = G->n_regions;
    const int32_t base = layer * R;
    if (!(eta >= (double)G->reg_eta_lo[base]) || !(eta < (double)G->reg_eta_hi[base + R - 1]))
        return -1;
    int32_t k = 0;
    for (int32_t j = 1; j < R; ++j)
        if (eta >= (double)G->reg_eta_lo[base + j]) k = k + 1;
    const int32_t r = base + k;
    int32_t ie = (int32_t)floor((eta - (double)G->reg_eta_lo[r]) * (double)G->reg_inv_deta[r]);
    int32_t ip = (int32_t)floor((phi - (double)G->reg_phi_lo[r]) * (double)G->reg_inv_dphi[r]);
    if (ie < 0) ie = 0;
    if (ie > G->reg_neta[r] - 1) ie = G->reg_neta[r] - 1;
    if (ip < 0) ip = 0;
    if (ip > G->reg_nphi[r] - 1) ip = G->reg_nphi[r] - 1;
    return G->reg_offset[r] + ie * G->reg_nphi[r] + ip;
}

/* The hit of one_hit (same counter, uniforms and bin) placed in FP64: the
 * radius (ir + u1) * dr, the angle at t = (ia + u2) / 8 turns with its
 * cosine and sine (the cosine a quarter turn back) from oracle_cos_turns,
 * then the same (eta, phi) formulas, the phi wrap and the lookup, all in
 * FP64; the position is returned rounded to FP32. */
static og_hit one_hit_f64(const og_geom *G, const float *cum, float r_max, uint64_t seed,
                          uint32_t i, uint32_t layer, uint32_t p, uint32_t ev,
                          float eta_p, float phi_p)
{
    uint32_t x[4];
    draw(seed, i, layer | (TAG_HIT << 8), p, ev, x);
    float u0 = u24(x[0]), u1 = u24(x[1]), u2 = u24(x[2]);
    og_hit h;
    h.w4 = x[3];
    h.bin = oracle_find_bin(cum, u0);
    int32_t ir = h.bin >> 3, ia = h.bin & 7;
    double r = ((double)ir + (double)u1) * (double)(r_max / 32.0f);
    double t = ((double)ia + (double)u2) * 0.125;
    double c = oracle_cos_turns(t);
    double s = oracle_cos_turns(t - 0.25);
    double inv_r = (double)G->layer_inv_r[layer];
    double eta = (double)eta_p + (r * c) * inv_r;
    double phi = (double)phi_p + (r * s) * inv_r;
    if (phi >= 3.14159265358979323846) phi = phi - TWO_PI;
    else if (phi < -3.14159265358979323846) phi = phi + TWO_PI;
    h.eta = (float)eta;
    h.phi = (float)phi;
    h.cell = lookup_f64(G, (int32_t)layer, eta, phi);
    return h;
}

/* Per-hit energy fluctuation (a chain variant of the constant Ehit of
 * Listing 1): the hit's energy is Ehit * x with x = -ln u exponential of
 * mean 1, u = ((w4 >> 8) + 1/2) 2^-24 from the draw's unused fourth word,
 * x in FP64 with oracle_log, one rounding to FP32. */
static double fluct_factor(uint32_t w4)
{
    double u = ((double)(w4 >> 8) + 0.5) * 0x1p-24;
    return -oracle_log(u);
}

static float fluct_energy(float ehit, uint32_t w4)
{
    return (float)((double)ehit * fluct_factor(w4));
}

/* exported single-hit evaluation for tests */
int32_t oracle_hit(const og_geom *G, const float *cum, float r_max, uint64_t seed, uint32_t i,
                   uint32_t layer, uint32_t p, uint32_t ev, float eta_p, float phi_p,
                   float *eta_out, float *phi_out, int32_t *bin_out)
{
    og_hit h = one_hit(G, cum, r_max, seed, i, layer, p, ev, eta_p, phi_p);
    *eta_out = h.eta;
    *phi_out = h.phi;
    *bin_out = h.bin;
    return h.cell;
}

/* ------------------------------------------------------------------------ */
/* Per-particle setup: set, Dirichlet layer energies, hit counts, Ehit      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t set;
    int32_t n[64];
    double elayer[64];
    float ehit[64];
} og_setup;

static int particle_setup(const og_param *P, const og_opts *O, const og_particle *pt,
                          int64_t task0, uint32_t p, uint32_t ev, og_setup *S)
{
    const int32_t L = P->n_layers;
    S->set = oracle_select_set(P, pt->pdg, pt->e, pt->eta);
    if (S->set < 0) return OG_E_ARG;
    int32_t t = S->set / (P->n_ebins * P->n_etabins);
    double g[64];
    double sum = 0.0;
    for (int32_t l = 0; l < L; ++l) {
        g[l] = oracle_gamma((double)P->alpha[t * L + l], O->seed, (uint32_t)l, p, ev);
        sum = sum + g[l];
    }
    for (int32_t l = 0; l < L; ++l) {
        double el = (double)pt->e * (g[l] / sum);
        S->elayer[l] = el;
        int32_t n = 0;
        if (el >= O->min_layer_energy && el > 0.0) {
            double mu = el / (double)O->hit_energy_scale;
            int64_t k = oracle_poisson(mu, O->seed, (uint32_t)l, p, ev);
            if (k < 1) k = 1;
            if (k > O->nhit_cap) k = O->nhit_cap;
            n = (int32_t)k;
        }
        S->n[l] = n;
        double e_used = O->elayer_override ? (double)O->elayer_override[task0 + l] : el;
        S->ehit[l] = n > 0 ? (float)(e_used / (double)n) : 0.0f;
    }
    return OG_OK;
}

/* ------------------------------------------------------------------------ */
/* The event loop                                                           */
/* ------------------------------------------------------------------------ */
int oracle_simulate(const og_geom *G, const og_param *P, const og_particle *parts,
                    const int64_t *ev_off, int64_t n_events, const og_opts *O, og_out *out)
{
    const int32_t L = P->n_layers;
    if (L > 64 || L != G->n_layers) return OG_E_ARG;
    const int64_t C = G->n_cells;
    double *cellE = (double *)calloc((size_t)C, sizeof(double));
    int32_t *cellN = (int32_t *)calloc((size_t)C, sizeof(int32_t));
    int32_t *touched = (int32_t *)malloc((size_t)C * sizeof(int32_t));
    if (!cellE || !cellN || !touched) {
        free(cellE); free(cellN); free(touched);
        return OG_E_NOMEM;
    }
    int rc = OG_OK;
    int64_t ncell_out = 0, nhit_out = 0;
    out->n_hits_total = 0;
    out->n_out_of_acc = 0;
    if (out->ev_cell_off) out->ev_cell_off[0] = 0;
    for (int64_t e = 0; e < n_events && rc == OG_OK; ++e) {
        const uint32_t ev = (uint32_t)(O->event_index_base + (uint64_t)e);
        int64_t n_touched = 0;
        for (int64_t gp = ev_off[e]; gp < ev_off[e + 1]; ++gp) {
            const uint32_t p = (uint32_t)(gp - ev_off[e]);
            const og_particle *pt = &parts[gp];
            og_setup S;
            rc = particle_setup(P, O, pt, gp * L, p, ev, &S);
            if (rc != OG_OK) break;
            for (int32_t l = 0; l < L; ++l) {
                const int64_t task = gp * L + l;
                if (out->n_hits) out->n_hits[task] = S.n[l];
                if (out->elayer) out->elayer[task] = S.elayer[l];
                if (out->ehit) out->ehit[task] = S.ehit[l];
                if (out->set) out->set[task] = S.set;
                const float *cum = P->cum + ((int64_t)S.set * L + l) * NBINS;
                for (int32_t i = 0; i < S.n[l]; ++i) {
                    og_hit h = O->placement_fp64
                                   ? one_hit_f64(G, cum, P->r_max, O->seed, (uint32_t)i, (uint32_t)l,
                                                 p, ev, pt->eta, pt->phi)
                                   : one_hit(G, cum, P->r_max, O->seed, (uint32_t)i, (uint32_t)l, p,
                                             ev, pt->eta, pt->phi);
                    const float e_hit = O->hit_energy_fluct ? fluct_energy(S.ehit[l], h.w4)
                                                            : S.ehit[l];
                    out->n_hits_total++;
                    if (h.cell < 0) {
                        out->n_out_of_acc++;
                    } else {
                        if (cellN[h.cell] == 0) touched[n_touched++] = h.cell;
                        cellN[h.cell] += 1;
                        cellE[h.cell] += (double)e_hit;
                    }
                    if (out->hit_eta) {
                        if (nhit_out >= out->hit_cap) {
                            rc = OG_E_CAPACITY;
                        } else {
                            out->hit_eta[nhit_out] = h.eta;
                            out->hit_phi[nhit_out] = h.phi;
                            out->hit_e[nhit_out] = e_hit;
                            out->hit_cell[nhit_out] = h.cell;
                            if (out->hit_bin) out->hit_bin[nhit_out] = h.bin;
                        }
                        nhit_out++;
                    }
                }
            }
        }
        /* gather the event's hit cells in ascending cell order (cells whose
         * hits all carry zero energy, possible only with an override, are
         * left out) */
        for (int64_t c = 0, done = 0; c < C && done < n_touched; ++c) {
            if (cellN[c] == 0) continue;
            done++;
            if (cellE[c] == 0.0) {
                cellN[c] = 0;
                continue;
            }
            if (ncell_out < out->cell_cap && out->cell_idx) {
                out->cell_idx[ncell_out] = (int32_t)c;
                out->cell_e[ncell_out] = cellE[c];
                if (out->cell_cnt) out->cell_cnt[ncell_out] = cellN[c];
            } else if (out->cell_idx) {
                rc = OG_E_CAPACITY;
            }
            ncell_out++;
            cellN[c] = 0;
            cellE[c] = 0.0;
        }
        if (out->ev_cell_off) out->ev_cell_off[e + 1] = ncell_out;
    }
    out->n_cells_nonzero = ncell_out;
    free(cellE);
    free(cellN);
    free(touched);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Differentiable form                                                      */
/* ------------------------------------------------------------------------ */

/* Perturbed layer energies for the loss targets: f'_l = max(f_l (1 + sigma
 * z_l), 0) renormalized, E'_l = E f'_l, with z_l a Box-Muller normal from
 * counter (0, layer | 4<<8, p, event). */
int oracle_perturbed_elayer(const og_param *P, const og_particle *parts, const int64_t *ev_off,
                            int64_t n_events, const og_opts *O, double sigma, float *eprime)
{
    const int32_t L = P->n_layers;
    og_opts o2 = *O;
    o2.elayer_override = NULL;
    for (int64_t e = 0; e < n_events; ++e) {
        const uint32_t ev = (uint32_t)(O->event_index_base + (uint64_t)e);
        for (int64_t gp = ev_off[e]; gp < ev_off[e + 1]; ++gp) {
            const uint32_t p = (uint32_t)(gp - ev_off[e]);
            og_setup S;
            int rc = particle_setup(P, &o2, &parts[gp], gp * L, p, ev, &S);
            if (rc != OG_OK) return rc;
            double tot = 0.0, fp[64];
            for (int32_t l = 0; l < L; ++l) tot = tot + S.elayer[l];
            double s2 = 0.0;
            for (int32_t l = 0; l < L; ++l) {
                uint32_t x[4];
                draw(O->seed, 0, (uint32_t)l | (TAG_PERTURB << 8), p, ev, x);
                double z = sqrt(-2.0 * oracle_log(u64(x[0]))) * oracle_cos_turns(u64(x[1]));
                double f = S.elayer[l] / tot;
                double v = f * (1.0 + sigma * z);
                fp[l] = v > 0.0 ? v : 0.0;
                s2 = s2 + fp[l];
            }
            for (int32_t l = 0; l < L; ++l)
                eprime[gp * L + l] = (float)((double)parts[gp].e * (s2 > 0.0 ? fp[l] / s2 : 0.0));
        }
    }
    return OG_OK;
}

/* Gradient of L = sum_c (E_c - T_c)^2 given g_c = dL/dE_c (dense, [n_events *
 * n_cells]).  Hit counts are frozen, so E_c is linear in the layer energy:
 *   dL/dE_l = (1/n_l) sum_{hits of the layer, in acceptance} g_{cell(hit)}.
 * Histogram weights use the likelihood-ratio surrogate with samples frozen at
 * the loaded weights w0: deposits carry p_b(w)/p_b(w0), p_b = w_b / W, so
 *   dL/dw_k = A_k / w_k - S / W,  A_k = sum_{hits in bin k} g Ehit,
 *   S = sum_k A_k   (bins with w_k = 0 are never sampled: A_k = 0).
 * grad_elayer [N * L], grad_w [n_hist * 256] (FP64). */
int oracle_gradient(const og_geom *G, const og_param *P, const float *w0, int64_t n_hist,
                    const og_particle *parts, const int64_t *ev_off, int64_t n_events,
                    const og_opts *O, const float *grad_cells, double *grad_elayer,
                    double *grad_w)
{
    const int32_t L = P->n_layers;
    const int64_t C = G->n_cells;
    double *A = (double *)calloc((size_t)(n_hist * NBINS), sizeof(double));
    if (!A) return OG_E_NOMEM;
    for (int64_t e = 0; e < n_events; ++e) {
        const uint32_t ev = (uint32_t)(O->event_index_base + (uint64_t)e);
        for (int64_t gp = ev_off[e]; gp < ev_off[e + 1]; ++gp) {
            const uint32_t p = (uint32_t)(gp - ev_off[e]);
            const og_particle *pt = &parts[gp];
            og_setup S;
            int rc = particle_setup(P, O, pt, gp * L, p, ev, &S);
            if (rc != OG_OK) { free(A); return rc; }
            for (int32_t l = 0; l < L; ++l) {
                const int64_t H = (int64_t)S.set * L + l;
                const float *cum = P->cum + H * NBINS;
                double gsum = 0.0;
                for (int32_t i = 0; i < S.n[l]; ++i) {
                    og_hit h = one_hit(G, cum, P->r_max, O->seed, (uint32_t)i, (uint32_t)l, p,
                                       ev, pt->eta, pt->phi);
                    if (h.cell < 0) continue;
                    double gc = (double)grad_cells[e * C + h.cell];
                    if (O->hit_energy_fluct) {
                        /* E_hit = (E_l / n) x: d E_hit / d E_l = x / n (the
                         * rounding of E_hit taken as identity) */
                        gsum = gsum + gc * fluct_factor(h.w4);
                        A[H * NBINS + h.bin] += gc * (double)fluct_energy(S.ehit[l], h.w4);
                    } else {
                        gsum = gsum + gc;
                        A[H * NBINS + h.bin] += gc * (double)S.ehit[l];
                    }
                }
                grad_elayer[gp * L + l] = S.n[l] > 0 ? gsum / (double)S.n[l] : 0.0;
            }
        }
    }
    for (int64_t H = 0; H < n_hist; ++H) {
        double W = 0.0, Ssum = 0.0;
        for (int b = 0; b < NBINS; ++b) {
            W = W + (double)w0[H * NBINS + b];
            Ssum = Ssum + A[H * NBINS + b];
        }
        for (int b = 0; b < NBINS; ++b) {
            double wb = (double)w0[H * NBINS + b];
            double lr = wb > 0.0 ? A[H * NBINS + b] / wb : 0.0;
            grad_w[H * NBINS + b] = lr - Ssum / W;
        }
    }
    free(A);
    return OG_OK;
}

/* The frozen-sample surrogate loss at weights w (samples drawn with the
 * cumulative tables built from w0): each hit deposits Ehit p_b(w)/p_b(w0).
 * targets: dense [n_events * n_cells].  Used to check the weight gradient by
 * finite differences. */
double oracle_surrogate_loss(const og_geom *G, const og_param *P, const float *w0,
                             const double *w, int64_t n_hist, const og_particle *parts,
                             const int64_t *ev_off, int64_t n_events, const og_opts *O,
                             const double *targets)
{
    const int32_t L = P->n_layers;
    const int64_t C = G->n_cells;
    double *W0 = (double *)malloc((size_t)n_hist * sizeof(double));
    double *W1 = (double *)malloc((size_t)n_hist * sizeof(double));
    double *cells = (double *)calloc((size_t)C, sizeof(double));
    if (!W0 || !W1 || !cells) { free(W0); free(W1); free(cells); return NAN; }
    for (int64_t H = 0; H < n_hist; ++H) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < NBINS; ++k) {
            a = a + (double)w0[H * NBINS + k];
            b = b + w[H * NBINS + k];
        }
        W0[H] = a;
        W1[H] = b;
    }
    double loss = 0.0;
    for (int64_t e = 0; e < n_events; ++e) {
        const uint32_t ev = (uint32_t)(O->event_index_base + (uint64_t)e);
        memset(cells, 0, (size_t)C * sizeof(double));
        for (int64_t gp = ev_off[e]; gp < ev_off[e + 1]; ++gp) {
            const uint32_t p = (uint32_t)(gp - ev_off[e]);
            const og_particle *pt = &parts[gp];
            og_setup S;
            if (particle_setup(P, O, pt, gp * L, p, ev, &S) != OG_OK) { loss = NAN; break; }
            for (int32_t l = 0; l < L; ++l) {
                const int64_t H = (int64_t)S.set * L + l;
                const float *cum = P->cum + H * NBINS;
                for (int32_t i = 0; i < S.n[l]; ++i) {
                    og_hit h = one_hit(G, cum, P->r_max, O->seed, (uint32_t)i, (uint32_t)l, p,
                                       ev, pt->eta, pt->phi);
                    if (h.cell < 0) continue;
                    double ratio = (w[H * NBINS + h.bin] / W1[H]) /
                                   ((double)w0[H * NBINS + h.bin] / W0[H]);
                    float e_hit = O->hit_energy_fluct ? fluct_energy(S.ehit[l], h.w4) : S.ehit[l];
                    cells[h.cell] += (double)e_hit * ratio;
                }
            }
        }
        for (int64_t c = 0; c < C; ++c) {
            double d = cells[c] - targets[e * C + c];
            loss = loss + d * d;
        }
    }
    free(W0); free(W1); free(cells);
    return loss;
}

/* ------------------------------------------------------------------------ */
/* Batch helpers for the statistical pins                                   */
/* ------------------------------------------------------------------------ */
void oracle_gamma_batch(double alpha, uint64_t seed, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_gamma(alpha, seed, 0, (uint32_t)i, 0);
}

void oracle_poisson_batch(double mu, uint64_t seed, int64_t n, int64_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_poisson(mu, seed, 0, (uint32_t)i, 0);
}

void oracle_sincos_batch(const int32_t *ia, const float *u, int64_t n, float *c, float *s)
{
    for (int64_t i = 0; i < n; ++i) oracle_sincos_bin(ia[i], u[i], &c[i], &s[i]);
}

void oracle_log_batch(const double *x, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_log(x[i]);
}

void oracle_exp_batch(const double *x, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_exp(x[i]);
}

void oracle_cos_turns_batch(const double *u, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_cos_turns(u[i]);
}

void oracle_lookup_batch(const og_geom *G, const int32_t *layer, const float *eta,
                         const float *phi, int64_t n, int32_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_lookup(G, layer[i], eta[i], phi[i]);
}

void oracle_find_bin_batch(const float *cum, const float *u, int64_t n, int32_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_find_bin(cum, u[i]);
}

void oracle_philox_batch(const uint32_t *ctr, const uint32_t key[2], int64_t n, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) oracle_philox(ctr + 4 * i, key, out + 4 * i);
}
