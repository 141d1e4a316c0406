/*
 * CPU oracle for the GI-1.0 per-frame indirect-lighting pass (two-level radiance caching).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file;
 * only tests, the smoke check and the CPU baseline of the benchmark do.  It shares no code
 * with the HIP library: every definition here is written out again, plainly, from the
 * method's description.
 *
 * The file is compiled twice:
 *   - FP32 parity mode (default): the same float32 operation order as the GPU path, so that
 *     every float-derived integer (hit index, hit distance bits, cell key, hemisphere cell,
 *     fixed-point sums) is reproduced bit for bit.  Build with -ffp-contract=off.
 *   - FP64 reference mode (-DORC_F64): the same algorithm in double precision and without
 *     fixed-point quantisation of the cache samples; used for closed forms and converged
 *     references.
 *
 * Section references are to the GI-1.0 paper (Boisse et al., 2022):
 *   Section 2.1.1 spawning, probe reprojection (Algorithm 1) and temporal upscaling, 2.1.2
 *   adaptive sampling (Algorithm 2) and ray guiding with the parallax-corrected
 *   reconstruction, 2.1.3 ray tracing of probes, 2.1.4 radiance blending (Algorithm 3) and
 *   backup, 2.1.5 probe masking (Algorithm 4), 2.1.6 probe-space filter (Algorithm 5), 2.1.7
 *   adaptive cell size (Algorithm 6), 2.2.1 spatial-hash world cache and its levels of
 *   detail, 2.2.2 light-leak bit, 2.2.3 temporal accumulation into cells and the two-level
 *   tiled cache with MIP prefiltering, 2.2.4 radiance feedback, 2.3 light sampling (one
 *   shadow ray; RIS over the light grid; world-space reservoir reuse), 2.4.1 per-pixel
 *   interpolation, 2.4.2 spherical harmonics (with SH reprojection), 2.4.3 screen-space denoising.
 * Definitions that the paper leaves open are marked READING and listed in the design notes.
 *
 * parity unpinned: none of the functions below lacks a pin; see tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_F64
typedef double real;
#define ORC(n) orc64_##n
#define RC(x) (x)
#define RSQRT(x) sqrt(x)
#define RFLOOR(x) floor(x)
#define RABS(x) fabs(x)
#else
typedef float real;
#define ORC(n) orc32_##n
#define RC(x) (x##f)
#define RSQRT(x) sqrtf(x)
#define RFLOOR(x) floorf(x)
#define RABS(x) fabsf(x)
#endif

#define MISS 0xFFFFFFFFu
#define SENTINEL 0xFFFFFFFFu
#define BUCKET 32u
#define NCELL 64

static real rmax(real a, real b) { return a > b ? a : b; }
static real rmin(real a, real b) { return a < b ? a : b; }

/* ---------------------------------------------------------------------------------------
 * Integer hashes (the two hash functions of the world cache, Section 2.2.1, and the
 * counter-based random numbers).  READING: the paper names only the survey of GPU hash
 * functions by Jarzynski and Olano (2020); we take its PCG-based hash for bucket selection
 * and random numbers, and the 32-bit xxHash finaliser for fingerprints.
 * ------------------------------------------------------------------------------------- */
static uint32_t pcg_hash(uint32_t v)
{
    uint32_t state = v * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

static uint32_t xxh32_hash(uint32_t v)
{
    /* XXH32 of the 4 little-endian bytes of v with seed 0: short-input path, then the
     * avalanche finaliser, with the published primes */
    uint32_t h = 374761393u + 4u;
    h += v * 3266489917u;
    h = ((h << 17) | (h >> 15)) * 668265263u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    h *= 3266489917u;
    h ^= h >> 16;
    return h;
}

/* random 32-bit word for (seed, frame, stream id, dimension): nested PCG hashing */
static uint32_t rng_u32(uint32_t seed, uint32_t frame, uint32_t id, uint32_t dim)
{
    return pcg_hash(dim + pcg_hash(id + pcg_hash(frame + pcg_hash(seed))));
}

/* top 24 bits of the word as a float in [0,1); exact in float32 */
static real rng_unit(uint32_t h)
{
    return (real)(h >> 8) * RC(5.9604644775390625e-08);
}

uint32_t ORC(pcg)(uint32_t v) { return pcg_hash(v); }
uint32_t ORC(xxh32)(uint32_t v) { return xxh32_hash(v); }
uint32_t ORC(rng)(uint32_t s, uint32_t f, uint32_t id, uint32_t k) { return rng_u32(s, f, id, k); }

/* number of repeated outputs of a hash over inputs [0, n) (test of injectivity); which = 0
 * for the PCG hash, 1 for XXH32 */
uint64_t ORC(hash_collisions)(uint32_t which, uint64_t n)
{
    uint64_t *bits = (uint64_t *)calloc((size_t)1 << 26, sizeof(uint64_t));
    uint64_t rep = 0;
    if (!bits) return ~(uint64_t)0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t h = which ? xxh32_hash((uint32_t)i) : pcg_hash((uint32_t)i);
        uint64_t m = (uint64_t)1 << (h & 63u);
        if (bits[h >> 6] & m) ++rep;
        bits[h >> 6] |= m;
    }
    free(bits);
    return rep;
}

/* ---------------------------------------------------------------------------------------
 * sin/cos of 2*pi*u for u in [0,1) without a library transcendental, so that both sides
 * produce identical bits.  Exact octant reduction (8u is exact), then Taylor polynomials
 * with coefficients 1/n! on [0, pi/4].  In FP64 mode the library functions are used.
 * ------------------------------------------------------------------------------------- */
static void sincos_2pi(real u, real *c_out, real *s_out)
{
#ifdef ORC_F64
    *c_out = cos(6.283185307179586 * u);
    *s_out = sin(6.283185307179586 * u);
#else
    float v = u * 8.0f;
    int k = (int)v;
    float fr = v - (float)k;
    float g = (k & 1) ? (1.0f - fr) : fr;
    float x = g * 0.785398163397448310f;
    float x2 = x * x;
    float s = x * (1.0f + x2 * (-0.166666666666666667f + x2 * (0.00833333333333333333f +
              x2 * (-0.000198412698412698413f + x2 * 2.75573192239858907e-06f))));
    float c = 1.0f + x2 * (-0.5f + x2 * (0.0416666666666666667f + x2 * (-0.00138888888888888889f +
              x2 * (2.48015873015873016e-05f + x2 * -2.75573192239858907e-07f))));
    float co, si;
    switch (k & 7) {
    case 0: co = c; si = s; break;
    case 1: co = s; si = c; break;
    case 2: co = -s; si = c; break;
    case 3: co = -c; si = s; break;
    case 4: co = -c; si = -s; break;
    case 5: co = -s; si = -c; break;
    case 6: co = s; si = -c; break;
    default: co = c; si = -s; break;
    }
    *c_out = co;
    *s_out = si;
#endif
}

void ORC(sincos2pi)(const real *u, uint32_t n, real *c, real *s)
{
    for (uint32_t i = 0; i < n; ++i) sincos_2pi(u[i], &c[i], &s[i]);
}

/* ---------------------------------------------------------------------------------------
 * Halton jitter of the spawn tile (Section 2.1.1): one jitter per frame, index f+1, bases 2
 * and 3, taken as floor(8 * radical_inverse) in exact integer arithmetic.  READING: the
 * paper does not say whether the jitter is per frame or per tile; per frame keeps the probe
 * grid regular for interpolation.
 * ------------------------------------------------------------------------------------- */
/* floor(n * radical inverse of index in base), exactly: the radical inverse is num / den */
static uint32_t halton_n(uint32_t index, uint32_t base, uint32_t n)
{
    uint64_t num = 0, den = 1;
    uint32_t i = index;
    while (i > 0) {
        num = num * base + (i % base);
        den *= base;
        i /= base;
    }
    return (uint32_t)(((uint64_t)n * num) / den);
}


void ORC(halton_jitter)(uint32_t frame, uint32_t n, uint32_t *jx, uint32_t *jy)
{
    *jx = halton_n(frame + 1u, 2u, n);
    *jy = halton_n(frame + 1u, 3u, n);
}

/* ---------------------------------------------------------------------------------------
 * Scene: triangles, unit geometric normals, emitters
 * ------------------------------------------------------------------------------------- */
typedef struct bnode {
    float lo[3], hi[3];
    uint32_t left;    /* inner: index of first child (second is left+1); leaf: first tri slot */
    uint32_t count;   /* 0 = inner node, else number of triangles */
} bnode;

typedef struct scene {
    uint32_t nt, nd, nm;
    float *tv;          /* [(nt+nd)][9] triangle vertices */
    real *tn;           /* [(nt+nd)][3] unit winding normal */
    uint32_t *tmat;     /* [(nt+nd)] */
    float *mats;        /* [nm][6] albedo rgb, Le rgb */
    uint32_t nd_cap;
    /* emitters over static and dynamic triangles */
    uint32_t ne;
    uint32_t *etri;
    uint32_t *ethr;
    real area_total;
    /* binary BVH over static triangles */
    bnode *nodes;
    uint32_t nnodes;
    uint32_t *order;
    int use_bvh;
} scene;

static void tri_normal(const float *v, real *n)
{
    real e1x = (real)v[3] - (real)v[0], e1y = (real)v[4] - (real)v[1], e1z = (real)v[5] - (real)v[2];
    real e2x = (real)v[6] - (real)v[0], e2y = (real)v[7] - (real)v[1], e2z = (real)v[8] - (real)v[2];
    real cx = e1y * e2z - e1z * e2y;
    real cy = e1z * e2x - e1x * e2z;
    real cz = e1x * e2y - e1y * e2x;
    real len = RSQRT(cx * cx + cy * cy + cz * cz);
    if (len > RC(0.0)) {
        n[0] = cx / len;
        n[1] = cy / len;
        n[2] = cz / len;
    } else {
        n[0] = n[1] = n[2] = RC(0.0);
    }
}

static double tri_area_f64(const float *v)
{
    double e1x = (double)v[3] - v[0], e1y = (double)v[4] - v[1], e1z = (double)v[5] - v[2];
    double e2x = (double)v[6] - v[0], e2y = (double)v[7] - v[1], e2z = (double)v[8] - v[2];
    double cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
    return 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
}

static int is_emitter(const scene *sc, uint32_t tri)
{
    const float *m = sc->mats + 6 * sc->tmat[tri];
    return m[3] > 0.0f || m[4] > 0.0f || m[5] > 0.0f;
}

/* Area-proportional emitter selection (one light sample per hit, the single-sample form of
 * the light sampling of Section 2.3.1).  Thresholds are the float64 running area sums,
 * scaled to 2^32; the last threshold is 2^32-1. */
static void build_emitters(scene *sc)
{
    uint32_t total = sc->nt + sc->nd;
    free(sc->etri);
    free(sc->ethr);
    sc->etri = NULL;
    sc->ethr = NULL;
    sc->ne = 0;
    uint32_t n = 0;
    for (uint32_t i = 0; i < total; ++i) n += is_emitter(sc, i) ? 1u : 0u;
    sc->area_total = RC(0.0);
    if (n == 0) return;
    sc->etri = (uint32_t *)malloc(sizeof(uint32_t) * n);
    sc->ethr = (uint32_t *)malloc(sizeof(uint32_t) * n);
    double *pre = (double *)malloc(sizeof(double) * n);
    double acc = 0.0;
    uint32_t k = 0;
    for (uint32_t i = 0; i < total; ++i) {
        if (!is_emitter(sc, i)) continue;
        acc += tri_area_f64(sc->tv + 9 * (size_t)i);
        pre[k] = acc;
        sc->etri[k++] = i;
    }
    for (uint32_t i = 0; i < n; ++i) {
        double t = floor(pre[i] / acc * 4294967296.0);
        sc->ethr[i] = (i + 1 == n || t >= 4294967295.0) ? 4294967295u : (uint32_t)t;
    }
    sc->ne = n;
    sc->area_total = (real)acc;
    free(pre);
}

static uint32_t pick_emitter(const scene *sc, uint32_t r)
{
    uint32_t lo = 0, hi = sc->ne - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2u;
        if (r < sc->ethr[mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

/* ---------------------------------------------------------------------------------------
 * Watertight ray/triangle intersection (Woop, Benthin and Wald, JCGT 2013), two-sided,
 * accepting 0 < t < tmax.  The paper traces closest-hit and any-hit queries (Section 2.1.3,
 * Section 4) with hardware traversal; the query result is defined here triangle by triangle.
 * ------------------------------------------------------------------------------------- */
typedef struct rayp {
    real o[3], d[3], inv[3];
    int kx, ky, kz;
    real sx, sy, sz;
} rayp;

static void ray_setup(rayp *r, const real *o, const real *d)
{
    for (int i = 0; i < 3; ++i) {
        r->o[i] = o[i];
        r->d[i] = d[i];
        /* a tiny stand-in for zero components keeps the slab test finite and conservative */
        real di = d[i];
        if (RABS(di) < RC(1e-30)) di = (di < RC(0.0)) ? RC(-1e-30) : RC(1e-30);
        r->inv[i] = RC(1.0) / di;
    }
    int kz = 0;
    if (RABS(d[1]) > RABS(d[kz])) kz = 1;
    if (RABS(d[2]) > RABS(d[kz])) kz = 2;
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    if (d[kz] < RC(0.0)) {
        int tmp = kx;
        kx = ky;
        ky = tmp;
    }
    r->kx = kx;
    r->ky = ky;
    r->kz = kz;
    r->sx = d[kx] / d[kz];
    r->sy = d[ky] / d[kz];
    r->sz = RC(1.0) / d[kz];
}

static int tri_intersect(const rayp *r, const float *v, real tmax, real *t_out)
{
    real A[3], B[3], C[3];
    for (int i = 0; i < 3; ++i) {
        A[i] = (real)v[i] - r->o[i];
        B[i] = (real)v[3 + i] - r->o[i];
        C[i] = (real)v[6 + i] - r->o[i];
    }
    real ax = A[r->kx] - r->sx * A[r->kz];
    real ay = A[r->ky] - r->sy * A[r->kz];
    real bx = B[r->kx] - r->sx * B[r->kz];
    real by = B[r->ky] - r->sy * B[r->kz];
    real cx = C[r->kx] - r->sx * C[r->kz];
    real cy = C[r->ky] - r->sy * C[r->kz];
    real U = cx * by - cy * bx;
    real V = ax * cy - ay * cx;
    real W = bx * ay - by * ax;
#ifndef ORC_F64
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)cx * (double)by - (double)cy * (double)bx);
        V = (float)((double)ax * (double)cy - (double)ay * (double)cx);
        W = (float)((double)bx * (double)ay - (double)by * (double)ax);
    }
#endif
    if ((U < RC(0.0) || V < RC(0.0) || W < RC(0.0)) && (U > RC(0.0) || V > RC(0.0) || W > RC(0.0)))
        return 0;
    real det = U + V + W;
    if (det == RC(0.0)) return 0;
    real az = r->sz * A[r->kz];
    real bz = r->sz * B[r->kz];
    real cz = r->sz * C[r->kz];
    real T = U * az + V * bz + W * cz;
    real t = T / det;
    if (!(t > RC(0.0)) || !(t < tmax)) return 0;
    *t_out = t;
    return 1;
}

/* conservative slab test: exit distance is widened so that rounding never rejects a box
 * that a triangle inside it is hit in */
static int box_enter(const rayp *r, const float *lo, const float *hi, real tlim, real *tnear)
{
    real tn = RC(0.0), tf = RC(3.0e38);
    for (int i = 0; i < 3; ++i) {
        real t0 = ((real)lo[i] - r->o[i]) * r->inv[i];
        real t1 = ((real)hi[i] - r->o[i]) * r->inv[i];
        if (t0 > t1) {
            real tmp = t0;
            t0 = t1;
            t1 = tmp;
        }
        tn = rmax(tn, t0);
        tf = rmin(tf, t1);
    }
    tf = tf * RC(1.00001);
    if (tn > tf) return 0;
    if (tn > tlim * RC(1.0001)) return 0;
    *tnear = tn;
    return 1;
}

/* ---------------------------------------------------------------------------------------
 * A plain binary BVH used only to make large scenes tractable.  The query result is the
 * brute-force one by construction (conservative box tests, no early culling beyond the best
 * distance); tests check BVH == brute force bit for bit.
 * ------------------------------------------------------------------------------------- */
typedef struct bref { float c; uint32_t tri; } bref;

static void tri_bounds(const float *v, float *lo, float *hi)
{
    for (int a = 0; a < 3; ++a) {
        float m0 = v[a], m1 = v[a];
        for (int k = 1; k < 3; ++k) {
            float x = v[3 * k + a];
            if (x < m0) m0 = x;
            if (x > m1) m1 = x;
        }
        lo[a] = m0;
        hi[a] = m1;
    }
}

static void select_kth(uint32_t *ids, const float *key, uint32_t n, uint32_t k)
{
    /* quickselect on key[ids[.]] so that ids[k] is the k-th smallest, stable by tri index */
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        float pv = key[ids[mid]];
        uint32_t pt = ids[mid];
        uint32_t i = lo, j = hi;
        while (i <= j) {
            while (key[ids[i]] < pv || (key[ids[i]] == pv && ids[i] < pt)) ++i;
            while (key[ids[j]] > pv || (key[ids[j]] == pv && ids[j] > pt)) --j;
            if (i <= j) {
                uint32_t t = ids[i];
                ids[i] = ids[j];
                ids[j] = t;
                ++i;
                if (j == 0) break;
                --j;
            }
        }
        if (k <= j) hi = j;
        else if (k >= i) lo = i;
        else break;
    }
}

static void bvh_build(scene *sc)
{
    uint32_t n = sc->nt;
    free(sc->nodes);
    free(sc->order);
    sc->nodes = NULL;
    sc->order = NULL;
    sc->nnodes = 0;
    if (n == 0) return;
    float *cen = (float *)malloc(sizeof(float) * 3 * (size_t)n);
    for (uint32_t i = 0; i < n; ++i) {
        const float *v = sc->tv + 9 * (size_t)i;
        for (int a = 0; a < 3; ++a) cen[3 * (size_t)i + a] = (v[a] + v[3 + a] + v[6 + a]) / 3.0f;
    }
    uint32_t *ids = (uint32_t *)malloc(sizeof(uint32_t) * n);
    for (uint32_t i = 0; i < n; ++i) ids[i] = i;
    uint32_t cap = 2 * n + 1;
    bnode *nodes = (bnode *)malloc(sizeof(bnode) * cap);
    float *keybuf = (float *)malloc(sizeof(float) * n);
    /* explicit work stack of (node, first, count) */
    uint32_t *ws = (uint32_t *)malloc(sizeof(uint32_t) * 3 * 128);
    uint32_t wsp = 0, nn = 1;
    ws[0] = 0; ws[1] = 0; ws[2] = n; wsp = 1;
    while (wsp > 0) {
        --wsp;
        uint32_t node = ws[3 * wsp], first = ws[3 * wsp + 1], count = ws[3 * wsp + 2];
        bnode *b = &nodes[node];
        for (int a = 0; a < 3; ++a) { b->lo[a] = 3.0e38f; b->hi[a] = -3.0e38f; }
        float clo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, chi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
        for (uint32_t i = first; i < first + count; ++i) {
            float lo[3], hi[3];
            tri_bounds(sc->tv + 9 * (size_t)ids[i], lo, hi);
            for (int a = 0; a < 3; ++a) {
                if (lo[a] < b->lo[a]) b->lo[a] = lo[a];
                if (hi[a] > b->hi[a]) b->hi[a] = hi[a];
                float c = cen[3 * (size_t)ids[i] + a];
                if (c < clo[a]) clo[a] = c;
                if (c > chi[a]) chi[a] = c;
            }
        }
        if (count <= 4) {
            b->left = first;
            b->count = count;
            continue;
        }
        int axis = 0;
        for (int a = 1; a < 3; ++a)
            if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
        for (uint32_t i = first; i < first + count; ++i) keybuf[ids[i]] = cen[3 * (size_t)ids[i] + axis];
        uint32_t half = count / 2;
        select_kth(ids + first, keybuf, count, half);
        b->left = nn;
        b->count = 0;
        uint32_t l = nn, r = nn + 1;
        nn += 2;
        ws[3 * wsp] = r; ws[3 * wsp + 1] = first + half; ws[3 * wsp + 2] = count - half; ++wsp;
        ws[3 * wsp] = l; ws[3 * wsp + 1] = first; ws[3 * wsp + 2] = half; ++wsp;
    }
    free(ws);
    free(keybuf);
    free(cen);
    sc->nodes = nodes;
    sc->nnodes = nn;
    sc->order = ids;
}

/* closest hit over static and dynamic triangles: lexicographic minimum of (t, index) */
static void closest_hit(const scene *sc, const real *o, const real *d, real tmax,
                        uint32_t *tri_out, real *t_out)
{
    rayp r;
    ray_setup(&r, o, d);
    uint32_t best = MISS;
    real bt = tmax;
    real t;
    if (sc->use_bvh && sc->nodes) {
        uint32_t stack[256];
        int sp = 0;
        real tn;
        if (box_enter(&r, sc->nodes[0].lo, sc->nodes[0].hi, bt, &tn)) stack[sp++] = 0;
        while (sp > 0) {
            const bnode *b = &sc->nodes[stack[--sp]];
            if (!box_enter(&r, b->lo, b->hi, bt, &tn)) continue;
            if (b->count) {
                for (uint32_t i = 0; i < b->count; ++i) {
                    uint32_t id = sc->order[b->left + i];
                    if (tri_intersect(&r, sc->tv + 9 * (size_t)id, tmax, &t)) {
                        if (t < bt || (t == bt && id < best)) { bt = t; best = id; }
                    }
                }
            } else {
                real t0, t1;
                int h0 = box_enter(&r, sc->nodes[b->left].lo, sc->nodes[b->left].hi, bt, &t0);
                int h1 = box_enter(&r, sc->nodes[b->left + 1].lo, sc->nodes[b->left + 1].hi, bt, &t1);
                if (h0 && h1) {
                    if (t0 <= t1) { stack[sp++] = b->left + 1; stack[sp++] = b->left; }
                    else { stack[sp++] = b->left; stack[sp++] = b->left + 1; }
                } else if (h0) stack[sp++] = b->left;
                else if (h1) stack[sp++] = b->left + 1;
            }
        }
    } else {
        for (uint32_t id = 0; id < sc->nt; ++id) {
            if (tri_intersect(&r, sc->tv + 9 * (size_t)id, tmax, &t)) {
                if (t < bt || (t == bt && id < best)) { bt = t; best = id; }
            }
        }
    }
    for (uint32_t k = 0; k < sc->nd; ++k) {
        uint32_t id = sc->nt + k;
        if (tri_intersect(&r, sc->tv + 9 * (size_t)id, tmax, &t)) {
            if (t < bt || (t == bt && id < best)) { bt = t; best = id; }
        }
    }
    *tri_out = best;
    *t_out = best == MISS ? RC(0.0) : bt;
}

/* any hit in (0, tmax) */
static int any_hit(const scene *sc, const real *o, const real *d, real tmax)
{
    rayp r;
    ray_setup(&r, o, d);
    real t;
    if (sc->use_bvh && sc->nodes) {
        uint32_t stack[256];
        int sp = 0;
        stack[sp++] = 0;
        real tn;
        while (sp > 0) {
            const bnode *b = &sc->nodes[stack[--sp]];
            if (!box_enter(&r, b->lo, b->hi, tmax, &tn)) continue;
            if (b->count) {
                for (uint32_t i = 0; i < b->count; ++i)
                    if (tri_intersect(&r, sc->tv + 9 * (size_t)sc->order[b->left + i], tmax, &t)) return 1;
            } else {
                stack[sp++] = b->left + 1;
                stack[sp++] = b->left;
            }
        }
    } else {
        for (uint32_t id = 0; id < sc->nt; ++id)
            if (tri_intersect(&r, sc->tv + 9 * (size_t)id, tmax, &t)) return 1;
    }
    for (uint32_t k = 0; k < sc->nd; ++k)
        if (tri_intersect(&r, sc->tv + 9 * (size_t)(sc->nt + k), tmax, &t)) return 1;
    return 0;
}

scene *ORC(scene_create)(const float *verts, uint32_t nv, const uint32_t *idx, uint32_t nt,
                         const uint32_t *tri_mat, const float *mats, uint32_t nm, uint32_t nd_cap,
                         int use_bvh)
{
    (void)nv;
    scene *sc = (scene *)calloc(1, sizeof(scene));
    sc->nt = nt;
    sc->nm = nm;
    sc->nd = 0;
    sc->nd_cap = nd_cap;
    size_t tot = (size_t)nt + nd_cap;
    sc->tv = (float *)malloc(sizeof(float) * 9 * (tot ? tot : 1));
    sc->tn = (real *)malloc(sizeof(real) * 3 * (tot ? tot : 1));
    sc->tmat = (uint32_t *)malloc(sizeof(uint32_t) * (tot ? tot : 1));
    sc->mats = (float *)malloc(sizeof(float) * 6 * (nm ? nm : 1));
    memcpy(sc->mats, mats, sizeof(float) * 6 * nm);
    for (uint32_t i = 0; i < nt; ++i) {
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a)
                sc->tv[9 * (size_t)i + 3 * k + a] = verts[3 * (size_t)idx[3 * (size_t)i + k] + a];
        tri_normal(sc->tv + 9 * (size_t)i, sc->tn + 3 * (size_t)i);
        sc->tmat[i] = tri_mat[i];
    }
    sc->use_bvh = use_bvh;
    if (use_bvh) bvh_build(sc);
    build_emitters(sc);
    return sc;
}

int ORC(scene_set_dynamic)(scene *sc, const float *tv, const uint32_t *mat, uint32_t nd)
{
    if (nd > sc->nd_cap) return -1;
    for (uint32_t k = 0; k < nd; ++k) {
        size_t id = (size_t)sc->nt + k;
        memcpy(sc->tv + 9 * id, tv + 9 * (size_t)k, sizeof(float) * 9);
        tri_normal(sc->tv + 9 * id, sc->tn + 3 * id);
        sc->tmat[id] = mat[k];
    }
    sc->nd = nd;
    build_emitters(sc);
    return 0;
}

void ORC(scene_destroy)(scene *sc)
{
    if (!sc) return;
    free(sc->tv); free(sc->tn); free(sc->tmat); free(sc->mats);
    free(sc->etri); free(sc->ethr); free(sc->nodes); free(sc->order);
    free(sc);
}

void ORC(scene_emitters)(const scene *sc, uint32_t *ne, uint32_t *etri, uint32_t *ethr, double *area)
{
    *ne = sc->ne;
    if (etri) memcpy(etri, sc->etri, sizeof(uint32_t) * sc->ne);
    if (ethr) memcpy(ethr, sc->ethr, sizeof(uint32_t) * sc->ne);
    *area = (double)sc->area_total;
}

void ORC(scene_normals)(const scene *sc, real *out)
{
    memcpy(out, sc->tn, sizeof(real) * 3 * ((size_t)sc->nt + sc->nd));
}

/* batch queries for tests: rays [n][3] origins and directions */
void ORC(trace_closest)(const scene *sc, const real *o, const real *d, uint32_t n, real tmax,
                        uint32_t *tri, real *t)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < (long)n; ++i) closest_hit(sc, o + 3 * i, d + 3 * i, tmax, tri + i, t + i);
}

void ORC(trace_any)(const scene *sc, const real *o, const real *d, uint32_t n, const real *tmax,
                    uint32_t *hit)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < (long)n; ++i) hit[i] = (uint32_t)any_hit(sc, o + 3 * i, d + 3 * i, tmax[i]);
}

uint32_t ORC(pick_emitter)(const scene *sc, uint32_t r) { return sc->ne ? sc->etri[pick_emitter(sc, r)] : MISS; }

/* ---------------------------------------------------------------------------------------
 * Configuration and frame (plain structs; the Python side fills them field by field)
 * ------------------------------------------------------------------------------------- */
typedef struct orc_config {
    uint32_t width, height, rays_per_probe, table_log2;
    uint32_t bounces, leak_bit, max_life, n_cap;
    uint32_t seed, frac_bits, probe_filter;
    float lod_scale;
    float cell_scale, r_max, eps_scale, t_sky;
    float sky[4];
    uint32_t temporal, upscale, ray_guiding, cache_tiles;
    uint32_t tile_min, light_grid, lgrid_dim, lgrid_k;
    uint32_t ris_m;
    float lgrid_tau;
    uint32_t restir, restir_log2, restir_cap, denoise;
    uint32_t dn_hist_max, dn_radius, pad11, pad12;
} orc_config;

typedef struct orc_frame {
    uint32_t index;
    float fov_y, tan_half, pad;
    float pos[4], fwd[4], right[4], up[4];
} orc_frame;

/* struct sizes, checked by the Python loader against its mirror */
uint32_t ORC(config_size)(void) { return (uint32_t)sizeof(orc_config); }

/* ---------------------------------------------------------------------------------------
 * G-buffer (test input; the paper rasterises it, Section 2.1.1): one primary ray through
 * every pixel centre, closest hit, face-forwarded normal, albedo, triangle index.
 * ------------------------------------------------------------------------------------- */
void ORC(render_gbuffer)(const scene *sc, const orc_frame *fr, uint32_t W, uint32_t H,
                         real *pos, real *nrm, real *alb, uint32_t *prim)
{
    real aspect = (real)W / (real)H;
#pragma omp parallel for schedule(dynamic, 16)
    for (long y = 0; y < (long)H; ++y) {
        for (uint32_t x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            real sx = (RC(2.0) * ((real)x + RC(0.5))) / (real)W - RC(1.0);
            real sy = RC(1.0) - (RC(2.0) * ((real)y + RC(0.5))) / (real)H;
            real a = (sx * (real)fr->tan_half) * aspect;
            real b = sy * (real)fr->tan_half;
            real d[3], o[3];
            for (int k = 0; k < 3; ++k) d[k] = ((real)fr->fwd[k] + a * (real)fr->right[k]) + b * (real)fr->up[k];
            real len = RSQRT(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int k = 0; k < 3; ++k) { d[k] = d[k] / len; o[k] = (real)fr->pos[k]; }
            uint32_t tri;
            real t;
            closest_hit(sc, o, d, RC(3.0e38), &tri, &t);
            prim[p] = tri;
            if (tri == MISS) {
                for (int k = 0; k < 4; ++k) pos[4 * p + k] = nrm[4 * p + k] = alb[4 * p + k] = RC(0.0);
                continue;
            }
            const real *n = sc->tn + 3 * (size_t)tri;
            real dn = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
            real s = dn > RC(0.0) ? RC(-1.0) : RC(1.0);
            const float *m = sc->mats + 6 * sc->tmat[tri];
            for (int k = 0; k < 3; ++k) {
                pos[4 * p + k] = o[k] + t * d[k];
                nrm[4 * p + k] = s * n[k];
                alb[4 * p + k] = (real)m[k];
            }
            pos[4 * p + 3] = t;
            nrm[4 * p + 3] = RC(0.0);
            alb[4 * p + 3] = RC(0.0);
        }
    }
}

/* ---------------------------------------------------------------------------------------
 * Per-frame state
 * ------------------------------------------------------------------------------------- */
typedef struct state {
    orc_config cfg;
    scene *sc;
    uint32_t W, H, TW, TH, P, R, N;
    uint32_t jx, jy;
    uint32_t nmip, mip_w[32], mip_h[32], mip_off[32], mask_total;
    uint32_t *mask;
    real *ppos, *pnrm;
    /* rays */
    int32_t *r_slot;
    real *r_t;
    uint32_t *r_tri, *r_cell;
    /* per-ray shading results (filled in the parallel phase, consumed in order) */
    real *r_sample;
    uint32_t *r_keylo, *r_keyhi, *r_valid;
    int32_t *r_bslot;
    /* world cache */
    uint32_t *fp;
    uint64_t *key;
    uint32_t *acc;         /* [N][4] fixed-point r,g,b and count */
    double *dacc;          /* [N][3] FP64 sums (reference mode) */
    real *L;               /* [N][3]; tiled: [N][64][3] level-0 cells */
    uint32_t *nhist, *life, *accessed;   /* nhist per cell ([N][64] tiled), life and accessed per slot */
    real *Lq;              /* tiled: [N][64][3] radiance returned to queries (prefiltered level) */
    uint32_t *r_tcell;     /* tiled: [P*R] cell of the hit inside its tile */
    real *r_y, *r_ny;      /* [P*R][3] hit point and face-forwarded normal */
    /* light grid (Section 2.3.2) */
    real lg_lo[3], lg_h;
    uint32_t lg_dim[3];
    uint32_t *lg_list;     /* [dim^3 cap][K] emitter indices (into etri) */
    uint32_t *lg_count;    /* [dim^3 cap] */
    /* world-space reservoirs (Section 2.3.1): two tables, the previous frame's read, this
     * frame's written; per slot the light point, contribution weight W, light, count M and
     * the normal of the vertex that stored it */
    uint32_t rs_N, rs_cur, rs_has_prev;
    uint32_t *rs_fp[2], *rs_k[2], *rs_M[2], *rs_claim;
    uint64_t *rs_key[2];
    real *rs_y[2], *rs_W[2], *rs_n[2];
    real *r_rsy, *r_rsW;   /* [P*R][3], [P*R]: each hit's final reservoir */
    /* screen-space denoiser (Section 2.4.3): accumulated irradiance and history length of the
     * previous frame, its G-buffer and camera */
    real *dn_hist, *dn_acc;  /* [H*W][4] rgb, history length */
    real *dn_ppos, *dn_pnrm; /* [H*W][4] */
    uint32_t *dn_pprim, *dn_rad;
    uint32_t dn_has_prev;
    orc_frame dn_pfr;
    uint32_t *r_rsk, *r_rsM; /* M = 0: none */
    /* probes */
    real *atlas;           /* [P][64][4] */
    real *sh;              /* [P][27] */
    double mom[NCELL][10]; /* omega, m(3), M(xx,yy,zz,xy,xz,yz) */
    uint64_t stats[16];
    real kappa;
    real cam[3];           /* camera of the last spawn (descriptor levels of detail) */
    /* temporal reuse of probes (Algorithms 1 and 3) */
    uint32_t has_prev;
    orc_frame prev_fr;     /* camera of the previous frame */
    uint32_t *prev_mask;   /* [P] level 0 of the previous frame's probe mask */
    real *prev_pos, *prev_nrm, *prev_atlas;
    real *prev_sh;         /* [P][27] the previous frame's SH (reprojected with the probes) */
    uint32_t *win;         /* [P] pixel (mask encoding) the previous probe moved to, or SENTINEL */
    uint32_t *hist;        /* [P] previous tile of that probe, or SENTINEL */
    uint32_t *traced;      /* [P] the tile's probe traces rays this frame */
    uint32_t sjx, sjy;     /* this frame's jitter inside the spawn tile of 8 upscale pixels */
    real *recon;           /* [P][64][4] reconstructed history radiance, distance; w < 0: empty */
    uint32_t *cdf;         /* [P][64] inclusive sums of the guiding weights; last 0: unguided */
    int guided;            /* this frame's probes have a reconstruction (ray guiding) */
} state;

enum { ST_RAYS, ST_HITS, ST_INSERTS, ST_OVERFLOW, ST_NONFINITE, ST_WRAPS, ST_SHADOW, ST_OCCLUDED,
       ST_EVICT, ST_LIVE, ST_RELAXED, ST_NOPROBE, ST_BOUNCE };

/* ---------------------------------------------------------------------------------------
 * Hemi-octahedral cell moments (float64 quadrature): for each of the 64 cells of the
 * 8x8 atlas (Section 2.1: octahedral mapping of the oriented hemisphere), the solid angle,
 * the first moment and the second moment of the direction.  Each cell is split into two
 * triangles along the diagonal on which the map has a kink, and each triangle is integrated
 * with a collapsed Gauss-Legendre product rule.
 * ------------------------------------------------------------------------------------- */
static const double GL16_X[16] = {
    -0.9894009349916499, -0.9445750230732326, -0.8656312023878318, -0.7554044083550030,
    -0.6178762444026438, -0.4580167776572274, -0.2816035507792589, -0.0950125098376374,
    0.0950125098376374, 0.2816035507792589, 0.4580167776572274, 0.6178762444026438,
    0.7554044083550030, 0.8656312023878318, 0.9445750230732326, 0.9894009349916499};
static const double GL16_W[16] = {
    0.0271524594117541, 0.0622535239386479, 0.0951585116824928, 0.1246289712555339,
    0.1495959888165767, 0.1691565193950025, 0.1826034150449236, 0.1894506104550685,
    0.1894506104550685, 0.1826034150449236, 0.1691565193950025, 0.1495959888165767,
    0.1246289712555339, 0.0951585116824928, 0.0622535239386479, 0.0271524594117541};

static void integrate_tri_uv(const double *p0, const double *p1, const double *p2, int sub, double *acc)
{
    /* subdivide the triangle into sub*sub similar triangles is awkward; instead split the
     * square [0,1]^2 of the collapsed map into sub x sub blocks */
    double e1u = p1[0] - p0[0], e1v = p1[1] - p0[1];
    double e2u = p2[0] - p1[0], e2v = p2[1] - p1[1];
    double jac = fabs(e1u * e2v - e1v * e2u);
    for (int bs = 0; bs < sub; ++bs)
        for (int bt = 0; bt < sub; ++bt)
            for (int i = 0; i < 16; ++i)
                for (int j = 0; j < 16; ++j) {
                    double s = (bs + 0.5 + 0.5 * GL16_X[i]) / sub;
                    double t = (bt + 0.5 + 0.5 * GL16_X[j]) / sub;
                    double w = GL16_W[i] * GL16_W[j] * 0.25 / ((double)sub * sub) * s * jac;
                    double u = p0[0] + s * e1u + s * t * e2u;
                    double v = p0[1] + s * e1v + s * t * e2v;
                    double a = 0.5 * (u + v), b = 0.5 * (u - v);
                    double z = 1.0 - fabs(a) - fabs(b);
                    double r2 = a * a + b * b + z * z;
                    double r = sqrt(r2);
                    double dw = w * 0.5 / (r2 * r);   /* d(omega) = du dv / (2 r^3) */
                    double wx = a / r, wy = b / r, wz = z / r;
                    acc[0] += dw;
                    acc[1] += dw * wx; acc[2] += dw * wy; acc[3] += dw * wz;
                    acc[4] += dw * wx * wx; acc[5] += dw * wy * wy; acc[6] += dw * wz * wz;
                    acc[7] += dw * wx * wy; acc[8] += dw * wx * wz; acc[9] += dw * wy * wz;
                }
}

void ORC(cell_moments)(double *out /* [64][10] */)
{
    for (int iy = 0; iy < 8; ++iy)
        for (int ix = 0; ix < 8; ++ix) {
            double u0 = -1.0 + ix * 0.25, u1 = u0 + 0.25, v0 = -1.0 + iy * 0.25, v1 = v0 + 0.25;
            double acc[10] = {0};
            double c00[2] = {u0, v0}, c10[2] = {u1, v0}, c01[2] = {u0, v1}, c11[2] = {u1, v1};
            if (ix + iy == 7) {
                /* kink along u = -v: split along the anti-diagonal c10-c01 */
                integrate_tri_uv(c00, c10, c01, 4, acc);
                integrate_tri_uv(c11, c01, c10, 4, acc);
            } else {
                /* split along the main diagonal c00-c11 (the kink u = v when ix == iy) */
                integrate_tri_uv(c00, c10, c11, 4, acc);
                integrate_tri_uv(c00, c11, c01, 4, acc);
            }
            for (int k = 0; k < 10; ++k) out[(iy * 8 + ix) * 10 + k] = acc[k];
        }
}

/* ---------------------------------------------------------------------------------------
 * Branchless orthonormal basis (Duff et al., JCGT 2017) around the probe normal
 * ------------------------------------------------------------------------------------- */
static void onb(const real *n, real *t, real *b)
{
    real sign = n[2] >= RC(0.0) ? RC(1.0) : RC(-1.0);
    real a = RC(-1.0) / (sign + n[2]);
    real bb = (n[0] * n[1]) * a;
    t[0] = RC(1.0) + ((sign * n[0]) * n[0]) * a;
    t[1] = sign * bb;
    t[2] = -(sign * n[0]);
    b[0] = bb;
    b[1] = sign + (n[1] * n[1]) * a;
    b[2] = -n[1];
}

/* cosine-distributed direction about n from two uniform numbers; also the hemi-oct cell of
 * the local direction (8x8 atlas, Section 2.1) */
static void cosine_dir(const real *n, real u0, real u1, real *d, uint32_t *cell)
{
    real c, s;
    sincos_2pi(u1, &c, &s);
    real r = RSQRT(u0);
    real lx = r * c, ly = r * s;
    real lz = RSQRT(rmax(RC(0.0), RC(1.0) - u0));
    real t[3], b[3];
    onb(n, t, b);
    for (int k = 0; k < 3; ++k) d[k] = (lx * t[k] + ly * b[k]) + lz * n[k];
    if (cell) {
        real sum = (RABS(lx) + RABS(ly)) + lz;
        real a = lx / sum, bb = ly / sum;
        real uu = a + bb, vv = a - bb;
        int ix = (int)RFLOOR(RC(4.0) * (uu + RC(1.0)));
        int iy = (int)RFLOOR(RC(4.0) * (vv + RC(1.0)));
        ix = ix < 0 ? 0 : (ix > 7 ? 7 : ix);
        iy = iy < 0 ? 0 : (iy > 7 ? 7 : iy);
        *cell = (uint32_t)(8 * iy + ix);
    }
}

void ORC(cosine_dirs)(const real *n, const real *u0, const real *u1, uint32_t cnt, real *d, uint32_t *cell)
{
    for (uint32_t i = 0; i < cnt; ++i) cosine_dir(n + 3 * i, u0[i], u1[i], d + 3 * i, cell + i);
}

static real offset_eps(const orc_config *c, const real *p)
{
    real m = rmax(rmax(RABS(p[0]), RABS(p[1])), RABS(p[2]));
    return (real)c->eps_scale * (RC(1.0) + m);
}

/* ---------------------------------------------------------------------------------------
 * World-cache descriptor (Section 2.2.1 and 2.2.2).  READING: the descriptor is the
 * quantised hit position floor(y * S) (S = 1 / cell size), a 6-way class of the
 * face-forwarded surface normal, and the light-leak bit (ray length < cell size); LOD = 0.
 * ------------------------------------------------------------------------------------- */
/* READING (Section 2.2.1, levels of detail of the world cache): the position quantisation is
 * coarsened with the distance d from the camera so that a cell keeps roughly the size of
 * Algorithm 6's adaptive cell, lod_scale * d: the cell size is the base size times 2^lod, the
 * smallest power of two (lod <= 7) with 2^lod >= lod_scale * d * S; lod enters the descriptor
 * and the leak test uses that level's cell size.  lod_scale = 0 keeps a single level. */
static uint32_t cell_lod(const orc_config *c, const real *cam, const real *y)
{
    if (!(c->lod_scale > 0.0f)) return 0;
    real dx = y[0] - cam[0], dy = y[1] - cam[1], dz = y[2] - cam[2];
    real d = RSQRT((dx * dx + dy * dy) + dz * dz);
    real x = ((real)c->lod_scale * d) * (real)c->cell_scale;
    uint32_t lod = 0;
    real p = RC(1.0);
    while (p < x && lod < 7) { p = p * RC(2.0); ++lod; }
    return lod;
}

/* floor(v / 8) for signed v */
static int32_t floor_div8(int32_t v) { return v >= 0 ? v / 8 : -((-v + 7) / 8); }

/* Two-level world cache (Section 2.2.3, prefiltering): with cache_tiles, the descriptor names
 * a tile of 8x8x8 cells (quantised position divided by 8, floor), and the hit's cell inside
 * the tile is 2D: the position's remainders modulo 8 along the two axes other than the main
 * axis of the normal (the axis of the normal class), u the lower-numbered one:
 * cell = 8 (v mod 8) + (u mod 8). */
static uint64_t cell_key_cell(const orc_config *c, const real *cam, const real *y, const real *n, real t,
                              int with_leak, uint32_t *tcell)
{
    uint32_t lod = cell_lod(c, cam, y);
    real S = (real)c->cell_scale * (RC(1.0) / (real)(1u << lod));
    int32_t qx = (int32_t)RFLOOR(y[0] * S);
    int32_t qy = (int32_t)RFLOOR(y[1] * S);
    int32_t qz = (int32_t)RFLOOR(y[2] * S);
    int axis = 0;
    real best = RABS(n[0]);
    if (RABS(n[1]) > best) { axis = 1; best = RABS(n[1]); }
    if (RABS(n[2]) > best) { axis = 2; }
    if (tcell) *tcell = 0;
    if (c->cache_tiles) {
        int32_t q[3] = {qx, qy, qz};
        int32_t u = q[axis == 0 ? 1 : 0], v = q[axis == 2 ? 1 : 2];
        if (tcell) *tcell = 8u * (uint32_t)(v - 8 * floor_div8(v)) + (uint32_t)(u - 8 * floor_div8(u));
        qx = floor_div8(qx);
        qy = floor_div8(qy);
        qz = floor_div8(qz);
    }
    uint64_t cls = (uint64_t)(2 * axis + (n[axis] < RC(0.0) ? 1 : 0));
    uint64_t leak = (with_leak && c->leak_bit && t * S < RC(1.0)) ? 1u : 0u;
    return ((uint64_t)(uint32_t)qx & 0x3FFFFu) | (((uint64_t)(uint32_t)qy & 0x3FFFFu) << 18) |
           (((uint64_t)(uint32_t)qz & 0x3FFFFu) << 36) | (cls << 54) | (leak << 57) | ((uint64_t)lod << 58);
}

static uint64_t cell_key(const orc_config *c, const real *cam, const real *y, const real *n, real t, int with_leak)
{
    return cell_key_cell(c, cam, y, n, t, with_leak, NULL);
}

/* world-cache entry of a hit: slot, or with tiles slot * 64 + cell inside the tile */
static int32_t cache_entry(const state *st, int32_t slot, uint32_t tcell)
{
    if (slot < 0) return slot;
    return st->cfg.cache_tiles ? slot * NCELL + (int32_t)tcell : slot;
}

/* the radiance readers see per entry: the cell's own, or with tiles its prefiltered level */
static const real *cache_L(const state *st) { return st->cfg.cache_tiles ? st->Lq : st->L; }

static uint32_t key_bucket(uint64_t key, uint32_t nbuckets)
{
    uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
    return pcg_hash(lo + pcg_hash(hi)) & (nbuckets - 1u);
}

static uint32_t key_fingerprint(uint64_t key)
{
    uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
    uint32_t h = xxh32_hash(lo + xxh32_hash(hi));
    return h == 0u ? 1u : h;
}

void ORC(keys)(const orc_config *c, const real *cam, const real *y, const real *n, const real *t, uint32_t cnt,
               uint64_t *key, uint32_t *bucket, uint32_t *fp)
{
    uint32_t nb = (1u << c->table_log2) / BUCKET;
    for (uint32_t i = 0; i < cnt; ++i) {
        key[i] = cell_key(c, cam, y + 3 * i, n + 3 * i, t[i], 1);
        bucket[i] = key_bucket(key[i], nb);
        fp[i] = key_fingerprint(key[i]);
    }
}

/* find an existing cell (lookup only): slot or -1 */
static int32_t table_find(const state *st, uint64_t key)
{
    uint32_t nb = st->N / BUCKET;
    uint32_t b = key_bucket(key, nb), f = key_fingerprint(key);
    for (uint32_t s = 0; s < BUCKET; ++s)
        if (st->fp[b * BUCKET + s] == f) return (int32_t)(b * BUCKET + s);
    return -1;
}

/* find-or-insert with linear probing inside the bucket (Section 2.2.1): the fingerprint is
 * searched first, otherwise the first empty slot is claimed; a full bucket drops the sample */
static int32_t table_insert(state *st, uint64_t key)
{
    uint32_t nb = st->N / BUCKET;
    uint32_t b = key_bucket(key, nb), f = key_fingerprint(key);
    for (uint32_t s = 0; s < BUCKET; ++s)
        if (st->fp[b * BUCKET + s] == f) return (int32_t)(b * BUCKET + s);
    for (uint32_t s = 0; s < BUCKET; ++s) {
        uint32_t slot = b * BUCKET + s;
        if (st->fp[slot] == 0u) {
            st->fp[slot] = f;
            st->key[slot] = key;
            st->stats[ST_INSERTS]++;
            return (int32_t)slot;
        }
    }
    st->stats[ST_OVERFLOW]++;
    return -1;
}

state *ORC(create)(const orc_config *cfg, scene *sc)
{
    state *st = (state *)calloc(1, sizeof(state));
    st->cfg = *cfg;
    st->sc = sc;
    st->W = cfg->width;
    st->H = cfg->height;
    st->TW = (cfg->width + 7) / 8;
    st->TH = (cfg->height + 7) / 8;
    st->P = st->TW * st->TH;
    st->R = cfg->rays_per_probe;
    st->N = 1u << cfg->table_log2;
    uint32_t w = st->TW, h = st->TH, off = 0, k = 0;
    for (;;) {
        st->mip_w[k] = w;
        st->mip_h[k] = h;
        st->mip_off[k] = off;
        off += w * h;
        ++k;
        if (w == 1 && h == 1) break;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    st->nmip = k;
    st->mask_total = off;
    size_t P = st->P, PR = (size_t)st->P * st->R, N = st->N;
    st->mask = (uint32_t *)calloc(off, sizeof(uint32_t));
    st->ppos = (real *)calloc(4 * P, sizeof(real));
    st->pnrm = (real *)calloc(4 * P, sizeof(real));
    st->r_slot = (int32_t *)calloc(PR, sizeof(int32_t));
    st->r_t = (real *)calloc(PR, sizeof(real));
    st->r_tri = (uint32_t *)calloc(PR, sizeof(uint32_t));
    st->r_cell = (uint32_t *)calloc(PR, sizeof(uint32_t));
    st->r_sample = (real *)calloc(3 * PR, sizeof(real));
    st->r_keylo = (uint32_t *)calloc(PR, sizeof(uint32_t));
    st->r_keyhi = (uint32_t *)calloc(PR, sizeof(uint32_t));
    st->r_valid = (uint32_t *)calloc(PR, sizeof(uint32_t));
    st->r_bslot = (int32_t *)calloc(PR, sizeof(int32_t));
    st->fp = (uint32_t *)calloc(N, sizeof(uint32_t));
    st->key = (uint64_t *)calloc(N, sizeof(uint64_t));
    size_t G = cfg->cache_tiles ? NCELL : 1;   /* cells per slot */
    st->acc = (uint32_t *)calloc(4 * N * G, sizeof(uint32_t));
    st->dacc = (double *)calloc(3 * N * G, sizeof(double));
    st->L = (real *)calloc(3 * N * G, sizeof(real));
    st->nhist = (uint32_t *)calloc(N * G, sizeof(uint32_t));
    st->Lq = (real *)calloc(cfg->cache_tiles ? 3 * N * G : 1, sizeof(real));
    st->r_tcell = (uint32_t *)calloc(PR, sizeof(uint32_t));
    st->r_y = (real *)calloc(3 * PR, sizeof(real));
    st->r_ny = (real *)calloc(3 * PR, sizeof(real));
    if (cfg->denoise) {
        size_t HW = (size_t)cfg->width * cfg->height;
        st->dn_hist = (real *)calloc(4 * HW, sizeof(real));
        st->dn_acc = (real *)calloc(4 * HW, sizeof(real));
        st->dn_ppos = (real *)calloc(4 * HW, sizeof(real));
        st->dn_pnrm = (real *)calloc(4 * HW, sizeof(real));
        st->dn_pprim = (uint32_t *)calloc(HW, sizeof(uint32_t));
        st->dn_rad = (uint32_t *)calloc(HW, sizeof(uint32_t));
    }
    if (cfg->restir) {
        st->rs_N = 1u << cfg->restir_log2;
        for (int t = 0; t < 2; ++t) {
            st->rs_fp[t] = (uint32_t *)calloc(st->rs_N, sizeof(uint32_t));
            st->rs_k[t] = (uint32_t *)calloc(st->rs_N, sizeof(uint32_t));
            st->rs_M[t] = (uint32_t *)calloc(st->rs_N, sizeof(uint32_t));
            st->rs_key[t] = (uint64_t *)calloc(st->rs_N, sizeof(uint64_t));
            st->rs_y[t] = (real *)calloc(3 * (size_t)st->rs_N, sizeof(real));
            st->rs_W[t] = (real *)calloc(st->rs_N, sizeof(real));
            st->rs_n[t] = (real *)calloc(3 * (size_t)st->rs_N, sizeof(real));
        }
        st->rs_claim = (uint32_t *)calloc(st->rs_N, sizeof(uint32_t));
        st->r_rsy = (real *)calloc(3 * PR, sizeof(real));
        st->r_rsW = (real *)calloc(PR, sizeof(real));
        st->r_rsk = (uint32_t *)calloc(PR, sizeof(uint32_t));
        st->r_rsM = (uint32_t *)calloc(PR, sizeof(uint32_t));
    }
    if (cfg->light_grid) {
        size_t ncell = (size_t)cfg->lgrid_dim * cfg->lgrid_dim * cfg->lgrid_dim;
        st->lg_list = (uint32_t *)calloc(ncell * (cfg->lgrid_k ? cfg->lgrid_k : 1), sizeof(uint32_t));
        st->lg_count = (uint32_t *)calloc(ncell, sizeof(uint32_t));
    }
    st->life = (uint32_t *)calloc(N, sizeof(uint32_t));
    st->accessed = (uint32_t *)calloc(N, sizeof(uint32_t));
    st->atlas = (real *)calloc(P * NCELL * 4, sizeof(real));
    st->sh = (real *)calloc(P * 27, sizeof(real));
    st->prev_mask = (uint32_t *)calloc(P, sizeof(uint32_t));
    st->prev_pos = (real *)calloc(4 * P, sizeof(real));
    st->prev_nrm = (real *)calloc(4 * P, sizeof(real));
    st->prev_atlas = (real *)calloc(P * NCELL * 4, sizeof(real));
    st->prev_sh = (real *)calloc(P * 27, sizeof(real));
    st->win = (uint32_t *)calloc(P, sizeof(uint32_t));
    st->hist = (uint32_t *)calloc(P, sizeof(uint32_t));
    st->traced = (uint32_t *)calloc(P, sizeof(uint32_t));
    st->recon = (real *)calloc(P * NCELL * 4, sizeof(real));
    st->cdf = (uint32_t *)calloc(P * NCELL, sizeof(uint32_t));
    for (size_t i = 0; i < P; ++i) st->win[i] = st->hist[i] = SENTINEL;
    ORC(cell_moments)(&st->mom[0][0]);
    return st;
}

void ORC(destroy)(state *st)
{
    if (!st) return;
    free(st->mask); free(st->ppos); free(st->pnrm);
    free(st->r_slot); free(st->r_t); free(st->r_tri); free(st->r_cell);
    free(st->r_sample); free(st->r_keylo); free(st->r_keyhi); free(st->r_valid); free(st->r_bslot);
    free(st->fp); free(st->key); free(st->acc); free(st->dacc); free(st->L);
    free(st->nhist); free(st->life); free(st->accessed); free(st->atlas); free(st->sh);
    free(st->Lq); free(st->r_tcell); free(st->r_y); free(st->r_ny); free(st->lg_list); free(st->lg_count);
    for (int t = 0; t < 2; ++t) {
        free(st->rs_fp[t]); free(st->rs_k[t]); free(st->rs_M[t]); free(st->rs_key[t]); free(st->rs_y[t]);
        free(st->rs_W[t]); free(st->rs_n[t]);
    }
    free(st->rs_claim); free(st->r_rsy); free(st->r_rsW); free(st->r_rsk); free(st->r_rsM);
    free(st->dn_hist); free(st->dn_acc); free(st->dn_ppos); free(st->dn_pnrm); free(st->dn_pprim); free(st->dn_rad);
    free(st->prev_mask); free(st->prev_pos); free(st->prev_nrm); free(st->prev_atlas); free(st->prev_sh); free(st->win);
    free(st->hist); free(st->traced); free(st->recon); free(st->cdf);
    free(st);
}

/* Algorithm 6: distance scale tan(fov_y * proj_size * max(1/H, H/W^2)), proj_size = 8,
 * computed in float64 on the host and rounded once */
float ORC(distance_scale)(float fov_y, uint32_t W, uint32_t H)
{
    double a = 1.0 / (double)H, b = (double)H / ((double)W * (double)W);
    return (float)tan((double)fov_y * 8.0 * (a > b ? a : b));
}

/* ---------------------------------------------------------------------------------------
 * Temporal reuse of screen probes: probe reprojection (Section 2.1.1, Algorithm 1).
 * Every pixel p of a tile that is not sky looks up, in the previous frame, the pixel q it was
 * seen at and the probe of q's tile; if that probe lies within the cell size (Algorithm 6) of
 * p's tangent plane and its normal is within the 0.95 cosine of p's, p bids the half-precision
 * distance to it, packed above its lane index; the smallest bid wins, and the tile's probe
 * moves to that pixel with the previous probe's radiance as history.
 * READING: motion vectors are the reprojection of the pixel's world position with the
 * previous frame's camera (static geometry; the moving light is not geometry of the G-buffer);
 * q is the pixel whose centre region holds the projection; lane = 8 (y % 8) + (x % 8); with
 * temporal reuse on, a tile with a winner places its probe at the winning pixel instead of
 * the frame's Halton pixel; with upscale 1x1 every tile that holds a probe traces every frame.
 * ------------------------------------------------------------------------------------- */
/* float -> IEEE binary16 bits, round to nearest even (for x >= 0 or NaN) */
static uint32_t half_bits(float x)
{
    uint32_t f;
    memcpy(&f, &x, 4);
    f &= 0x7FFFFFFFu;
    if (f >= 0x7F800000u) return f > 0x7F800000u ? 0x7E00u : 0x7C00u;
    int32_t e = (int32_t)(f >> 23) - 127 + 15;
    if (e >= 31) return 0x7C00u;
    if (e <= 0) {
        if (e < -10) return 0u;
        uint32_t m = (f & 0x7FFFFFu) | 0x800000u;
        uint32_t sh = (uint32_t)(14 - e);
        uint32_t h = m >> sh, rem = m & ((1u << sh) - 1u), hf = 1u << (sh - 1u);
        if (rem > hf || (rem == hf && (h & 1u))) ++h;
        return h;
    }
    uint32_t h = ((uint32_t)e << 10) | ((f & 0x7FFFFFu) >> 13);
    uint32_t rem = f & 0x1FFFu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;
    return h;
}

uint32_t ORC(half_bits)(float x) { return half_bits(x); }

/* pixel of the previous frame in which world point X was seen; 0 if behind or off screen */
static int project_prev(const state *st, const real *X, int32_t *qx, int32_t *qy)
{
    const orc_frame *pf = &st->prev_fr;
    real v[3] = {X[0] - (real)pf->pos[0], X[1] - (real)pf->pos[1], X[2] - (real)pf->pos[2]};
    real z = (v[0] * (real)pf->fwd[0] + v[1] * (real)pf->fwd[1]) + v[2] * (real)pf->fwd[2];
    if (!(z > RC(0.0))) return 0;
    real a = ((v[0] * (real)pf->right[0] + v[1] * (real)pf->right[1]) + v[2] * (real)pf->right[2]) / z;
    real b = ((v[0] * (real)pf->up[0] + v[1] * (real)pf->up[1]) + v[2] * (real)pf->up[2]) / z;
    real aspect = (real)st->W / (real)st->H;
    real sx = a / ((real)pf->tan_half * aspect), sy = b / (real)pf->tan_half;
    real fx = ((sx + RC(1.0)) * (real)st->W) * RC(0.5), fy = ((RC(1.0) - sy) * (real)st->H) * RC(0.5);
    if (!(fx >= RC(0.0) && fx < (real)st->W && fy >= RC(0.0) && fy < (real)st->H)) return 0;
    *qx = (int32_t)fx;
    *qy = (int32_t)fy;
    return 1;
}

static void reproject(state *st, const orc_frame *fr, const real *gpos, const real *gnrm, const uint32_t *gprim)
{
    real kappa = (real)ORC(distance_scale)(fr->fov_y, st->W, st->H);
    const uint32_t init = (half_bits(65504.0f) << 16) | 0xFFFFu;
#pragma omp parallel for schedule(static)
    for (long t = 0; t < (long)st->P; ++t) {
        uint32_t tx = (uint32_t)t % st->TW, ty = (uint32_t)t / st->TW;
        uint32_t best = init, best_q = SENTINEL;
        for (uint32_t lane = 0; lane < 64; ++lane) {
            uint32_t x = 8 * tx + (lane & 7u), y = 8 * ty + (lane >> 3);
            if (x >= st->W || y >= st->H) continue;
            size_t pix = (size_t)y * st->W + x;
            if (gprim[pix] == MISS) continue;
            const real *X = gpos + 4 * pix, *n = gnrm + 4 * pix;
            int32_t qx, qy;
            if (!project_prev(st, X, &qx, &qy)) continue;
            uint32_t q = (uint32_t)(qy >> 3) * st->TW + (uint32_t)(qx >> 3);
            if (st->prev_mask[q] == SENTINEL) continue;
            const real *wq = st->prev_pos + 4 * (size_t)q, *nq = st->prev_nrm + 4 * (size_t)q;
            real dx = X[0] - (real)fr->pos[0], dy = X[1] - (real)fr->pos[1], dz = X[2] - (real)fr->pos[2];
            real cs = kappa * RSQRT((dx * dx + dy * dy) + dz * dz);
            real pd = RABS(((wq[0] - X[0]) * n[0] + (wq[1] - X[1]) * n[1]) + (wq[2] - X[2]) * n[2]);
            real nc = (nq[0] * n[0] + nq[1] * n[1]) + nq[2] * n[2];
            if (pd < cs && nc > RC(0.95)) {
                real ex = wq[0] - X[0], ey = wq[1] - X[1], ez = wq[2] - X[2];
                real dist = RSQRT((ex * ex + ey * ey) + ez * ez);
                uint32_t score = (half_bits((float)dist) << 16) | lane;
                if (score < best) {
                    best = score;
                    best_q = q;
                }
            }
        }
        if (best_q != SENTINEL) {
            uint32_t lane = best & 0xFFFFu;
            st->win[t] = ((8 * ty + (lane >> 3)) << 16) | (8 * tx + (lane & 7u));
            st->hist[t] = best_q;
        } else {
            st->win[t] = st->hist[t] = SENTINEL;
        }
    }
}

/* ---------------------------------------------------------------------------------------
 * Spawn (Section 2.1.1) and probe mask with its MIP chain (Section 2.1.5).
 * READING: a tile whose jittered pixel is off screen or sky gets the sentinel; the mask packs
 * (y << 16) | x; each MIP entry keeps the first valid probe of its 2x2 children in raster order.
 * ------------------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------------------
 * Temporal upscaling and adaptive sampling (Section 2.1.1 spawn tiles; Section 2.1.2,
 * Algorithm 2).  With upscale u, a spawn tile is u x u probe tiles; the frame's Halton jitter
 * in [0, 8u)^2 picks one pixel per spawn tile, and only the probe tile that holds it (if the
 * pixel is not sky) is spawned and traces.  A tile whose previous probe reprojected keeps it:
 * it traces if spawned (an "override" tile), else it keeps its history without rays.  A tile
 * neither spawned nor reprojected is empty; each empty tile picks a random override tile and
 * takes its rays, placing a new probe at its own pixel of the jitter.
 * READING: an empty tile can take rays only if that pixel (jitter mod 8 inside the tile) is
 * not sky; the override tiles are listed in tile order and the pick is a counter-based
 * random number (seed, frame, tile, dimension 7) modulo their count; where several empty
 * tiles pick the same override tile (the paper's atomic exchange leaves this to timing), the
 * lowest-numbered one takes it and the others stay empty.  With u = 1 every tile that holds
 * a probe traces, as without temporal upscaling.
 * ------------------------------------------------------------------------------------- */
static uint32_t in_tile_pixel(const state *st, uint32_t tx, uint32_t ty, const uint32_t *gprim)
{
    uint32_t px = 8 * tx + st->sjx % 8u, py = 8 * ty + st->sjy % 8u;
    if (px < st->W && py < st->H && gprim[(size_t)py * st->W + px] != MISS) return (py << 16) | px;
    return SENTINEL;
}

static void place_probes(state *st, const orc_frame *fr, const uint32_t *gprim, uint32_t *place)
{
    const uint32_t u = st->cfg.upscale > 1 ? st->cfg.upscale : 1u;
    uint32_t *over = (uint32_t *)malloc(sizeof(uint32_t) * st->P);
    uint32_t *assigned = (uint32_t *)malloc(sizeof(uint32_t) * st->P);
    uint32_t nover = 0;
    for (uint32_t t = 0; t < st->P; ++t) {
        uint32_t tx = t % st->TW, ty = t / st->TW;
        uint32_t spx = 8u * u * (tx / u) + st->sjx, spy = 8u * u * (ty / u) + st->sjy;
        int spawned = spx / 8u == tx && spy / 8u == ty && spx < st->W && spy < st->H &&
                      gprim[(size_t)spy * st->W + spx] != MISS;
        int reproj = st->cfg.temporal && st->win[t] != SENTINEL;
        place[t] = reproj ? st->win[t] : (spawned ? ((spy << 16) | spx) : SENTINEL);
        st->traced[t] = u == 1 ? place[t] != SENTINEL : (uint32_t)spawned;
        assigned[t] = SENTINEL;
        if (u > 1 && spawned && reproj) over[nover++] = t;
    }
    if (u > 1 && nover > 0) {
        for (uint32_t e = 0; e < st->P; ++e) {
            int reproj = st->cfg.temporal && st->win[e] != SENTINEL;
            if (place[e] != SENTINEL || reproj) continue;
            if (in_tile_pixel(st, e % st->TW, e / st->TW, gprim) == SENTINEL) continue;
            uint32_t o = over[rng_u32(st->cfg.seed, fr->index, e, 7u) % nover];
            if (e < assigned[o]) assigned[o] = e;
        }
        for (uint32_t k = 0; k < nover; ++k) {
            uint32_t o = over[k], e = assigned[o];
            if (e == SENTINEL) continue;
            st->traced[o] = 0;
            st->traced[e] = 1;
            place[e] = in_tile_pixel(st, e % st->TW, e / st->TW, gprim);
        }
    }
    free(over);
    free(assigned);
}

/* ---------------------------------------------------------------------------------------
 * Ray guiding (Section 2.1.2): parallax-corrected reconstruction of each new probe's
 * hemisphere from the previous frame's probes, and the sampling distribution built from it.
 * For a new probe p: the previous probes in the 3x3 tiles around the previous-frame tile that
 * holds p's projection are taken if they pass the cell-size tests of the reprojection (plane
 * distance below p's cell size, normal cosine above 0.95).  Each of their 64 cells gives the
 * point its radiance came from (probe position + travelled distance along the cell's centre
 * direction); seen from p that point falls in one of p's cells, which receives the radiance
 * and the new distance.  Cells receiving nothing are empty.
 * The weights are the reconstruction's luminance (channel mean), quantised as
 * floor(2^20 lum / max lum); a ray picks a cell with probability proportional to its weight
 * (integer inverse CDF of a 32-bit counter hash, dimension 8) and a uniform point inside
 * that cell of the 8x8 hemi-octahedral square (dimensions 0 and 1).
 * READING: previous-frame neighbourhood around p's own projection (not its history tile); the
 * same plane and normal tests as Algorithm 1; cells accumulated in (tile, cell) order; a
 * probe with no reconstruction or zero total weight samples the cosine distribution as
 * without guiding; a ray keeps the picked cell as its atlas cell.
 * ------------------------------------------------------------------------------------- */
static void cell_direction(int cell, const real *n, real *d);

static uint32_t local_cell(real lx, real ly, real lz)
{
    real sum = (RABS(lx) + RABS(ly)) + lz;
    real a = lx / sum, bb = ly / sum;
    real uu = a + bb, vv = a - bb;
    int ix = (int)RFLOOR(RC(4.0) * (uu + RC(1.0)));
    int iy = (int)RFLOOR(RC(4.0) * (vv + RC(1.0)));
    ix = ix < 0 ? 0 : (ix > 7 ? 7 : ix);
    iy = iy < 0 ? 0 : (iy > 7 ? 7 : iy);
    return (uint32_t)(8 * iy + ix);
}

/* the reconstruction of one probe (position pp, unit normal pn, cell size cs) from nq
 * candidate previous probes; recon [64][4] (w = -1 where empty) and cdf [64] */
static void recon_probe(const real *pp, const real *pn, real cs, uint32_t nq, const real *const *qpos,
                        const real *const *qnrm, const real *const *qatlas, real *rc, uint32_t *cdf)
{
    const real third = RC(1.0) / RC(3.0);
    real sum[NCELL][4];
    uint32_t cnt[NCELL];
    memset(cnt, 0, sizeof(cnt));
    for (int i = 0; i < NCELL; ++i) sum[i][0] = sum[i][1] = sum[i][2] = sum[i][3] = RC(0.0);
    real t[3], b[3];
    onb(pn, t, b);
    for (uint32_t j = 0; j < nq; ++j) {
        const real *wq = qpos[j], *nq3 = qnrm[j], *qa = qatlas[j];
        real pd = RABS(((wq[0] - pp[0]) * pn[0] + (wq[1] - pp[1]) * pn[1]) + (wq[2] - pp[2]) * pn[2]);
        real nc = (nq3[0] * pn[0] + nq3[1] * pn[1]) + nq3[2] * pn[2];
        if (!(pd < cs && nc > RC(0.95))) continue;
        for (int c = 0; c < NCELL; ++c) {
            real d[3];
            cell_direction(c, nq3, d);
            real al = qa[4 * c + 3];
            real v[3];
            for (int k = 0; k < 3; ++k) v[k] = (wq[k] + al * d[k]) - pp[k];
            real lz = (v[0] * pn[0] + v[1] * pn[1]) + v[2] * pn[2];
            if (!(lz > RC(0.0))) continue;
            real lx = (v[0] * t[0] + v[1] * t[1]) + v[2] * t[2];
            real ly = (v[0] * b[0] + v[1] * b[1]) + v[2] * b[2];
            uint32_t k = local_cell(lx, ly, lz);
            real dist = RSQRT((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
            for (int i = 0; i < 3; ++i) sum[k][i] = sum[k][i] + qa[4 * c + i];
            sum[k][3] = sum[k][3] + dist;
            cnt[k]++;
        }
    }
    real maxl = RC(0.0);
    real lum[NCELL];
    for (int i = 0; i < NCELL; ++i) {
        if (!cnt[i]) {
            rc[4 * i] = rc[4 * i + 1] = rc[4 * i + 2] = RC(0.0);
            rc[4 * i + 3] = RC(-1.0);
            lum[i] = RC(0.0);
            continue;
        }
        real fc = (real)cnt[i];
        for (int k = 0; k < 4; ++k) rc[4 * i + k] = sum[i][k] / fc;
        lum[i] = (rc[4 * i] * third + rc[4 * i + 1] * third) + rc[4 * i + 2] * third;
        maxl = rmax(maxl, lum[i]);
    }
    uint32_t acc = 0;
    for (int i = 0; i < NCELL; ++i) {
        uint32_t w = 0;
        if (cnt[i] && maxl > RC(0.0)) w = (uint32_t)((lum[i] / maxl) * RC(1048576.0));
        acc += w;
        cdf[i] = acc;
    }
}

void ORC(reconstruct_probe)(const real *pp, const real *pn, real cs, uint32_t nq, const real *qpos,
                            const real *qnrm, const real *qatlas, real *recon, uint32_t *cdf)
{
    /* test entry: candidates given as arrays [nq][4], [nq][4], [nq][64][4] */
    const real *a[9], *b[9], *c[9];
    uint32_t n = nq > 9 ? 9 : nq;
    for (uint32_t j = 0; j < n; ++j) {
        a[j] = qpos + 4 * (size_t)j;
        b[j] = qnrm + 4 * (size_t)j;
        c[j] = qatlas + (size_t)j * NCELL * 4;
    }
    recon_probe(pp, pn, cs, n, a, b, c, recon, cdf);
}

static void reconstruct(state *st, const orc_frame *fr)
{
    real kappa = (real)ORC(distance_scale)(fr->fov_y, st->W, st->H);
#pragma omp parallel for schedule(dynamic, 16)
    for (long p = 0; p < (long)st->P; ++p) {
        real *rc = st->recon + (size_t)p * NCELL * 4;
        uint32_t *cdf = st->cdf + (size_t)p * NCELL;
        const real *qp[9], *qn[9], *qa[9];
        uint32_t nq = 0;
        const real *pp = st->ppos + 4 * p, *pn = st->pnrm + 4 * p;
        real cs = RC(0.0);
        int32_t qx = 0, qy = 0;
        if (st->mask[p] != SENTINEL && project_prev(st, pp, &qx, &qy)) {
            real ex = pp[0] - st->cam[0], ey = pp[1] - st->cam[1], ez = pp[2] - st->cam[2];
            cs = kappa * RSQRT((ex * ex + ey * ey) + ez * ez);
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int32_t tx = (qx >> 3) + dx, ty = (qy >> 3) + dy;
                    if (tx < 0 || ty < 0 || tx >= (int32_t)st->TW || ty >= (int32_t)st->TH) continue;
                    uint32_t q = (uint32_t)ty * st->TW + (uint32_t)tx;
                    if (st->prev_mask[q] == SENTINEL) continue;
                    qp[nq] = st->prev_pos + 4 * (size_t)q;
                    qn[nq] = st->prev_nrm + 4 * (size_t)q;
                    qa[nq] = st->prev_atlas + (size_t)q * NCELL * 4;
                    ++nq;
                }
        }
        recon_probe(pp, pn, cs, nq, qp, qn, qa, rc, cdf);
    }
}

/* a ray's direction inside atlas cell k: uniform point (u0, u1) of the cell's square in the
 * hemi-octahedral domain, mapped back to the hemisphere about n */
static void guided_dir(const real *n, uint32_t k, real u0, real u1, real *d)
{
    real uu = ((real)(k & 7u) + u0) * RC(0.25) - RC(1.0);
    real vv = ((real)(k >> 3) + u1) * RC(0.25) - RC(1.0);
    real a = (uu + vv) * RC(0.5), b = (uu - vv) * RC(0.5);
    real z = (RC(1.0) - RABS(a)) - RABS(b);
    real len = RSQRT((a * a + b * b) + z * z);
    real lx = a / len, ly = b / len, lz = z / len;
    real t[3], bb[3];
    onb(n, t, bb);
    for (int j = 0; j < 3; ++j) d[j] = (lx * t[j] + ly * bb[j]) + lz * n[j];
}

/* cell picked by a 32-bit random number r: the first whose inclusive weight sum exceeds
 * floor(r * total / 2^32) */
static uint32_t pick_cell(const uint32_t *cdf, uint32_t r)
{
    uint32_t target = (uint32_t)(((uint64_t)r * cdf[NCELL - 1]) >> 32);
    uint32_t k = 0;
    while (cdf[k] <= target) ++k;
    return k;
}

void ORC(guided_dirs)(const real *n, const uint32_t *cdf, const uint32_t *r, const real *u0, const real *u1,
                      uint32_t cnt, real *d, uint32_t *cell)
{
    /* test entry: ray directions of a probe with normal n and weight sums cdf */
    for (uint32_t i = 0; i < cnt; ++i) {
        cell[i] = pick_cell(cdf, r[i]);
        guided_dir(n, cell[i], u0[i], u1[i], d + 3 * i);
    }
}

void ORC(spawn)(state *st, const orc_frame *fr, const real *gpos, const real *gnrm, const uint32_t *gprim)
{
    const uint32_t u = st->cfg.upscale > 1 ? st->cfg.upscale : 1u;
    st->sjx = halton_n(fr->index + 1u, 2u, 8u * u);
    st->sjy = halton_n(fr->index + 1u, 3u, 8u * u);
    st->jx = st->sjx % 8u;    /* lattice offset of the interpolation */
    st->jy = st->sjy % 8u;
    for (int k = 0; k < 3; ++k) st->cam[k] = (real)fr->pos[k];
    if (st->cfg.temporal && st->has_prev) reproject(st, fr, gpos, gnrm, gprim);
    else for (uint32_t t = 0; t < st->P; ++t) st->win[t] = st->hist[t] = SENTINEL;
    uint32_t *place = (uint32_t *)malloc(sizeof(uint32_t) * st->P);
    place_probes(st, fr, gprim, place);
    for (uint32_t ty = 0; ty < st->TH; ++ty)
        for (uint32_t tx = 0; tx < st->TW; ++tx) {
            uint32_t p = ty * st->TW + tx;
            uint32_t m = place[p];
            uint32_t px = m & 0xFFFFu, py = m >> 16;
            st->mask[p] = m;
            for (int k = 0; k < 4; ++k) {
                if (m == SENTINEL) {
                    st->ppos[4 * p + k] = st->pnrm[4 * p + k] = RC(0.0);
                } else {
                    size_t pix = (size_t)py * st->W + px;
                    st->ppos[4 * p + k] = gpos[4 * pix + k];
                    st->pnrm[4 * p + k] = gnrm[4 * pix + k];
                }
            }
        }
    free(place);
    st->guided = st->cfg.ray_guiding && st->cfg.temporal && st->has_prev;
    if (st->guided) reconstruct(st, fr);
    for (uint32_t k = 1; k < st->nmip; ++k) {
        const uint32_t *src = st->mask + st->mip_off[k - 1];
        uint32_t *dst = st->mask + st->mip_off[k];
        uint32_t sw = st->mip_w[k - 1], sh = st->mip_h[k - 1];
        for (uint32_t y = 0; y < st->mip_h[k]; ++y)
            for (uint32_t x = 0; x < st->mip_w[k]; ++x) {
                uint32_t v = SENTINEL;
                for (uint32_t c = 0; c < 4 && v == SENTINEL; ++c) {
                    uint32_t cx = 2 * x + (c & 1), cy = 2 * y + (c >> 1);
                    if (cx < sw && cy < sh) v = src[cy * sw + cx];
                }
                dst[y * st->mip_w[k] + x] = v;
            }
    }
}

/* ---------------------------------------------------------------------------------------
 * Trace (Sections 2.1.3, 2.2.1-2.2.4, 2.3.1): every probe ray finds its closest hit; a hit
 * looks up (or creates) its world-cache cell and contributes one radiance sample to it:
 * next-event estimation with one shadow ray towards an area-sampled emitter point, plus, with
 * two bounces, the cached outgoing radiance found at the end of a cosine-sampled ray
 * (temporal radiance feedback).  Samples are accumulated in fixed point (FP32 mode).
 * ------------------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------------------
 * Light grid and resampled light sampling (Section 2.3: importance sampling of the lights
 * with RIS and weighted reservoir sampling; the light grid of Section 2.3.2 feeds the
 * candidates).  Lights are the emitter triangles: area A, centroid c, unit normal n (the
 * emitting side), luminance l of Le (Rec. 709), power-like weight phi = l A.
 * Light grid: over the axis-aligned box of this frame's probe-ray hit points, cubic cells of
 * side h = (largest extent) / lgrid_dim, at most lgrid_dim per axis.  A light is culled from
 * a cell when the cell's bounding sphere (centre, radius h sqrt(3) / 2) lies entirely behind
 * the light's plane, or farther from its centroid than its range sqrt(phi / lgrid_tau) plus
 * the radius.  Importance = the mean over the cell's 8 corners of phi cos / max(d^2, A) (a
 * small-source contribution, cos from the light's normal; the mean of the corners is the
 * volume integral of their trilinear interpolant over the cell volume); each cell keeps the
 * min(lgrid_k, lights) most important lights with importance > 0 (ties: lower index first).
 * RIS: ris_m candidates, each a light picked uniformly from the hit's cell list and a
 * uniform point on it (source pdf 1 / (count A)), target l cos_y cos_l / d^2, weight
 * target / source pdf; streaming weighted reservoir sampling keeps one candidate; one
 * shadow ray; the estimate is Le cos_y cos_l / d^2 * (sum of weights) / (ris_m target).
 * READING: grid bounds from the probe-ray hits (the shading points); no spotlights or point
 * lights (the scenes' lights are emissive triangles); the reservoirs are not stored in a
 * hash grid and not reused over time (not built).
 * ------------------------------------------------------------------------------------- */
static real lum709(const float *le)
{
    return ((real)0.2126f * (real)le[0] + (real)0.7152f * (real)le[1]) + (real)0.0722f * (real)le[2];
}

static void light_attr(const scene *sc, uint32_t k, real *cen, real *A, const real **n, const float **le)
{
    uint32_t t = sc->etri[k];
    const float *v = sc->tv + 9 * (size_t)t;
    for (int j = 0; j < 3; ++j) cen[j] = (real)((((double)v[j] + (double)v[3 + j]) + (double)v[6 + j]) / 3.0);
    *A = (real)tri_area_f64(v);
    *n = sc->tn + 3 * (size_t)t;
    *le = sc->mats + 6 * sc->tmat[t] + 3;
}

static uint32_t lgrid_cell_of(const state *st, const real *y)
{
    uint32_t ix[3];
    for (int k = 0; k < 3; ++k) {
        real f = RFLOOR((y[k] - st->lg_lo[k]) / st->lg_h);
        int32_t i = f < RC(0.0) ? 0 : (f > (real)(st->lg_dim[k] - 1) ? (int32_t)st->lg_dim[k] - 1 : (int32_t)f);
        ix[k] = (uint32_t)i;
    }
    return (ix[2] * st->lg_dim[1] + ix[1]) * st->lg_dim[0] + ix[0];
}

static real light_importance(const state *st, uint32_t cx, uint32_t cy, uint32_t cz, uint32_t k)
{
    const scene *sc = st->sc;
    real cen[3], A;
    const real *n;
    const float *le;
    light_attr(sc, k, cen, &A, &n, &le);
    real phi = lum709(le) * A;
    real h = st->lg_h;
    uint32_t ci[3] = {cx, cy, cz};
    real cc[3];
    for (int j = 0; j < 3; ++j) cc[j] = st->lg_lo[j] + ((real)ci[j] + RC(0.5)) * h;
    real R = h * RC(0.8660254037844386);
    real sd = ((cc[0] - cen[0]) * n[0] + (cc[1] - cen[1]) * n[1]) + (cc[2] - cen[2]) * n[2];
    if (sd < -R) return RC(-1.0);
    real dx = cc[0] - cen[0], dy = cc[1] - cen[1], dz = cc[2] - cen[2];
    real dist = RSQRT((dx * dx + dy * dy) + dz * dz);
    real range = RSQRT(phi / (real)st->cfg.lgrid_tau);
    if (dist > range + R) return RC(-1.0);
    real imp = RC(0.0);
    for (uint32_t q = 0; q < 8; ++q) {
        real v[3];
        for (int j = 0; j < 3; ++j) v[j] = (st->lg_lo[j] + (real)(ci[j] + ((q >> j) & 1u)) * h) - cen[j];
        real vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
        real len = RSQRT(vv);
        real cs = len > RC(0.0) ? ((v[0] * n[0] + v[1] * n[1]) + v[2] * n[2]) / len : RC(0.0);
        if (cs > RC(0.0)) imp = imp + (phi * cs) / rmax(vv, A);
    }
    return imp * RC(0.125);
}

static void light_grid_build(state *st, const real *lo, const real *hi)
{
    const orc_config *c = &st->cfg;
    real emax = RC(0.0);
    for (int k = 0; k < 3; ++k) {
        st->lg_lo[k] = lo[k];
        emax = rmax(emax, hi[k] - lo[k]);
    }
    real h = emax / (real)c->lgrid_dim;
    st->lg_h = h > RC(0.0) ? h : RC(1.0);
    for (int k = 0; k < 3; ++k) {
        real q = -RFLOOR(-((hi[k] - lo[k]) / st->lg_h));
        uint32_t d = q < RC(1.0) ? 1u : (uint32_t)q;
        st->lg_dim[k] = d > c->lgrid_dim ? c->lgrid_dim : d;
    }
    uint32_t K = c->lgrid_k < st->sc->ne ? c->lgrid_k : st->sc->ne;
    uint32_t ncell = st->lg_dim[0] * st->lg_dim[1] * st->lg_dim[2];
#pragma omp parallel for schedule(dynamic, 4)
    for (long ci = 0; ci < (long)ncell; ++ci) {
        uint32_t cx = (uint32_t)ci % st->lg_dim[0], cy = ((uint32_t)ci / st->lg_dim[0]) % st->lg_dim[1];
        uint32_t cz = (uint32_t)ci / (st->lg_dim[0] * st->lg_dim[1]);
        uint32_t ne = st->sc->ne, cnt = 0;
        real *imp = (real *)malloc(sizeof(real) * (ne ? ne : 1));
        for (uint32_t k = 0; k < ne; ++k) imp[k] = light_importance(st, cx, cy, cz, k);
        /* the K largest, ties by lower index (selection by repeated maximum) */
        for (uint32_t r = 0; r < K; ++r) {
            uint32_t best = 0xFFFFFFFFu;
            for (uint32_t k = 0; k < ne; ++k)
                if (imp[k] > RC(0.0) && (best == 0xFFFFFFFFu || imp[k] > imp[best])) best = k;
            if (best == 0xFFFFFFFFu) break;
            st->lg_list[(size_t)ci * c->lgrid_k + cnt++] = best;
            imp[best] = RC(-1.0);
        }
        st->lg_count[ci] = cnt;
        free(imp);
    }
}

void ORC(light_grid_set)(state *st, const real *lo, const real *hi)
{
    /* test entry: build the grid over a given box */
    light_grid_build(st, lo, hi);
}

void ORC(light_grid_export)(const state *st, real *geom /* lo[3], h */, uint32_t *dims, uint32_t *list,
                            uint32_t *count)
{
    for (int k = 0; k < 3; ++k) geom[k] = st->lg_lo[k];
    geom[3] = st->lg_h;
    for (int k = 0; k < 3; ++k) dims[k] = st->lg_dim[k];
    uint32_t n = st->lg_dim[0] * st->lg_dim[1] * st->lg_dim[2];
    memcpy(list, st->lg_list, sizeof(uint32_t) * (size_t)n * st->cfg.lgrid_k);
    memcpy(count, st->lg_count, sizeof(uint32_t) * n);
}

/* World-space reservoir reuse (Section 2.3.1): the reservoir table is a spatial hash like the
 * world cache's over the quantised position alone (the descriptor with normal class 0, no
 * leak bit; levels of detail as the cache's), with the storing vertex's normal beside it.
 * READING: a hit reuses the previous frame's reservoir of its cell when the normals' cosine
 * exceeds 0.9 (bilateral test); the stored count is capped at restir_cap x ris_m; the reused sample
 * enters with weight target_here(y) * W * M and one more weighted-reservoir step (hash
 * dimension 48); every hit's final reservoir (before its shadow ray) is offered to its cell
 * of this frame's table, where the lowest ray id is kept. */
static uint64_t pos_key(const orc_config *c, const real *cam, const real *y)
{
    orc_config cc = *c;
    cc.cache_tiles = 0;
    real n[3] = {RC(1.0), RC(0.0), RC(0.0)};
    return cell_key_cell(&cc, cam, y, n, RC(0.0), 0, NULL);
}

static int32_t rs_find(const state *st, int t, uint64_t key)
{
    uint32_t nb = st->rs_N / BUCKET;
    uint32_t b = key_bucket(key, nb), f = key_fingerprint(key);
    for (uint32_t s = 0; s < BUCKET; ++s)
        if (st->rs_fp[t][b * BUCKET + s] == f) return (int32_t)(b * BUCKET + s);
    return -1;
}

static int32_t rs_insert(state *st, int t, uint64_t key)
{
    uint32_t nb = st->rs_N / BUCKET;
    uint32_t b = key_bucket(key, nb), f = key_fingerprint(key);
    for (uint32_t s = 0; s < BUCKET; ++s)
        if (st->rs_fp[t][b * BUCKET + s] == f) return (int32_t)(b * BUCKET + s);
    for (uint32_t s = 0; s < BUCKET; ++s) {
        uint32_t slot = b * BUCKET + s;
        if (st->rs_fp[t][slot] == 0u) {
            st->rs_fp[t][slot] = f;
            st->rs_key[t][slot] = key;
            return (int32_t)slot;
        }
    }
    return -1;
}

/* a light point x on emitter k seen from yo with normal ny: target (luminance * g) and g */
static void light_target(const scene *sc, uint32_t k, const real *x, const real *yo, const real *ny, real *ph,
                         real *g, real *om, real *dist)
{
    uint32_t t = sc->etri[k];
    real w[3];
    for (int q = 0; q < 3; ++q) w[q] = x[q] - yo[q];
    real d2 = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
    *ph = RC(0.0);
    *g = RC(0.0);
    *dist = RC(0.0);
    om[0] = om[1] = om[2] = RC(0.0);
    if (!(d2 > RC(0.0))) return;
    *dist = RSQRT(d2);
    for (int q = 0; q < 3; ++q) om[q] = w[q] / *dist;
    const real *nl = sc->tn + 3 * (size_t)t;
    real cos_y = (ny[0] * om[0] + ny[1] * om[1]) + ny[2] * om[2];
    real cos_l = -((nl[0] * om[0] + nl[1] * om[1]) + nl[2] * om[2]);
    if (cos_y > RC(0.0) && cos_l > RC(0.0)) {
        *g = (cos_y * cos_l) / d2;
        *ph = lum709(sc->mats + 6 * sc->tmat[t] + 3) * *g;
    }
}

/* RIS over the cell's light list (+ the previous frame's reservoir with restir): E
 * (irradiance estimate times pi, before albedo); with restir, the final reservoir of the hit
 * into the per-ray arrays at gid */
static void ris_light(state *st, const orc_frame *fr, uint32_t gid, const real *y, const real *yo,
                      const real *ny, real *E, uint64_t *stat_shadow, uint64_t *stat_occ, int store)
{
    const orc_config *c = &st->cfg;
    const scene *sc = st->sc;
    uint32_t cell = lgrid_cell_of(st, y);
    uint32_t m = st->lg_count[cell];
    const uint32_t *list = st->lg_list + (size_t)cell * c->lgrid_k;
    real wsum = RC(0.0), ph_sel = RC(0.0), g_sel = RC(0.0), dist_sel = RC(0.0);
    real om_sel[3] = {RC(0.0), RC(0.0), RC(0.0)}, x_sel[3] = {RC(0.0), RC(0.0), RC(0.0)};
    uint32_t k_sel = 0xFFFFFFFFu, M = 0;
    if (m > 0) {
        M = c->ris_m;
        for (uint32_t j = 0; j < c->ris_m; ++j) {
            uint32_t rp = rng_u32(c->seed, fr->index, gid, 16u + 4u * j);
            uint32_t k = list[(uint32_t)(((uint64_t)rp * m) >> 32)];
            real u3 = rng_unit(rng_u32(c->seed, fr->index, gid, 17u + 4u * j));
            real u4 = rng_unit(rng_u32(c->seed, fr->index, gid, 18u + 4u * j));
            real us = rng_unit(rng_u32(c->seed, fr->index, gid, 19u + 4u * j));
            uint32_t t = sc->etri[k];
            real su = RSQRT(u3);
            real b0 = RC(1.0) - su, b1 = su * (RC(1.0) - u4), b2 = su * u4;
            const float *v = sc->tv + 9 * (size_t)t;
            real x[3];
            for (int q = 0; q < 3; ++q) x[q] = (b0 * (real)v[q] + b1 * (real)v[3 + q]) + b2 * (real)v[6 + q];
            real ph, g, dist, om[3];
            light_target(sc, k, x, yo, ny, &ph, &g, om, &dist);
            real A = (real)tri_area_f64(v);
            real wj = (ph * (real)m) * A;
            wsum = wsum + wj;
            if (wj > RC(0.0) && us * wsum < wj) {
                k_sel = k;
                ph_sel = ph;
                g_sel = g;
                dist_sel = dist;
                for (int q = 0; q < 3; ++q) { om_sel[q] = om[q]; x_sel[q] = x[q]; }
            }
        }
    }
    if (c->restir && st->rs_has_prev) {
        int pt = (int)st->rs_cur;
        int32_t s = rs_find(st, pt, pos_key(c, st->cam, y));
        if (s >= 0) {
            const real *np = st->rs_n[pt] + 3 * (size_t)s;
            real cn = (ny[0] * np[0] + ny[1] * np[1]) + ny[2] * np[2];
            if (cn > RC(0.9)) {
                uint32_t kp = st->rs_k[pt][s];
                const real *xp = st->rs_y[pt] + 3 * (size_t)s;
                uint32_t cap = c->restir_cap * c->ris_m;
                uint32_t Mp = st->rs_M[pt][s] < cap ? st->rs_M[pt][s] : cap;
                real ph, g, dist, om[3];
                light_target(sc, kp, xp, yo, ny, &ph, &g, om, &dist);
                real wp = (ph * st->rs_W[pt][s]) * (real)Mp;
                wsum = wsum + wp;
                real us = rng_unit(rng_u32(c->seed, fr->index, gid, 48u));
                if (wp > RC(0.0) && us * wsum < wp) {
                    k_sel = kp;
                    ph_sel = ph;
                    g_sel = g;
                    dist_sel = dist;
                    for (int q = 0; q < 3; ++q) { om_sel[q] = om[q]; x_sel[q] = xp[q]; }
                }
                M = M + Mp;
            }
        }
    }
    if (k_sel == 0xFFFFFFFFu) return;
    real W = wsum / ((real)M * ph_sel);
    if (store && c->restir) {
        st->r_rsM[gid] = M;
        st->r_rsk[gid] = k_sel;
        st->r_rsW[gid] = W;
        for (int q = 0; q < 3; ++q) st->r_rsy[3 * (size_t)gid + q] = x_sel[q];
    }
    (*stat_shadow)++;
    if (any_hit(sc, yo, om_sel, dist_sel * RC(0.9999))) {
        (*stat_occ)++;
        return;
    }
    const float *le = sc->mats + 6 * sc->tmat[sc->etri[k_sel]] + 3;
    real gw = g_sel * W;
    for (int q = 0; q < 3; ++q) E[q] = (real)le[q] * gw;
}

/* this frame's reservoirs into the table written this frame (ray order: the lowest ray id of
 * a cell stays), then that table becomes the one read next frame */
static void restir_store(state *st)
{
    int nt = (int)(st->rs_cur ^ 1u);
    memset(st->rs_fp[nt], 0, sizeof(uint32_t) * st->rs_N);
    memset(st->rs_key[nt], 0, sizeof(uint64_t) * st->rs_N);
    memset(st->rs_claim, 0, sizeof(uint32_t) * st->rs_N);
    size_t PR = (size_t)st->P * st->R;
    for (size_t gid = 0; gid < PR; ++gid) {
        if (!(st->r_cell[gid] & 0x100u) || st->r_rsM[gid] == 0) continue;
        int32_t s = rs_insert(st, nt, pos_key(&st->cfg, st->cam, st->r_y + 3 * gid));
        if (s < 0 || st->rs_claim[s]) continue;
        st->rs_claim[s] = 1;
        st->rs_k[nt][s] = st->r_rsk[gid];
        st->rs_M[nt][s] = st->r_rsM[gid];
        st->rs_W[nt][s] = st->r_rsW[gid];
        for (int q = 0; q < 3; ++q) {
            st->rs_y[nt][3 * (size_t)s + q] = st->r_rsy[3 * gid + q];
            st->rs_n[nt][3 * (size_t)s + q] = st->r_ny[3 * gid + q];
        }
    }
    st->rs_cur = (uint32_t)nt;
    st->rs_has_prev = 1;
}

/* the reservoir table written by the last trace, live slots in slot order */
uint32_t ORC(restir_export)(const state *st, uint64_t *id, uint64_t *key, real *y, real *W, real *n, uint32_t *k,
                            uint32_t *M, uint32_t cap)
{
    if (!st->cfg.restir) return 0;
    int t = (int)st->rs_cur;
    uint32_t cnt = 0;
    for (uint32_t s = 0; s < st->rs_N; ++s) {
        if (st->rs_fp[t][s] == 0u) continue;
        if (cnt < cap) {
            id[cnt] = ((uint64_t)(s / BUCKET) << 32) | st->rs_fp[t][s];
            key[cnt] = st->rs_key[t][s];
            for (int q = 0; q < 3; ++q) {
                y[3 * (size_t)cnt + q] = st->rs_y[t][3 * (size_t)s + q];
                n[3 * (size_t)cnt + q] = st->rs_n[t][3 * (size_t)s + q];
            }
            W[cnt] = st->rs_W[t][s];
            k[cnt] = st->rs_k[t][s];
            M[cnt] = st->rs_M[t][s];
        }
        ++cnt;
    }
    return cnt;
}

static void shade_hit(state *st, const orc_frame *fr, uint32_t gid, const real *y,
                      const real *ny, real *s_out, int32_t *bslot, uint64_t *stat_shadow,
                      uint64_t *stat_occ, uint64_t *stat_bounce, int store)
{
    const orc_config *c = &st->cfg;
    const scene *sc = st->sc;
    real E[3] = {RC(0.0), RC(0.0), RC(0.0)};
    real eps = offset_eps(c, y);
    real yo[3];
    for (int k = 0; k < 3; ++k) yo[k] = y[k] + ny[k] * eps;
    if (sc->ne > 0 && c->light_grid) {
        ris_light(st, fr, gid, y, yo, ny, E, stat_shadow, stat_occ, store);
    } else if (sc->ne > 0) {
        uint32_t e = sc->etri[pick_emitter(sc, rng_u32(c->seed, fr->index, gid, 2u))];
        real u3 = rng_unit(rng_u32(c->seed, fr->index, gid, 3u));
        real u4 = rng_unit(rng_u32(c->seed, fr->index, gid, 4u));
        real su = RSQRT(u3);
        real b0 = RC(1.0) - su, b1 = su * (RC(1.0) - u4), b2 = su * u4;
        const float *v = sc->tv + 9 * (size_t)e;
        real xl[3], w[3];
        for (int k = 0; k < 3; ++k) xl[k] = (b0 * (real)v[k] + b1 * (real)v[3 + k]) + b2 * (real)v[6 + k];
        for (int k = 0; k < 3; ++k) w[k] = xl[k] - yo[k];
        real d2 = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
        if (d2 > RC(0.0)) {
            real dist = RSQRT(d2);
            real om[3] = {w[0] / dist, w[1] / dist, w[2] / dist};
            const real *ne = sc->tn + 3 * (size_t)e;
            real cos_y = (ny[0] * om[0] + ny[1] * om[1]) + ny[2] * om[2];
            real cos_l = -((ne[0] * om[0] + ne[1] * om[1]) + ne[2] * om[2]);
            if (cos_y > RC(0.0) && cos_l > RC(0.0)) {
                (*stat_shadow)++;
                if (!any_hit(sc, yo, om, dist * RC(0.9999))) {
                    real g = ((cos_y * cos_l) * sc->area_total) / d2;
                    const float *m = sc->mats + 6 * sc->tmat[e];
                    for (int k = 0; k < 3; ++k) E[k] = (real)m[3 + k] * g;
                } else {
                    (*stat_occ)++;
                }
            }
        }
    }
    real Lb[3] = {RC(0.0), RC(0.0), RC(0.0)};
    *bslot = -1;
    if (c->bounces >= 2) {
        (*stat_bounce)++;
        real u5 = rng_unit(rng_u32(c->seed, fr->index, gid, 5u));
        real u6 = rng_unit(rng_u32(c->seed, fr->index, gid, 6u));
        real d[3];
        cosine_dir(ny, u5, u6, d, NULL);
        uint32_t tri;
        real t;
        closest_hit(sc, yo, d, RC(3.0e38), &tri, &t);
        if (tri == MISS) {
            for (int k = 0; k < 3; ++k) Lb[k] = (real)c->sky[k];
        } else {
            real z[3], nz[3];
            const real *n = sc->tn + 3 * (size_t)tri;
            real dn = (n[0] * d[0] + n[1] * d[1]) + n[2] * d[2];
            real sg = dn > RC(0.0) ? RC(-1.0) : RC(1.0);
            for (int k = 0; k < 3; ++k) { z[k] = yo[k] + t * d[k]; nz[k] = sg * n[k]; }
            uint32_t tc;
            uint64_t bkey = cell_key_cell(c, st->cam, z, nz, t, 1, &tc);
            int32_t e = cache_entry(st, table_find(st, bkey), tc);
            *bslot = e;
            if (e >= 0)
                for (int k = 0; k < 3; ++k) Lb[k] = cache_L(st)[3 * (size_t)e + k];
        }
    }
    for (int k = 0; k < 3; ++k) s_out[k] = E[k] * RC(0.31830988618379067) + Lb[k];
}

void ORC(trace)(state *st, const orc_frame *fr)
{
    const orc_config *c = &st->cfg;
    const scene *sc = st->sc;
    uint32_t R = st->R;
    uint64_t nshadow = 0, nocc = 0, nbounce = 0;
    /* parallel phase: rays, hits, keys, samples; nothing here writes the table */
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nshadow, nocc, nbounce)
    for (long p = 0; p < (long)st->P; ++p) {
        int valid = st->traced[p] != 0;
        for (uint32_t r = 0; r < R; ++r) {
            size_t gid = (size_t)p * R + r;
            st->r_slot[gid] = -1;
            st->r_t[gid] = RC(0.0);
            st->r_tri[gid] = MISS;
            st->r_cell[gid] = 0;
            st->r_valid[gid] = 0;
            st->r_bslot[gid] = -1;
            if (!valid) continue;
            const real *pp = st->ppos + 4 * p, *pn = st->pnrm + 4 * p;
            real u0 = rng_unit(rng_u32(c->seed, fr->index, (uint32_t)gid, 0u));
            real u1 = rng_unit(rng_u32(c->seed, fr->index, (uint32_t)gid, 1u));
            real d[3], o[3];
            uint32_t cell;
            const uint32_t *cdf = st->cdf + (size_t)p * NCELL;
            if (st->guided && cdf[NCELL - 1] > 0) {
                cell = pick_cell(cdf, rng_u32(c->seed, fr->index, (uint32_t)gid, 8u));
                guided_dir(pn, cell, u0, u1, d);
            } else {
                cosine_dir(pn, u0, u1, d, &cell);
            }
            real eps = offset_eps(c, pp);
            for (int k = 0; k < 3; ++k) o[k] = pp[k] + pn[k] * eps;
            uint32_t tri;
            real t;
            closest_hit(sc, o, d, RC(3.0e38), &tri, &t);
            uint32_t flags = cell | 0x10000u;   /* bit 16: probe ray traced */
            if (tri == MISS) {
                st->r_t[gid] = (real)c->t_sky;
                st->r_cell[gid] = flags;
                continue;
            }
            const real *n = sc->tn + 3 * (size_t)tri;
            real dn = (n[0] * d[0] + n[1] * d[1]) + n[2] * d[2];
            real sg = dn > RC(0.0) ? RC(-1.0) : RC(1.0);
            real y[3], ny[3];
            for (int k = 0; k < 3; ++k) { y[k] = o[k] + t * d[k]; ny[k] = sg * n[k]; }
            flags |= 0x100u;                     /* bit 8: hit */
            if (dn < RC(0.0)) {
                flags |= 0x200u;                 /* bit 9: front face (one-sided emission) */
                const float *mt = sc->mats + 6 * sc->tmat[tri];
                if (mt[3] > 0.0f || mt[4] > 0.0f || mt[5] > 0.0f) flags |= 0x400u;   /* bit 10: emitter */
            }
            st->r_t[gid] = t;
            st->r_tri[gid] = tri;
            st->r_cell[gid] = flags;
            uint64_t key = cell_key_cell(c, st->cam, y, ny, t, 1, &st->r_tcell[gid]);
            st->r_keylo[gid] = (uint32_t)key;
            st->r_keyhi[gid] = (uint32_t)(key >> 32);
            for (int k = 0; k < 3; ++k) { st->r_y[3 * gid + k] = y[k]; st->r_ny[3 * gid + k] = ny[k]; }
        }
    }
    size_t PR = (size_t)st->P * R;
    if (c->light_grid) {
        /* the light grid over the box of this frame's hit points */
        real lo[3] = {RC(0.0), RC(0.0), RC(0.0)}, hi[3] = {RC(0.0), RC(0.0), RC(0.0)};
        int any = 0;
        for (size_t gid = 0; gid < PR; ++gid) {
            if (!(st->r_cell[gid] & 0x100u)) continue;
            for (int k = 0; k < 3; ++k) {
                real v = st->r_y[3 * gid + k];
                if (!any || v < lo[k]) lo[k] = v;
                if (!any || v > hi[k]) hi[k] = v;
            }
            any = 1;
        }
        light_grid_build(st, lo, hi);
    }
    /* shading of the hits (light sample, cached bounce) */
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nshadow, nocc, nbounce)
    for (long g = 0; g < (long)PR; ++g) {
        size_t gid = (size_t)g;
        if (!(st->r_cell[gid] & 0x100u)) continue;
        real s[3];
        if (c->restir) st->r_rsM[gid] = 0;
        shade_hit(st, fr, (uint32_t)gid, st->r_y + 3 * gid, st->r_ny + 3 * gid, s, &st->r_bslot[gid], &nshadow,
                  &nocc, &nbounce, 1);
        const float *m = sc->mats + 6 * sc->tmat[st->r_tri[gid]];
        for (int k = 0; k < 3; ++k) st->r_sample[3 * gid + k] = (real)m[k] * s[k];
        st->r_valid[gid] = 1;
    }
    st->stats[ST_SHADOW] += nshadow;
    st->stats[ST_OCCLUDED] += nocc;
    st->stats[ST_BOUNCE] += nbounce;
    /* sequential phase: cell lookup/creation and accumulation in ray order */
    for (size_t gid = 0; gid < PR; ++gid) {
        if (!(st->r_cell[gid] & 0x10000u)) continue;
        st->stats[ST_RAYS]++;
        if (!st->r_valid[gid]) continue;
        st->stats[ST_HITS]++;
        uint64_t key = (uint64_t)st->r_keylo[gid] | ((uint64_t)st->r_keyhi[gid] << 32);
        int32_t tslot = table_insert(st, key);
        int32_t slot = cache_entry(st, tslot, st->r_tcell[gid]);
        st->r_slot[gid] = slot;
        if (slot < 0) continue;
        st->accessed[tslot] = 1;
        const real *s = st->r_sample + 3 * gid;
        if (!isfinite((double)s[0]) || !isfinite((double)s[1]) || !isfinite((double)s[2])) {
            st->stats[ST_NONFINITE]++;
            continue;
        }
        for (int k = 0; k < 3; ++k) {
            real v = rmin(rmax(s[k], RC(0.0)), (real)c->r_max);
#ifdef ORC_F64
            st->dacc[3 * (size_t)slot + k] += v;
#else
            float scaled = v * (float)(1u << c->frac_bits);
            uint32_t q = (uint32_t)rintf(scaled);
            uint32_t old = st->acc[4 * (size_t)slot + k];
            st->acc[4 * (size_t)slot + k] = old + q;
            if (old + q < old) st->stats[ST_WRAPS]++;
#endif
        }
        st->acc[4 * (size_t)slot + 3] += 1u;
    }
    /* cells found by bounce lookups count as accessed; the lookups saw the table as it was
     * before this frame's insertions, so their order does not matter */
    for (size_t gid = 0; gid < PR; ++gid)
        if (st->r_bslot[gid] >= 0)
            st->accessed[st->cfg.cache_tiles ? st->r_bslot[gid] / NCELL : st->r_bslot[gid]] = 1u;
    if (c->restir && c->light_grid) restir_store(st);
}

/* NEE radiance estimate E/pi (before albedo) for a surface point and normal, one estimate per
 * sample id: the estimator used when filling cells (test entry; bounces are not taken) */
void ORC(nee_samples)(state *st, const orc_frame *fr, const real *y, const real *ny,
                      const uint32_t *ids, uint32_t n, real *out)
{
    uint32_t saved = st->cfg.bounces;
    st->cfg.bounces = 1;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)n; ++i) {
        uint64_t a = 0, b = 0, c = 0;
        int32_t bs;
        shade_hit(st, fr, ids[i], y, ny, out + 3 * i, &bs, &a, &b, &c, 0);
    }
    st->cfg.bounces = saved;
}

/* ---------------------------------------------------------------------------------------
 * Cache update (Section 2.2.1 decay and deallocation; Section 2.2.3 temporal accumulation).
 * READING: the frame's mean sample enters an exponential moving average weighted by sample
 * counts, capped at n_cap samples of history; the decay value is an integer life reset to
 * max_life on access, decremented otherwise, and the cell is freed at zero.
 * ------------------------------------------------------------------------------------- */
/* moving average of one cell (entry e) with this frame's samples (Section 2.2.3) */
static void ema_entry(state *st, size_t e)
{
    const orc_config *c = &st->cfg;
    double scale = (double)(1u << c->frac_bits);
    (void)scale;
    uint32_t cnt = st->acc[4 * e + 3];
    if (cnt == 0) return;
    uint32_t h = st->nhist[e] < c->n_cap ? st->nhist[e] : c->n_cap;
    real w = (real)cnt / (real)((double)h + (double)cnt);
    for (int k = 0; k < 3; ++k) {
#ifdef ORC_F64
        real mean = st->dacc[3 * e + k] / (double)cnt;
#else
        real mean = (float)((double)st->acc[4 * e + k] / ((double)cnt * scale));
#endif
        real L = st->L[3 * e + k];
        st->L[3 * e + k] = L + w * (mean - L);
    }
    uint64_t nh = (uint64_t)st->nhist[e] + cnt;
    st->nhist[e] = nh < c->n_cap ? (uint32_t)nh : c->n_cap;
}

/* Tile MIP levels (Section 2.2.3): level k+1 entry = sample-weighted box filter of its 2x2
 * children at level k (children in raster order), samples summed; each level-0 cell then
 * answers queries with the finest of its level and its parents that holds at least tile_min
 * samples, else the coarsest level if it holds any, else zero.
 * READING: "box filtering of radiance samples" weights each child by its sample count; the
 * levels are rebuilt from level 0 at every update, after the moving average. */
static void prefilter_cells(const real *L0, const uint32_t *n0, uint32_t T, real *Lq)
{
    real Lv[4][NCELL][3];
    uint32_t nv[4][NCELL];
    for (int i = 0; i < NCELL; ++i) {
        nv[0][i] = n0[i];
        for (int k = 0; k < 3; ++k) Lv[0][i][k] = L0[3 * i + k];
    }
    for (int lv = 1; lv < 4; ++lv) {
        int side = 8 >> lv;
        for (int y = 0; y < side; ++y)
            for (int x = 0; x < side; ++x) {
                real ws[3] = {RC(0.0), RC(0.0), RC(0.0)};
                uint32_t ns = 0;
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        int ch = (2 * y + dy) * (2 * side) + (2 * x + dx);
                        real fn = (real)nv[lv - 1][ch];
                        for (int k = 0; k < 3; ++k) ws[k] = ws[k] + fn * Lv[lv - 1][ch][k];
                        ns += nv[lv - 1][ch];
                    }
                int o = y * side + x;
                nv[lv][o] = ns;
                for (int k = 0; k < 3; ++k) Lv[lv][o][k] = ns ? ws[k] / (real)ns : RC(0.0);
            }
    }
    for (int i = 0; i < NCELL; ++i) {
        int x = i & 7, y = i >> 3;
        int pick = -1, o = 0;
        for (int lv = 0; lv < 4; ++lv) {
            o = (y >> lv) * (8 >> lv) + (x >> lv);
            if (nv[lv][o] >= T) { pick = lv; break; }
        }
        if (pick < 0 && nv[3][0] > 0) { pick = 3; o = 0; }
        for (int k = 0; k < 3; ++k) Lq[3 * i + k] = pick < 0 ? RC(0.0) : Lv[pick][o][k];
    }
}

static void prefilter_tile(state *st, uint32_t s)
{
    size_t e = (size_t)s * NCELL;
    prefilter_cells(st->L + 3 * e, st->nhist + e, st->cfg.tile_min, st->Lq + 3 * e);
}

void ORC(prefilter)(const real *L0, const uint32_t *n0, uint32_t T, real *Lq)
{
    /* test entry: one tile's 64 level-0 cells */
    prefilter_cells(L0, n0, T, Lq);
}

static void cache_update(state *st)
{
    const orc_config *c = &st->cfg;
    const size_t G = c->cache_tiles ? NCELL : 1;
    uint64_t live = 0;
    for (uint32_t s = 0; s < st->N; ++s) {
        if (st->fp[s] == 0u) continue;
        for (size_t i = 0; i < G; ++i) ema_entry(st, (size_t)s * G + i);
        if (st->accessed[s]) st->life[s] = c->max_life;
        else st->life[s] = st->life[s] - 1u;
        if (st->life[s] == 0u) {
            st->fp[s] = 0u;
            st->key[s] = 0u;
            for (size_t i = 0; i < G; ++i) {
                size_t e = (size_t)s * G + i;
                st->nhist[e] = 0u;
                for (int k = 0; k < 3; ++k) st->L[3 * e + k] = RC(0.0);
                if (c->cache_tiles)
                    for (int k = 0; k < 3; ++k) st->Lq[3 * e + k] = RC(0.0);
            }
            st->stats[ST_EVICT]++;
        } else {
            ++live;
            if (c->cache_tiles) prefilter_tile(st, s);
        }
        for (size_t i = 0; i < G; ++i) {
            size_t e = (size_t)s * G + i;
            for (int k = 0; k < 4; ++k) st->acc[4 * e + k] = 0u;
            for (int k = 0; k < 3; ++k) st->dacc[3 * e + k] = 0.0;
        }
        st->accessed[s] = 0u;
    }
    st->stats[ST_LIVE] = live;
}

/* ---------------------------------------------------------------------------------------
 * Probe gather (Section 2.1.4): per probe, every ray's radiance (sky on a miss, else the
 * hit's front-face emission plus the updated cached outgoing radiance) is averaged per
 * atlas cell in ray order; cells that received no ray get the mean of the populated cells
 * (radiance backup); alpha holds the mean travelled distance.  Every mean here is its sum
 * times the rounded reciprocal of its count (the paper fixes no rounding).
 * ------------------------------------------------------------------------------------- */
/* The radiance backup's mean (Section 2.1.4 fills the cells without rays with the average of
 * the populated ones; the order of that sum is not given): a balanced pairwise sum over the
 * 64 cells in index order, cells without a value counting as zero -- pairs (0,1), (2,3), ...,
 * then pairs of those sums, and so on. */
static real pair_sum64(const real *v, int stride)
{
    real t[NCELL];
    for (int i = 0; i < NCELL; ++i) t[i] = v[(size_t)i * stride];
    for (int w = 1; w < NCELL; w *= 2)
        for (int i = 0; i < NCELL; i += 2 * w) t[i] = t[i] + t[i + w];
    return t[0];
}

static void gather(state *st)
{
    const orc_config *c = &st->cfg;
    const scene *sc = st->sc;
    uint32_t R = st->R;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)st->P; ++p) {
        real *at = st->atlas + (size_t)p * NCELL * 4;
        for (int i = 0; i < NCELL * 4; ++i) at[i] = RC(0.0);
        if (st->mask[p] == SENTINEL) continue;
        if (!st->traced[p]) {
            /* a kept probe that traces nothing this frame (temporal upscaling) keeps the
             * radiance of the probe it was reprojected from; with ray guiding, the
             * parallax-corrected reconstruction, its empty cells filled with the mean of the
             * others */
            if (st->guided) {
                const real *rc = st->recon + (size_t)p * NCELL * 4;
                real val[NCELL * 4], mean[4];
                uint32_t npop = 0;
                for (int i = 0; i < NCELL; ++i) {
                    const int has = !(rc[4 * i + 3] < RC(0.0));
                    for (int k = 0; k < 4; ++k) val[4 * i + k] = has ? rc[4 * i + k] : RC(0.0);
                    npop += (uint32_t)has;
                }
                if (npop == 0) continue;
                const real inv = RC(1.0) / (real)npop;
                for (int k = 0; k < 4; ++k) mean[k] = pair_sum64(val + k, 4) * inv;
                for (int i = 0; i < NCELL; ++i)
                    for (int k = 0; k < 4; ++k) at[4 * i + k] = rc[4 * i + 3] < RC(0.0) ? mean[k] : rc[4 * i + k];
            } else if (st->hist[p] != SENTINEL) {
                memcpy(at, st->prev_atlas + (size_t)st->hist[p] * NCELL * 4, sizeof(real) * NCELL * 4);
            }
            continue;
        }
        real sum[NCELL][4];
        uint32_t cnt[NCELL];
        memset(cnt, 0, sizeof(cnt));
        for (int i = 0; i < NCELL; ++i) sum[i][0] = sum[i][1] = sum[i][2] = sum[i][3] = RC(0.0);
        for (uint32_t r = 0; r < R; ++r) {
            size_t gid = (size_t)p * R + r;
            uint32_t fl = st->r_cell[gid];
            uint32_t cell = fl & 63u;
            real v[3];
            if (!(fl & 0x100u)) {
                for (int k = 0; k < 3; ++k) v[k] = (real)c->sky[k];
            } else {
                const float *m = sc->mats + 6 * sc->tmat[st->r_tri[gid]];
                int32_t slot = st->r_slot[gid];
                for (int k = 0; k < 3; ++k) {
                    real le = (fl & 0x200u) ? (real)m[3 + k] : RC(0.0);
                    real lr = slot >= 0 ? cache_L(st)[3 * (size_t)slot + k] : RC(0.0);
                    v[k] = le + lr;
                }
            }
            for (int k = 0; k < 3; ++k) sum[cell][k] = sum[cell][k] + v[k];
            sum[cell][3] = sum[cell][3] + st->r_t[gid];
            cnt[cell]++;
        }
        real mean[4];
        uint32_t npop = 0;
        for (int i = 0; i < NCELL; ++i) {
            if (!cnt[i]) continue;
            const real inv = RC(1.0) / (real)cnt[i];
            for (int k = 0; k < 4; ++k) at[4 * i + k] = sum[i][k] * inv;
            ++npop;
        }
        if (npop == 0) continue;
        const real inv = RC(1.0) / (real)npop;
        for (int k = 0; k < 4; ++k) mean[k] = pair_sum64(at + k, 4) * inv;
        for (int i = 0; i < NCELL; ++i)
            if (!cnt[i])
                for (int k = 0; k < 4; ++k) at[4 * i + k] = mean[k];
    }
}

/* ---------------------------------------------------------------------------------------
 * Spherical harmonics (Section 2.4.2): projection of the piecewise-constant atlas onto the
 * real SH basis of bands 0..2, exact per cell through the cell's direction moments rotated
 * into the probe frame; irradiance is the dot product with the projected clamped cosine
 * (Ramamoorthi and Hanrahan 2001: band factors pi, 2pi/3, pi/4).
 * ------------------------------------------------------------------------------------- */
#define SH_C0 0.28209479177387814   /* 1/(2 sqrt(pi)) */
#define SH_C1 0.48860251190291992   /* sqrt(3/(4 pi)) */
#define SH_C2 1.09254843059207907   /* sqrt(15/pi)/2 */
#define SH_C20 0.31539156525252005  /* sqrt(5/pi)/4 */
#define SH_C22 0.54627421529603959  /* sqrt(15/pi)/4 */

/* SH reprojection (Section 2.4.2): a kept probe that traces nothing this frame and keeps the
 * reprojected probe's atlas as it is (no ray guiding, no probe filter) keeps that probe's SH
 * too, so only the other probes are projected.
 * READING: the SH is world-space radiance, so the moved probe keeps it as it was rather than
 * re-projecting the copied cells in its own (slightly turned) frame. */
static int keeps_previous_sh(const state *st, long p)
{
    return st->cfg.temporal && !st->guided && !st->cfg.probe_filter && !st->traced[p] &&
           st->hist[p] != SENTINEL && st->mask[p] != SENTINEL;
}

static void sh_project(state *st)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)st->P; ++p) {
        real *out = st->sh + (size_t)p * 27;
        for (int i = 0; i < 27; ++i) out[i] = RC(0.0);
        if (st->mask[p] == SENTINEL) continue;
        if (keeps_previous_sh(st, p)) {
            memcpy(out, st->prev_sh + (size_t)st->hist[p] * 27, sizeof(real) * 27);
            continue;
        }
        const real *n = st->pnrm + 4 * p;
        real t[3], b[3];
        onb(n, t, b);
        real Rm[3][3];   /* columns t, b, n */
        for (int i = 0; i < 3; ++i) { Rm[i][0] = t[i]; Rm[i][1] = b[i]; Rm[i][2] = n[i]; }
        const real *at = st->atlas + (size_t)p * NCELL * 4;
        for (int cidx = 0; cidx < NCELL; ++cidx) {
            const double *mo = st->mom[cidx];
            real om = (real)mo[0];
            real ml[3] = {(real)mo[1], (real)mo[2], (real)mo[3]};
            real Ml[3][3] = {{(real)mo[4], (real)mo[7], (real)mo[8]},
                             {(real)mo[7], (real)mo[5], (real)mo[9]},
                             {(real)mo[8], (real)mo[9], (real)mo[6]}};
            real mw[3], Mw[3][3];
            for (int i = 0; i < 3; ++i) mw[i] = (Rm[i][0] * ml[0] + Rm[i][1] * ml[1]) + Rm[i][2] * ml[2];
            real tmp[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    tmp[i][j] = (Rm[i][0] * Ml[0][j] + Rm[i][1] * Ml[1][j]) + Rm[i][2] * Ml[2][j];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    Mw[i][j] = (tmp[i][0] * Rm[j][0] + tmp[i][1] * Rm[j][1]) + tmp[i][2] * Rm[j][2];
            real I[9];
            I[0] = (real)SH_C0 * om;
            I[1] = (real)SH_C1 * mw[1];
            I[2] = (real)SH_C1 * mw[2];
            I[3] = (real)SH_C1 * mw[0];
            I[4] = (real)SH_C2 * Mw[0][1];
            I[5] = (real)SH_C2 * Mw[1][2];
            I[6] = (real)SH_C20 * (RC(3.0) * Mw[2][2] - om);
            I[7] = (real)SH_C2 * Mw[0][2];
            I[8] = (real)SH_C22 * (Mw[0][0] - Mw[1][1]);
            for (int l = 0; l < 9; ++l)
                for (int k = 0; k < 3; ++k) out[3 * l + k] = out[3 * l + k] + at[4 * cidx + k] * I[l];
        }
    }
}

static void sh_irradiance(const real *c, const real *n, real *E)
{
    real Y[9];
    Y[0] = (real)SH_C0;
    Y[1] = (real)SH_C1 * n[1];
    Y[2] = (real)SH_C1 * n[2];
    Y[3] = (real)SH_C1 * n[0];
    Y[4] = (real)SH_C2 * (n[0] * n[1]);
    Y[5] = (real)SH_C2 * (n[1] * n[2]);
    Y[6] = (real)SH_C20 * (RC(3.0) * (n[2] * n[2]) - RC(1.0));
    Y[7] = (real)SH_C2 * (n[0] * n[2]);
    Y[8] = (real)SH_C22 * (n[0] * n[0] - n[1] * n[1]);
    const real A[9] = {(real)3.14159265358979324, (real)2.09439510239319549, (real)2.09439510239319549,
                       (real)2.09439510239319549, (real)0.78539816339744831, (real)0.78539816339744831,
                       (real)0.78539816339744831, (real)0.78539816339744831, (real)0.78539816339744831};
    for (int k = 0; k < 3; ++k) {
        real acc = RC(0.0);
        for (int l = 0; l < 9; ++l) acc = acc + (A[l] * c[3 * l + k]) * Y[l];
        E[k] = acc;
    }
}

void ORC(sh_eval)(const real *coef, const real *n, uint32_t cnt, real *E)
{
    for (uint32_t i = 0; i < cnt; ++i) sh_irradiance(coef + 27 * (size_t)i, n + 3 * (size_t)i, E + 3 * (size_t)i);
}

/* project arbitrary atlases [cnt][64][4] with given normals [cnt][3] (test entry) */
void ORC(sh_project_atlas)(state *st, const real *atlas, const real *nrm, uint32_t cnt, real *out)
{
    real *sa = st->atlas, *ss = st->sh, *sn = st->pnrm;
    uint32_t *sm = st->mask;
    uint32_t sp = st->P;
    st->atlas = (real *)atlas;
    st->sh = out;
    st->pnrm = (real *)calloc(4 * (size_t)cnt, sizeof(real));
    st->mask = (uint32_t *)calloc(cnt, sizeof(uint32_t));
    for (uint32_t i = 0; i < cnt; ++i)
        for (int k = 0; k < 3; ++k) st->pnrm[4 * (size_t)i + k] = nrm[3 * (size_t)i + k];
    st->P = cnt;
    sh_project(st);
    free(st->pnrm);
    free(st->mask);
    st->atlas = sa; st->sh = ss; st->pnrm = sn; st->mask = sm; st->P = sp;
}

/* ---------------------------------------------------------------------------------------
 * Algorithm 5: separable 7x7 sparse filter of the probes' radiance in probe space, one pass
 * along x, then one along y.  For every cell of a probe p, the probes found by Algorithm 4
 * at tile steps -1, +1, -2, +2, -3, +3 along the pass axis contribute their cell of the same
 * index, unless the plane distance exceeds p's cell size (Algorithm 6), the cell direction
 * points below their surface, or the hit point their ray reached (at the smaller of the two
 * travelled distances) is seen from p more than pi/50 away from the cell direction.
 * Contributions are depth-weighted; the travelled distance is re-averaged after each one.
 * READING: the test's undefined `direction` is the cell direction; the depth weight, which
 * the paper leaves undefined, is cs / (cs + |d_q - d_p|) with cs p's cell size and d the
 * primary-ray distance; the cell direction is the normalised centre of the hemi-octahedral
 * cell, rotated into the probe frame; a hit point at p itself is rejected.
 * ------------------------------------------------------------------------------------- */
#define COS_PI_50 0.9980267284282716

static uint32_t find_closest_probe(const state *st, int32_t px, int32_t py, int32_t ox, int32_t oy);

static void cell_direction(int cell, const real *n, real *d)
{
    real u = (real)(2 * (cell & 7) + 1) / RC(8.0) - RC(1.0);
    real v = (real)(2 * (cell >> 3) + 1) / RC(8.0) - RC(1.0);
    real a = (u + v) * RC(0.5), b = (u - v) * RC(0.5);
    real z = (RC(1.0) - RABS(a)) - RABS(b);
    real len = RSQRT((a * a + b * b) + z * z);
    real lx = a / len, ly = b / len, lz = z / len;
    real t[3], bb[3];
    onb(n, t, bb);
    for (int k = 0; k < 3; ++k) d[k] = (lx * t[k] + ly * bb[k]) + lz * n[k];
}

static void filter_pass(const state *st, const real *cam, real kappa, int32_t ax, int32_t ay, const real *in,
                        real *out)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)st->P; ++p) {
        const real *ip = in + (size_t)p * NCELL * 4;
        real *op = out + (size_t)p * NCELL * 4;
        if (st->mask[p] == SENTINEL) {
            for (int i = 0; i < NCELL * 4; ++i) op[i] = ip[i];
            continue;
        }
        int32_t px = (int32_t)(st->mask[p] & 0xFFFFu), py = (int32_t)(st->mask[p] >> 16);
        const real *wp = st->ppos + 4 * (size_t)p, *np = st->pnrm + 4 * (size_t)p;
        real cx = wp[0] - cam[0], cy = wp[1] - cam[1], cz = wp[2] - cam[2];
        real cs = kappa * RSQRT((cx * cx + cy * cy) + cz * cz);
        for (int cell = 0; cell < NCELL; ++cell) {
            real dir[3];
            cell_direction(cell, np, dir);
            real rad[4] = {ip[4 * cell], ip[4 * cell + 1], ip[4 * cell + 2], ip[4 * cell + 3]};
            real hit = rad[3], wsum = RC(1.0);
            for (int i = 0; i < 6; ++i) {
                int32_t step = (((i & 1) << 1) - 1) * ((i >> 1) + 1);
                uint32_t qm = find_closest_probe(st, px, py, step * ax, step * ay);
                if (qm == SENTINEL) continue;
                uint32_t q = ((qm >> 16) >> 3) * st->TW + ((qm & 0xFFFFu) >> 3);
                const real *wq = st->ppos + 4 * (size_t)q, *nq = st->pnrm + 4 * (size_t)q;
                real pd = RABS(((wq[0] - wp[0]) * np[0] + (wq[1] - wp[1]) * np[1]) + (wq[2] - wp[2]) * np[2]);
                real nc = (dir[0] * nq[0] + dir[1] * nq[1]) + dir[2] * nq[2];
                if (pd > cs || nc < RC(0.0)) continue;
                const real *rq = in + (size_t)q * NCELL * 4 + 4 * cell;
                real hd = rmin(rq[3], hit);
                real e[3];
                for (int k = 0; k < 3; ++k) e[k] = (wq[k] + dir[k] * hd) - wp[k];
                real el = RSQRT((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]);
                if (!(el > RC(0.0))) continue;
                real ang = (dir[0] * (e[0] / el) + dir[1] * (e[1] / el)) + dir[2] * (e[2] / el);
                if (ang < (real)COS_PI_50) continue;
                real w = cs / (cs + RABS(wq[3] - wp[3]));
                for (int k = 0; k < 3; ++k) rad[k] = rad[k] + w * rq[k];
                rad[3] = rad[3] + w * hd;
                wsum = wsum + w;
                hit = rad[3] / wsum;
            }
            for (int k = 0; k < 4; ++k) op[4 * cell + k] = rad[k] / wsum;
        }
    }
}

/* the filter on caller data (test entry): atlas [P][64][4] in, out; probes as in the state */
void ORC(filter_atlas)(const state *st, const orc_frame *fr, int32_t ax, int32_t ay, const real *in, real *out)
{
    real cam[3] = {(real)fr->pos[0], (real)fr->pos[1], (real)fr->pos[2]};
    real kappa = (real)ORC(distance_scale)(fr->fov_y, st->W, st->H);
    filter_pass(st, cam, kappa, ax, ay, in, out);
}

/* ---------------------------------------------------------------------------------------
 * Radiance blending (Section 2.1.4) with the biased shadow-preserving temporal hysteresis of
 * Algorithm 3: per cell, the luminances l1 (new) and l2 (history) give
 * alpha = clamp(max(l1 - l2 - min(l1, l2), 0) / max(max(l1, l2), 1e-4), 0, 0.95)^2 and the
 * cell becomes lerp(new, history, alpha): a cell brighter than twice its history is held back,
 * a darker one is taken at once.
 * READING: the history is the reprojected probe's final radiance of the previous frame; the
 * travelled distance is blended with the same alpha.
 * ------------------------------------------------------------------------------------- */
static void temporal_blend(state *st)
{
    const real third = RC(1.0) / RC(3.0);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)st->P; ++p) {
        if (st->mask[p] == SENTINEL || !st->traced[p]) continue;
        /* the history: the reprojected probe's atlas, or with ray guiding the reconstruction
         * (its empty cells take the new estimate as it is) */
        if (!st->guided && st->hist[p] == SENTINEL) continue;
        real *at = st->atlas + (size_t)p * NCELL * 4;
        const real *pv = st->guided ? st->recon + (size_t)p * NCELL * 4
                                    : st->prev_atlas + (size_t)st->hist[p] * NCELL * 4;
        for (int cell = 0; cell < NCELL; ++cell) {
            real *c = at + 4 * cell;
            const real *q = pv + 4 * cell;
            if (st->guided && q[3] < RC(0.0)) continue;
            real l1 = (c[0] * third + c[1] * third) + c[2] * third;
            real l2 = (q[0] * third + q[1] * third) + q[2] * third;
            real a = rmax((l1 - l2) - rmin(l1, l2), RC(0.0)) / rmax(rmax(l1, l2), RC(1e-4));
            a = a < RC(0.0) ? RC(0.0) : (a > RC(0.95) ? RC(0.95) : a);
            a = a * a;
            for (int k = 0; k < 4; ++k) c[k] = c[k] + a * (q[k] - c[k]);
        }
    }
}

static void save_history(state *st, const orc_frame *fr)
{
    memcpy(st->prev_mask, st->mask, sizeof(uint32_t) * st->P);
    memcpy(st->prev_pos, st->ppos, sizeof(real) * 4 * st->P);
    memcpy(st->prev_nrm, st->pnrm, sizeof(real) * 4 * st->P);
    memcpy(st->prev_atlas, st->atlas, sizeof(real) * 4 * NCELL * st->P);
    memcpy(st->prev_sh, st->sh, sizeof(real) * 27 * st->P);
    st->prev_fr = *fr;
    st->has_prev = 1;
}

void ORC(temporal_blend_atlas)(const real *curr, const real *prev, uint32_t n, real *out)
{
    /* Algorithm 3 on caller cells [n][4] (test entry) */
    const real third = RC(1.0) / RC(3.0);
    for (uint32_t i = 0; i < n; ++i) {
        const real *c = curr + 4 * (size_t)i, *q = prev + 4 * (size_t)i;
        real l1 = (c[0] * third + c[1] * third) + c[2] * third;
        real l2 = (q[0] * third + q[1] * third) + q[2] * third;
        real a = rmax((l1 - l2) - rmin(l1, l2), RC(0.0)) / rmax(rmax(l1, l2), RC(1e-4));
        a = a < RC(0.0) ? RC(0.0) : (a > RC(0.95) ? RC(0.95) : a);
        a = a * a;
        for (int k = 0; k < 4; ++k) out[4 * (size_t)i + k] = c[k] + a * (q[k] - c[k]);
    }
}

void ORC(guiding_export)(const state *st, real *recon, uint32_t *cdf)
{
    memcpy(recon, st->recon, sizeof(real) * 4 * NCELL * st->P);
    memcpy(cdf, st->cdf, sizeof(uint32_t) * NCELL * st->P);
}

void ORC(temporal_export)(const state *st, uint32_t *win, uint32_t *hist, uint32_t *traced)
{
    memcpy(win, st->win, sizeof(uint32_t) * st->P);
    memcpy(hist, st->hist, sizeof(uint32_t) * st->P);
    memcpy(traced, st->traced, sizeof(uint32_t) * st->P);
}

/* The per-probe half of the update (Sections 2.1.4, 2.1.6, 2.4.2): gather with backup,
 * the temporal blend and probe filter when configured, SH projection.  ORC(update) is the
 * cache update (Sections 2.2.1, 2.2.3) followed by this; the split exists so that the two
 * halves can be timed separately. */
void ORC(probe_pass)(state *st, const orc_frame *fr);

void ORC(update)(state *st, const orc_frame *fr)
{
    cache_update(st);
    ORC(probe_pass)(st, fr);
}

void ORC(probe_pass)(state *st, const orc_frame *fr)
{
    gather(st);
    if (st->cfg.temporal) temporal_blend(st);
    if (st->cfg.probe_filter) {
        real cam[3] = {(real)fr->pos[0], (real)fr->pos[1], (real)fr->pos[2]};
        real kappa = (real)ORC(distance_scale)(fr->fov_y, st->W, st->H);
        real *tmp = (real *)malloc(sizeof(real) * (size_t)st->P * NCELL * 4);
        filter_pass(st, cam, kappa, 1, 0, st->atlas, tmp);
        filter_pass(st, cam, kappa, 0, 1, tmp, st->atlas);
        free(tmp);
    }
    sh_project(st);
    if (st->cfg.temporal) save_history(st, fr);
}

/* ---------------------------------------------------------------------------------------
 * Algorithm 4: sparse directional search through the probe-mask MIP chain.
 * READING: "pixel /= 2" is a floor division (arithmetic shift), so negative lattice
 * positions stay out of bounds.
 * ------------------------------------------------------------------------------------- */
static uint32_t find_closest_probe(const state *st, int32_t px, int32_t py, int32_t ox, int32_t oy)
{
    int32_t x = px >> 3, y = py >> 3;
    for (uint32_t mip = 0; mip < st->nmip; ++mip) {
        int32_t qx = x + ox, qy = y + oy;
        if (qx < 0 || qy < 0 || qx >= (int32_t)st->mip_w[mip] || qy >= (int32_t)st->mip_h[mip]) break;
        uint32_t v = st->mask[st->mip_off[mip] + (uint32_t)qy * st->mip_w[mip] + (uint32_t)qx];
        if (v != SENTINEL) return v;
        x >>= 1;
        y >>= 1;
    }
    return SENTINEL;
}

uint32_t ORC(find_probe)(const state *st, int32_t px, int32_t py, int32_t ox, int32_t oy)
{
    return find_closest_probe(st, px, py, ox, oy);
}

/* ---------------------------------------------------------------------------------------
 * Per-pixel interpolation (Section 2.4.1) with the adaptive cell size of Algorithm 6.
 * READING: the four neighbours are the 2x2 lattice probes around the pixel, each found with
 * Algorithm 4 from its lattice tile; weight = bilinear * [plane distance <= cell size] *
 * max(0, n_p . n_q); if every weight is zero but a probe was found, equal weights (relaxed,
 * flag 1); no probe found: flag 2; sky pixel: flag 3.  Pixel jitter is off.
 * ------------------------------------------------------------------------------------- */
void ORC(interpolate)(state *st, const orc_frame *fr, const real *gpos, const real *gnrm,
                      const uint32_t *gprim, real *out)
{
    real kappa = (real)ORC(distance_scale)(fr->fov_y, st->W, st->H);
    st->kappa = kappa;
    uint64_t relaxed = 0, noprobe = 0;
#pragma omp parallel for schedule(static) reduction(+ : relaxed, noprobe)
    for (long y = 0; y < (long)st->H; ++y) {
        for (uint32_t x = 0; x < st->W; ++x) {
            size_t pix = (size_t)y * st->W + x;
            real *o = out + 4 * pix;
            if (gprim[pix] == MISS) { o[0] = o[1] = o[2] = RC(0.0); o[3] = RC(3.0); continue; }
            const real *pp = gpos + 4 * pix, *pn = gnrm + 4 * pix;
            real dx = pp[0] - (real)fr->pos[0], dy = pp[1] - (real)fr->pos[1], dz = pp[2] - (real)fr->pos[2];
            real cell_size = kappa * RSQRT((dx * dx + dy * dy) + dz * dz);
            int32_t ux = (int32_t)x - (int32_t)st->jx, uy = (int32_t)y - (int32_t)st->jy;
            int32_t bx = ux >> 3, by = uy >> 3;
            real fx = (real)(ux - 8 * bx) * RC(0.125), fy = (real)(uy - 8 * by) * RC(0.125);
            real acc[3] = {RC(0.0), RC(0.0), RC(0.0)}, wsum = RC(0.0);
            real eq[4][3];
            int nfound = 0;
            for (int k = 0; k < 4; ++k) {
                int32_t ox = k & 1, oy = k >> 1;
                uint32_t m = find_closest_probe(st, 8 * bx, 8 * by, ox, oy);
                if (m == SENTINEL) continue;
                uint32_t qx = m & 0xFFFFu, qy = m >> 16;
                uint32_t q = (qy >> 3) * st->TW + (qx >> 3);
                const real *qp = st->ppos + 4 * (size_t)q, *qn = st->pnrm + 4 * (size_t)q;
                real wb = (ox ? fx : RC(1.0) - fx) * (oy ? fy : RC(1.0) - fy);
                real pd = RABS(((qp[0] - pp[0]) * pn[0] + (qp[1] - pp[1]) * pn[1]) + (qp[2] - pp[2]) * pn[2]);
                real nd = (pn[0] * qn[0] + pn[1] * qn[1]) + pn[2] * qn[2];
                real w = (pd <= cell_size) ? wb * rmax(RC(0.0), nd) : RC(0.0);
                real E[3];
                sh_irradiance(st->sh + 27 * (size_t)q, pn, E);
                for (int c = 0; c < 3; ++c) { eq[nfound][c] = E[c]; acc[c] = acc[c] + w * E[c]; }
                wsum = wsum + w;
                ++nfound;
            }
            if (wsum > RC(0.0)) {
                for (int c = 0; c < 3; ++c) o[c] = acc[c] / wsum;
                o[3] = RC(0.0);
            } else if (nfound > 0) {
                for (int c = 0; c < 3; ++c) {
                    real s = RC(0.0);
                    for (int i = 0; i < nfound; ++i) s = s + eq[i][c];
                    o[c] = s / (real)nfound;
                }
                o[3] = RC(1.0);
                ++relaxed;
            } else {
                o[0] = o[1] = o[2] = RC(0.0);
                o[3] = RC(2.0);
                ++noprobe;
            }
        }
    }
    st->stats[ST_RELAXED] = relaxed;
    st->stats[ST_NOPROBE] = noprobe;
}

/* ---------------------------------------------------------------------------------------
 * Screen-space denoiser (Section 2.4.3): temporal accumulation of the interpolated irradiance
 * and a spatial filter whose radius shrinks as the history grows.
 * Temporal: a pixel's world position projected with the previous camera lands on a previous
 * pixel; the history is valid when that pixel was not sky, lies within the pixel's cell size
 * (Algorithm 6) of its tangent plane and has a normal cosine above 0.9.  With a valid history
 * the history length becomes n = min(n_prev + 1, dn_hist_max) and the accumulated value
 * E_hist + (E - E_hist) / n (the running mean over the last n frames, capped); without one,
 * n = 1 and the value is this frame's.  A pixel without a probe (flag 2) keeps its history as
 * it is, or stays empty (n = 0).
 * Spatial: radius r = floor(dn_radius / n) (r = dn_radius at n = 0), dilated to the largest r
 * of the 3x3 neighbourhood (the dilated blur mask); the output is the mean over the (2R+1)^2
 * window of the neighbours' accumulated values that hold one, weighted by cs / (cs + |depth
 * difference|) (cs the pixel's cell size) times max(0, normal cosine)^8.  The history kept is
 * the accumulated value before the spatial filter.
 * READING: every constant above (0.9, the radius law, the weights, the exponent 8) fills a
 * point the paper leaves open; flags pass through in the output's fourth channel.
 * ------------------------------------------------------------------------------------- */
static int project_cam(const orc_frame *pf, uint32_t W, uint32_t H, const real *X, int32_t *qx, int32_t *qy)
{
    real v[3] = {X[0] - (real)pf->pos[0], X[1] - (real)pf->pos[1], X[2] - (real)pf->pos[2]};
    real z = (v[0] * (real)pf->fwd[0] + v[1] * (real)pf->fwd[1]) + v[2] * (real)pf->fwd[2];
    if (!(z > RC(0.0))) return 0;
    real a = ((v[0] * (real)pf->right[0] + v[1] * (real)pf->right[1]) + v[2] * (real)pf->right[2]) / z;
    real b = ((v[0] * (real)pf->up[0] + v[1] * (real)pf->up[1]) + v[2] * (real)pf->up[2]) / z;
    real aspect = (real)W / (real)H;
    real sx = a / ((real)pf->tan_half * aspect), sy = b / (real)pf->tan_half;
    real fx = ((sx + RC(1.0)) * (real)W) * RC(0.5), fy = ((RC(1.0) - sy) * (real)H) * RC(0.5);
    if (!(fx >= RC(0.0) && fx < (real)W && fy >= RC(0.0) && fy < (real)H)) return 0;
    *qx = (int32_t)fx;
    *qy = (int32_t)fy;
    return 1;
}

void ORC(denoise)(state *st, const orc_frame *fr, const real *gpos, const real *gnrm, const uint32_t *gprim,
                  const real *in, real *out)
{
    const orc_config *c = &st->cfg;
    const uint32_t W = st->W, H = st->H, NM = c->dn_hist_max, RM = c->dn_radius;
    real kappa = (real)ORC(distance_scale)(fr->fov_y, W, H);
    real *acc = st->dn_acc;
#pragma omp parallel for schedule(static)
    for (long y = 0; y < (long)H; ++y)
        for (uint32_t x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            real *a = acc + 4 * p;
            a[0] = a[1] = a[2] = a[3] = RC(0.0);
            if (gprim[p] == MISS) continue;
            const real *X = gpos + 4 * p, *n = gnrm + 4 * p, *E = in + 4 * p;
            int hv = 0;
            size_t q = 0;
            int32_t qx, qy;
            if (st->dn_has_prev && project_cam(&st->dn_pfr, W, H, X, &qx, &qy)) {
                q = (size_t)qy * W + (size_t)qx;
                if (st->dn_pprim[q] != MISS && st->dn_hist[4 * q + 3] > RC(0.0)) {
                    const real *Xq = st->dn_ppos + 4 * q, *nq = st->dn_pnrm + 4 * q;
                    real ex = X[0] - (real)fr->pos[0], ey = X[1] - (real)fr->pos[1], ez = X[2] - (real)fr->pos[2];
                    real cs = kappa * RSQRT((ex * ex + ey * ey) + ez * ez);
                    real pd = RABS(((Xq[0] - X[0]) * n[0] + (Xq[1] - X[1]) * n[1]) + (Xq[2] - X[2]) * n[2]);
                    real nc = (nq[0] * n[0] + nq[1] * n[1]) + nq[2] * n[2];
                    hv = pd < cs && nc > RC(0.9);
                }
            }
            const real *Hh = st->dn_hist + 4 * q;
            if (E[3] == RC(2.0)) {
                if (hv)
                    for (int k = 0; k < 4; ++k) a[k] = Hh[k];
                continue;
            }
            if (hv) {
                real np = Hh[3] + RC(1.0);
                real nn = np < (real)NM ? np : (real)NM;
                for (int k = 0; k < 3; ++k) a[k] = Hh[k] + (E[k] - Hh[k]) / nn;
                a[3] = nn;
            } else {
                for (int k = 0; k < 3; ++k) a[k] = E[k];
                a[3] = RC(1.0);
            }
        }
    /* radius per pixel, then the dilated mask inside the filter */
    uint32_t *rad = st->dn_rad;
    for (size_t p = 0; p < (size_t)W * H; ++p) {
        uint32_t n = (uint32_t)acc[4 * p + 3];
        rad[p] = gprim[p] == MISS ? 0u : (n == 0 ? RM : RM / n);
    }
#pragma omp parallel for schedule(static)
    for (long y = 0; y < (long)H; ++y)
        for (uint32_t x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            real *o = out + 4 * p;
            o[3] = in[4 * p + 3];
            if (gprim[p] == MISS) { o[0] = o[1] = o[2] = RC(0.0); continue; }
            uint32_t R = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    long yy = y + dy, xx = (long)x + dx;
                    if (yy < 0 || xx < 0 || yy >= (long)H || xx >= (long)W) continue;
                    uint32_t r = rad[(size_t)yy * W + (size_t)xx];
                    R = r > R ? r : R;
                }
            const real *a = acc + 4 * p;
            if (R == 0) { o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; continue; }
            const real *X = gpos + 4 * p, *n = gnrm + 4 * p;
            real ex = X[0] - (real)fr->pos[0], ey = X[1] - (real)fr->pos[1], ez = X[2] - (real)fr->pos[2];
            real cs = kappa * RSQRT((ex * ex + ey * ey) + ez * ez);
            real s[3] = {RC(0.0), RC(0.0), RC(0.0)}, ws = RC(0.0);
            for (int dy = -(int)R; dy <= (int)R; ++dy)
                for (int dx = -(int)R; dx <= (int)R; ++dx) {
                    long yy = y + dy, xx = (long)x + dx;
                    if (yy < 0 || xx < 0 || yy >= (long)H || xx >= (long)W) continue;
                    size_t q = (size_t)yy * W + (size_t)xx;
                    if (gprim[q] == MISS || acc[4 * q + 3] == RC(0.0)) continue;
                    const real *nq = gnrm + 4 * q;
                    real nd = (n[0] * nq[0] + n[1] * nq[1]) + n[2] * nq[2];
                    nd = rmax(nd, RC(0.0));
                    real n2 = nd * nd, n4 = n2 * n2, n8 = n4 * n4;
                    real w = (cs / (cs + RABS(gpos[4 * q + 3] - X[3]))) * n8;
                    for (int k = 0; k < 3; ++k) s[k] = s[k] + w * acc[4 * q + k];
                    ws = ws + w;
                }
            for (int k = 0; k < 3; ++k) o[k] = ws > RC(0.0) ? s[k] / ws : a[k];
        }
    /* the accumulated values become the history */
    memcpy(st->dn_hist, acc, sizeof(real) * 4 * (size_t)W * H);
    memcpy(st->dn_ppos, gpos, sizeof(real) * 4 * (size_t)W * H);
    memcpy(st->dn_pnrm, gnrm, sizeof(real) * 4 * (size_t)W * H);
    memcpy(st->dn_pprim, gprim, sizeof(uint32_t) * (size_t)W * H);
    st->dn_pfr = *fr;
    st->dn_has_prev = 1;
}

void ORC(denoise_export)(const state *st, real *hist, uint32_t *rad)
{
    size_t HW = (size_t)st->W * st->H;
    memcpy(hist, st->dn_hist, sizeof(real) * 4 * HW);
    memcpy(rad, st->dn_rad, sizeof(uint32_t) * HW);
}

/* lookup-only query of the world cache for caller points (pos.w >= 0 is the ray length for
 * the leak bit); result rgb and a = 1 if the cell exists */
void ORC(query)(const state *st, const real *pos, const real *nrm, uint32_t n, real *out)
{
    for (uint32_t i = 0; i < n; ++i) {
        const real *p = pos + 4 * (size_t)i, *nn = nrm + 4 * (size_t)i;
        int with_leak = p[3] >= RC(0.0);
        uint32_t tc;
        uint64_t key = cell_key_cell(&st->cfg, st->cam, p, nn, with_leak ? p[3] : RC(0.0), with_leak, &tc);
        int32_t slot = cache_entry(st, table_find(st, key), tc);
        for (int k = 0; k < 3; ++k) out[4 * (size_t)i + k] = slot >= 0 ? cache_L(st)[3 * (size_t)slot + k] : RC(0.0);
        out[4 * (size_t)i + 3] = slot >= 0 ? RC(1.0) : RC(0.0);
    }
}

/* ---------------------------------------------------------------------------------------
 * Exports for comparison
 * ------------------------------------------------------------------------------------- */
void ORC(dims)(const state *st, uint32_t *out /* P, R, N, TW, TH, nmip, mask_total, jx, jy */)
{
    out[0] = st->P; out[1] = st->R; out[2] = st->N; out[3] = st->TW; out[4] = st->TH;
    out[5] = st->nmip; out[6] = st->mask_total; out[7] = st->jx; out[8] = st->jy;
}

void ORC(export_probes)(const state *st, uint32_t *mask, real *ppos, real *pnrm, real *atlas, real *sh)
{
    if (mask) memcpy(mask, st->mask, sizeof(uint32_t) * st->mask_total);
    if (ppos) memcpy(ppos, st->ppos, sizeof(real) * 4 * st->P);
    if (pnrm) memcpy(pnrm, st->pnrm, sizeof(real) * 4 * st->P);
    if (atlas) memcpy(atlas, st->atlas, sizeof(real) * (size_t)st->P * NCELL * 4);
    if (sh) memcpy(sh, st->sh, sizeof(real) * (size_t)st->P * 27);
}

void ORC(export_rays)(const state *st, int32_t *slot, real *t, uint32_t *tri, uint32_t *cell,
                      uint64_t *key, real *sample)
{
    size_t PR = (size_t)st->P * st->R;
    if (slot) memcpy(slot, st->r_slot, sizeof(int32_t) * PR);
    if (t) memcpy(t, st->r_t, sizeof(real) * PR);
    if (tri) memcpy(tri, st->r_tri, sizeof(uint32_t) * PR);
    if (cell) memcpy(cell, st->r_cell, sizeof(uint32_t) * PR);
    if (key)
        for (size_t i = 0; i < PR; ++i) key[i] = (uint64_t)st->r_keylo[i] | ((uint64_t)st->r_keyhi[i] << 32);
    if (sample) memcpy(sample, st->r_sample, sizeof(real) * 3 * PR);
}

/* hit point and face-forwarded normal of every probe ray's hit, [P*R][3] each (meaningful
 * where the ray's flags hold the hit bit) */
void ORC(export_hits)(const state *st, real *y, real *ny)
{
    size_t PR = (size_t)st->P * st->R;
    if (y) memcpy(y, st->r_y, sizeof(real) * 3 * PR);
    if (ny) memcpy(ny, st->r_ny, sizeof(real) * 3 * PR);
}

/* live cells in slot order: bucket*2^32|fp, key, acc[4], L[3], nhist, life; returns count */
uint32_t ORC(export_table)(const state *st, uint64_t *id, uint64_t *key, uint32_t *acc, real *L,
                           uint32_t *nhist, uint32_t *life, uint32_t cap)
{
    uint32_t n = 0;
    for (uint32_t s = 0; s < st->N; ++s) {
        if (st->fp[s] == 0u) continue;
        if (n < cap) {
            id[n] = ((uint64_t)(s / BUCKET) << 32) | st->fp[s];
            key[n] = st->key[s];
            for (int k = 0; k < 4; ++k) acc[4 * (size_t)n + k] = st->acc[4 * (size_t)s + k];
            for (int k = 0; k < 3; ++k) L[3 * (size_t)n + k] = st->L[3 * (size_t)s + k];
            nhist[n] = st->nhist[s];
            life[n] = st->life[s];
        }
        ++n;
    }
    return n;
}

/* live tiles in slot order: bucket*2^32|fp, key, life, and per cell acc[4], L[3], nhist and
 * the query radiance Lq[3]; returns count */
uint32_t ORC(export_tiles)(const state *st, uint64_t *id, uint64_t *key, uint32_t *life, uint32_t *acc, real *L,
                           uint32_t *nhist, real *Lq, uint32_t cap)
{
    uint32_t n = 0;
    if (!st->cfg.cache_tiles) return 0;
    for (uint32_t s = 0; s < st->N; ++s) {
        if (st->fp[s] == 0u) continue;
        if (n < cap) {
            id[n] = ((uint64_t)(s / BUCKET) << 32) | st->fp[s];
            key[n] = st->key[s];
            life[n] = st->life[s];
            for (int i = 0; i < NCELL; ++i) {
                size_t e = (size_t)s * NCELL + (size_t)i, o = (size_t)n * NCELL + (size_t)i;
                for (int k = 0; k < 4; ++k) acc[4 * o + k] = st->acc[4 * e + k];
                for (int k = 0; k < 3; ++k) L[3 * o + k] = st->L[3 * e + k];
                for (int k = 0; k < 3; ++k) Lq[3 * o + k] = st->Lq[3 * e + k];
                nhist[o] = st->nhist[e];
            }
        }
        ++n;
    }
    return n;
}

/* keys and in-tile cells of caller hits (test entry) */
void ORC(tile_keys)(const orc_config *c, const real *cam, const real *y, const real *n, const real *t, uint32_t cnt,
                    uint64_t *keys, uint32_t *cells)
{
    for (uint32_t i = 0; i < cnt; ++i)
        keys[i] = cell_key_cell(c, cam, y + 3 * (size_t)i, n + 3 * (size_t)i, t[i], 1, &cells[i]);
}

/* write a cell directly (tests of update / gather rules) */
int ORC(poke_cell)(state *st, uint64_t key, const uint32_t *acc4, const real *L3, uint32_t nhist,
                   uint32_t life, uint32_t accessed)
{
    int32_t slot = table_insert(st, key);
    if (slot < 0) return -1;
    for (int k = 0; k < 4; ++k) st->acc[4 * (size_t)slot + k] = acc4[k];
    for (int k = 0; k < 3; ++k) st->L[3 * (size_t)slot + k] = L3[k];
    st->nhist[slot] = nhist;
    st->life[slot] = life;
    st->accessed[slot] = accessed;
    return slot;
}

void ORC(cache_update_only)(state *st) { cache_update(st); }

void ORC(stats)(const state *st, uint64_t *out) { memcpy(out, st->stats, sizeof(st->stats)); }

real ORC(kappa)(const state *st) { return st->kappa; }
