/*
 * FP64 CPU oracle for keyframe fusion and the voxel-hashed projective TSDF.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP path: both implement the same written conventions
 * independently, and this file favours the plain definition over speed.
 *
 * Paper: Maier, Schaller, Cremers, "Efficient Online Surface Correction for
 * Real-time Large-Scale 3D Reconstruction" (arXiv 1709.03763).
 *
 * Continuous quantities are FP64.  Every discrete decision (validity, pixel
 * choice, band membership, quantised weights) is taken in FP32 with the
 * written operation order below and no FMA contraction (build with
 * -ffp-contract=off), exactly as the GPU takes it, so that both sides decide
 * identically.  Accumulations that feed a later decision are exact integers.
 *
 * Conventions
 *   pose T = (R, t) maps camera to world, g(T,p) = R p + t   (Sec. 3, Prelim.)
 *   pinhole: u = fx X / Z + cx, pixel centres at integers       (Sec. 3)
 *   voxel n in Z^3 has centre s*n; block b = floor(n / 8)       (Sec. 3, SDF)
 *   quantised weight q(w) = rint(w * 2^10) / 2^10
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    OV_OK = 0,
    OV_EINVAL = -1,
    OV_ENOMEM = -2,
    OV_ENOTALLOC = -5,
    OV_EWEIGHT = -6,
};

#define BSZ 8
#define BVOX 512
#define WQ_SCALE 1024.0f /* 2^10 */
#define W_LIMIT 16384.0   /* 2^14: weights stay exact in FP32 below this */

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

static int64_t floor_div8(int64_t a) { return (a >= 0) ? a / 8 : -((-a + 7) / 8); }

static uint64_t mix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static uint64_t pack_key(int64_t x, int64_t y, int64_t z)
{
    return ((uint64_t)(x & 0x1FFFFF) << 42) | ((uint64_t)(y & 0x1FFFFF) << 21) | (uint64_t)(z & 0x1FFFFF);
}

/* a growable open-addressing map from 64-bit keys to int64 values */
typedef struct {
    int64_t cap;
    int64_t n;
    uint64_t* keys;
    int64_t* vals;
} omap;

#define OMAP_EMPTY 0xFFFFFFFFFFFFFFFFull

static int omap_init(omap* m, int64_t cap)
{
    m->cap = 16;
    while (m->cap < cap) m->cap <<= 1;
    m->n = 0;
    m->keys = (uint64_t*)malloc(sizeof(uint64_t) * m->cap);
    m->vals = (int64_t*)malloc(sizeof(int64_t) * m->cap);
    if (!m->keys || !m->vals) return OV_ENOMEM;
    memset(m->keys, 0xFF, sizeof(uint64_t) * m->cap);
    return OV_OK;
}

static void omap_free(omap* m)
{
    free(m->keys);
    free(m->vals);
    m->keys = NULL;
    m->vals = NULL;
}

static int64_t omap_get(const omap* m, uint64_t key)
{
    int64_t h = (int64_t)(mix64(key) & (uint64_t)(m->cap - 1));
    for (;;) {
        if (m->keys[h] == key) return m->vals[h];
        if (m->keys[h] == OMAP_EMPTY) return -1;
        h = (h + 1) & (m->cap - 1);
    }
}

static int omap_put(omap* m, uint64_t key, int64_t val);

static int omap_grow(omap* m)
{
    omap g;
    if (omap_init(&g, m->cap * 2) != OV_OK) return OV_ENOMEM;
    for (int64_t i = 0; i < m->cap; ++i)
        if (m->keys[i] != OMAP_EMPTY) omap_put(&g, m->keys[i], m->vals[i]);
    omap_free(m);
    *m = g;
    return OV_OK;
}

/* inserts if absent; returns 1 if inserted, 0 if present */
static int omap_put(omap* m, uint64_t key, int64_t val)
{
    if (2 * (m->n + 1) > m->cap)
        if (omap_grow(m) != OV_OK) return OV_ENOMEM;
    int64_t h = (int64_t)(mix64(key) & (uint64_t)(m->cap - 1));
    for (;;) {
        if (m->keys[h] == key) return 0;
        if (m->keys[h] == OMAP_EMPTY) {
            m->keys[h] = key;
            m->vals[h] = val;
            m->n++;
            return 1;
        }
        h = (h + 1) & (m->cap - 1);
    }
}

/* ------------------------------------------------------------------------- */
/* volume                                                                    */
/* ------------------------------------------------------------------------- */

typedef struct {
    float s;       /* voxel size, metres */
    float mu;      /* truncation, metres */
    int color_f32; /* 0: colour stored as uint8 per channel, 1: FP64 in [0,1] */
    omap map;      /* block key -> block index */
    int64_t n, cap;
    int64_t* bxyz; /* n x 3 block coordinates */
    double* D;     /* n x 512 */
    double* W;     /* n x 512 */
    double* C;     /* n x 512 x 3 */
} ovol;

ovol* ov_create(float voxel_size, float trunc, int color_f32)
{
    ovol* v = (ovol*)calloc(1, sizeof(ovol));
    if (!v) return NULL;
    v->s = voxel_size;
    v->mu = trunc;
    v->color_f32 = color_f32;
    if (omap_init(&v->map, 1024) != OV_OK) return NULL;
    return v;
}

void ov_destroy(ovol* v)
{
    if (!v) return;
    omap_free(&v->map);
    free(v->bxyz);
    free(v->D);
    free(v->W);
    free(v->C);
    free(v);
}

int64_t ov_n_blocks(const ovol* v) { return v->n; }

static int64_t ov_alloc_block(ovol* v, int64_t bx, int64_t by, int64_t bz)
{
    uint64_t key = pack_key(bx, by, bz);
    int64_t idx = omap_get(&v->map, key);
    if (idx >= 0) return idx;
    if (v->n == v->cap) {
        int64_t nc = v->cap ? v->cap * 2 : 256;
        v->bxyz = (int64_t*)realloc(v->bxyz, sizeof(int64_t) * 3 * nc);
        v->D = (double*)realloc(v->D, sizeof(double) * BVOX * nc);
        v->W = (double*)realloc(v->W, sizeof(double) * BVOX * nc);
        v->C = (double*)realloc(v->C, sizeof(double) * BVOX * 3 * nc);
        if (!v->bxyz || !v->D || !v->W || !v->C) return -1;
        v->cap = nc;
    }
    idx = v->n++;
    v->bxyz[3 * idx + 0] = bx;
    v->bxyz[3 * idx + 1] = by;
    v->bxyz[3 * idx + 2] = bz;
    memset(v->D + BVOX * idx, 0, sizeof(double) * BVOX);
    memset(v->W + BVOX * idx, 0, sizeof(double) * BVOX);
    memset(v->C + BVOX * 3 * idx, 0, sizeof(double) * BVOX * 3);
    omap_put(&v->map, key, idx);
    return idx;
}

/* ------------------------------------------------------------------------- */
/* one keyframe at one pose                                                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    /* keyframe (Sec. 4.1: fused depth Z*, fusion weight W*, colour C*) */
    const float* Z;
    const float* Wk;
    const uint8_t* rgba; /* H x W x 4, used when colour is uint8 */
    const float* rgbf;   /* H x W x 3 in [0,1], used when colour is FP32 */
    int W, H;
    float fx, fy, cx, cy;
    /* integration pose, camera -> world */
    double R[9], t[3];
    /* derived per-call constants (decision convention) */
    float a[3][3]; /* a[c][r] = fl32(s * R[c][r]): camera-frame step of one voxel along world axis c */
} oop;

static void oop_setup(oop* P, const ovol* v)
{
    double s = (double)v->s;
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) P->a[c][r] = (float)(s * P->R[3 * c + r]);
}

/* Camera point of voxel n under the decision convention: the block origin is
 * mapped in FP64 and rounded once to FP32, then the in-block offset is added
 * in FP32 along x, then y, then z.  This is p = R^T (s n - t) (inverse of the
 * camera->world map g, Sec. 3), evaluated in a fixed order. */
static void cam_point_f32(const ovol* v, const oop* P, const int64_t n[3], float p[3])
{
    int64_t b[3], k[3];
    for (int c = 0; c < 3; ++c) {
        b[c] = floor_div8(n[c]);
        k[c] = n[c] - 8 * b[c];
    }
    double s8 = 8.0 * (double)v->s;
    double o[3] = {s8 * (double)b[0], s8 * (double)b[1], s8 * (double)b[2]};
    double e[3] = {o[0] - P->t[0], o[1] - P->t[1], o[2] - P->t[2]};
    for (int r = 0; r < 3; ++r) {
        /* row r of R^T is column r of R */
        double q = (P->R[0 * 3 + r] * e[0] + P->R[1 * 3 + r] * e[1]) + P->R[2 * 3 + r] * e[2];
        float qf = (float)q;
        float acc = qf + (float)k[0] * P->a[0][r];
        acc = acc + (float)k[1] * P->a[1][r];
        acc = acc + (float)k[2] * P->a[2][r];
        p[r] = acc;
    }
}

/* Camera z of the voxel centre in FP64 (the continuous value). */
static void cam_point_f64(const ovol* v, const oop* P, const int64_t n[3], double p[3])
{
    double s = (double)v->s;
    double e[3] = {s * (double)n[0] - P->t[0], s * (double)n[1] - P->t[1], s * (double)n[2] - P->t[2]};
    for (int r = 0; r < 3; ++r) p[r] = (P->R[0 * 3 + r] * e[0] + P->R[1 * 3 + r] * e[1]) + P->R[2 * 3 + r] * e[2];
}

/* Nearest pixel of pi(p) (Sec. 3): u = (fx X)/Z + cx, iu = floor(u + 1/2). */
static int nearest_pixel(const oop* P, const float p[3], int* iu, int* iv)
{
    if (!(p[2] > 0.0f)) return 0;
    float u = (P->fx * p[0]) / p[2] + P->cx;
    float w = (P->fy * p[1]) / p[2] + P->cy;
    float fu = floorf(u + 0.5f);
    float fv = floorf(w + 0.5f);
    if (!(fu >= 0.0f && fu <= (float)(P->W - 1))) return 0;
    if (!(fv >= 0.0f && fv <= (float)(P->H - 1))) return 0;
    *iu = (int)fu;
    *iv = (int)fv;
    return 1;
}

static float qweight(float w) { return rintf(w * WQ_SCALE) / WQ_SCALE; }

typedef struct {
    int pix;    /* keyframe pixel index */
    float w;    /* quantised sampling weight */
    double d;   /* projective signed distance, FP64 (Sec. 4.3: along z) */
    double c[3];
    float pf[3]; /* FP32 camera point (decision convention) */
} touch_t;

/* The touched test of voxel n by (keyframe, pose): in front of the camera,
 * nearest pixel in bounds, positive keyframe weight, and |Z*(x) - p_z| <= mu
 * (projective distance along the z axis, Sec. 4.3). */
static int touch(const ovol* v, const oop* P, const int64_t n[3], touch_t* out)
{
    float p[3];
    cam_point_f32(v, P, n, p);
    int iu, iv;
    if (!nearest_pixel(P, p, &iu, &iv)) return 0;
    int pix = iv * P->W + iu;
    float w = qweight(P->Wk[pix]);
    if (!(w > 0.0f)) return 0;
    float z = P->Z[pix];
    float d32 = z - p[2];
    if (!(fabsf(d32) <= v->mu)) return 0;
    if (out) {
        double p64[3];
        cam_point_f64(v, P, n, p64);
        out->pix = pix;
        out->w = w;
        out->d = (double)z - p64[2];
        for (int c = 0; c < 3; ++c) {
            if (v->color_f32 && P->rgbf)
                out->c[c] = (double)P->rgbf[3 * pix + c];
            else if (!v->color_f32 && P->rgba)
                out->c[c] = (double)P->rgba[4 * pix + c];
            else
                out->c[c] = 0.0;
        }
        out->pf[0] = p[0];
        out->pf[1] = p[1];
        out->pf[2] = p[2];
    }
    return 1;
}

/* round-half-to-even of the exact rational N / M, M > 0, N >= 0 */
static int64_t rne_div(int64_t N, int64_t M)
{
    int64_t q = N / M, r = N % M;
    if (2 * r > M) return q + 1;
    if (2 * r == M) return q + (q & 1);
    return q;
}

/* Running weighted average (Sec. 3, SDF volume) for sign = +1 and its exact
 * reversal, Eq. (2), for sign = -1.  Colour stored as uint8 is rounded to the
 * nearest integer (ties to even) after every update, from the exact rational
 * (C W + c w) / W' on the 2^-10 weight grid, and clamped to [0, 255]. */
static int update_voxel(ovol* v, int64_t bi, int k, const touch_t* T, int sign)
{
    double* D = v->D + BVOX * bi + k;
    double* W = v->W + BVOX * bi + k;
    double* C = v->C + (BVOX * bi + k) * 3;
    double w = (double)T->w;
    double W0 = *W;
    double W1 = (sign > 0) ? W0 + w : W0 - w;
    if (sign > 0 && W1 >= W_LIMIT) return OV_EWEIGHT;
    if (sign < 0 && W1 < 0.0) return OV_EWEIGHT;
    if (W1 == 0.0) {
        *D = 0.0;
        *W = 0.0;
        C[0] = C[1] = C[2] = 0.0;
        return OV_OK;
    }
    if (sign > 0) {
        *D = (*D * W0 + T->d * w) / W1;
    } else {
        *D = (*D * W0 - T->d * w) / W1;
    }
    if (v->color_f32) {
        for (int c = 0; c < 3; ++c)
            C[c] = (sign > 0) ? (C[c] * W0 + T->c[c] * w) / W1 : (C[c] * W0 - T->c[c] * w) / W1;
    } else {
        int64_t Wq = llrint(W0 * 1024.0), wq = llrint(w * 1024.0), W1q = llrint(W1 * 1024.0);
        for (int c = 0; c < 3; ++c) {
            int64_t N = (int64_t)C[c] * Wq + (int64_t)sign * (int64_t)T->c[c] * wq;
            int64_t val = (N <= 0) ? 0 : rne_div(N, W1q);
            if (val > 255) val = 255;
            C[c] = (double)val;
        }
    }
    *W = W1;
    return OV_OK;
}

/* ---- enumeration of candidate blocks ---------------------------------- */

/* Conservative block range of one keyframe pixel: the world AABB of its
 * frustum cell (u +- 1/2, v +- 1/2) between depths Z* - mu and Z* + mu,
 * padded so that FP32 rounding in the decision convention cannot escape it. */
static void pixel_block_range(const ovol* v, const oop* P, int u, int w, float z, int64_t lo[3], int64_t hi[3])
{
    double mu = (double)v->mu;
    double zl = (double)z - mu - 1e-3, zh = (double)z + mu + 1e-3;
    if (zl < 0.0) zl = 0.0;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int cu = 0; cu < 2; ++cu)
        for (int cv = 0; cv < 2; ++cv)
            for (int cz = 0; cz < 2; ++cz) {
                double uu = (double)u + (cu ? 0.55 : -0.55);
                double vv = (double)w + (cv ? 0.55 : -0.55);
                double zz = cz ? zh : zl;
                double pc[3] = {(uu - (double)P->cx) * zz / (double)P->fx, (vv - (double)P->cy) * zz / (double)P->fy, zz};
                for (int r = 0; r < 3; ++r) {
                    double x = P->R[3 * r + 0] * pc[0] + P->R[3 * r + 1] * pc[1] + P->R[3 * r + 2] * pc[2] + P->t[r];
                    if (x < mn[r]) mn[r] = x;
                    if (x > mx[r]) mx[r] = x;
                }
            }
    double s = (double)v->s;
    for (int r = 0; r < 3; ++r) {
        double pad = 1e-3 + 1e-6 * fabs(mn[r]);
        int64_t nlo = (int64_t)ceil((mn[r] - pad) / s);
        int64_t nhi = (int64_t)floor((mx[r] + pad) / s);
        lo[r] = floor_div8(nlo);
        hi[r] = floor_div8(nhi);
    }
}

typedef struct {
    int64_t n;
    int64_t cap;
    int64_t* b; /* n x 3 */
} blist;

static int blist_push(blist* L, int64_t x, int64_t y, int64_t z)
{
    if (L->n == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 1024;
        int64_t* nb = (int64_t*)realloc(L->b, sizeof(int64_t) * 3 * nc);
        if (!nb) return OV_ENOMEM;
        L->b = nb;
        L->cap = nc;
    }
    L->b[3 * L->n + 0] = x;
    L->b[3 * L->n + 1] = y;
    L->b[3 * L->n + 2] = z;
    L->n++;
    return OV_OK;
}

/* sparse enumeration: union of the per-pixel conservative block ranges */
static int candidates_sparse(const ovol* v, const oop* P, blist* out)
{
    omap seen;
    if (omap_init(&seen, 4096) != OV_OK) return OV_ENOMEM;
    for (int iv = 0; iv < P->H; ++iv)
        for (int iu = 0; iu < P->W; ++iu) {
            int pix = iv * P->W + iu;
            if (!(qweight(P->Wk[pix]) > 0.0f)) continue;
            float z = P->Z[pix];
            if (!(z > 0.0f) || !isfinite(z)) continue;
            int64_t lo[3], hi[3];
            pixel_block_range(v, P, iu, iv, z, lo, hi);
            for (int64_t bx = lo[0]; bx <= hi[0]; ++bx)
                for (int64_t by = lo[1]; by <= hi[1]; ++by)
                    for (int64_t bz = lo[2]; bz <= hi[2]; ++bz)
                        if (omap_put(&seen, pack_key(bx, by, bz), 0) == 1)
                            if (blist_push(out, bx, by, bz) != OV_OK) {
                                omap_free(&seen);
                                return OV_ENOMEM;
                            }
        }
    omap_free(&seen);
    return OV_OK;
}

/* brute force: every block of an explicit box of block coordinates */
static int candidates_box(const int64_t blo[3], const int64_t bhi[3], blist* out)
{
    for (int64_t bx = blo[0]; bx <= bhi[0]; ++bx)
        for (int64_t by = blo[1]; by <= bhi[1]; ++by)
            for (int64_t bz = blo[2]; bz <= bhi[2]; ++bz)
                if (blist_push(out, bx, by, bz) != OV_OK) return OV_ENOMEM;
    return OV_OK;
}

static void voxel_of(const int64_t* b, int k, int64_t n[3])
{
    n[0] = 8 * b[0] + (k & 7);
    n[1] = 8 * b[1] + ((k >> 3) & 7);
    n[2] = 8 * b[2] + (k >> 6);
}

/*
 * Integrate (sign = +1) or de-integrate (sign = -1, Eq. 2) one keyframe at a
 * pose.  Integration allocates every block with at least one touched voxel
 * before updating (Sec. 3, SDF volume); de-integration never allocates and
 * reports OV_ENOTALLOC if a touched voxel lies in an unallocated block.
 * If box_lo/box_hi are non-NULL every block in that box is tested (brute
 * force); otherwise the sparse per-pixel candidate set is used.
 */
int ov_op(ovol* v, const float* Z, const float* Wk, const uint8_t* rgba, const float* rgbf, int W, int H,
          const float* intr, const double* R, const double* t, int sign, const int64_t* box_lo,
          const int64_t* box_hi)
{
    if (!v || !Z || !Wk || W <= 0 || H <= 0 || (sign != 1 && sign != -1)) return OV_EINVAL;
    if (v->color_f32 ? !rgbf : !rgba) return OV_EINVAL;
    oop P;
    memset(&P, 0, sizeof(P));
    P.Z = Z;
    P.Wk = Wk;
    P.rgba = rgba;
    P.rgbf = rgbf;
    P.W = W;
    P.H = H;
    P.fx = intr[0];
    P.fy = intr[1];
    P.cx = intr[2];
    P.cy = intr[3];
    memcpy(P.R, R, sizeof(P.R));
    memcpy(P.t, t, sizeof(P.t));
    oop_setup(&P, v);

    blist L = {0, 0, NULL};
    int rc = (box_lo && box_hi) ? candidates_box(box_lo, box_hi, &L) : candidates_sparse(v, &P, &L);
    if (rc != OV_OK) {
        free(L.b);
        return rc;
    }
    /* pass 1: which candidate blocks hold a touched voxel */
    char* hit = (char*)calloc((size_t)(L.n ? L.n : 1), 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < L.n; ++i) {
        for (int k = 0; k < BVOX; ++k) {
            int64_t n[3];
            voxel_of(L.b + 3 * i, k, n);
            if (touch(v, &P, n, NULL)) {
                hit[i] = 1;
                break;
            }
        }
    }
    /* pass 2: allocation (integration) or existence check (de-integration) */
    int64_t* bidx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L.n ? L.n : 1));
    int err = OV_OK;
    for (int64_t i = 0; i < L.n; ++i) {
        bidx[i] = -1;
        if (!hit[i]) continue;
        int64_t* b = L.b + 3 * i;
        if (sign > 0) {
            bidx[i] = ov_alloc_block(v, b[0], b[1], b[2]);
            if (bidx[i] < 0) err = OV_ENOMEM;
        } else {
            bidx[i] = omap_get(&v->map, pack_key(b[0], b[1], b[2]));
            if (bidx[i] < 0) err = OV_ENOTALLOC;
        }
    }
    /* pass 3: per-voxel update; voxels are independent within one keyframe */
    int uerr = OV_OK;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < L.n; ++i) {
        if (bidx[i] < 0) continue;
        for (int k = 0; k < BVOX; ++k) {
            int64_t n[3];
            touch_t T;
            voxel_of(L.b + 3 * i, k, n);
            if (!touch(v, &P, n, &T)) continue;
            int e = update_voxel(v, bidx[i], k, &T, sign);
            if (e != OV_OK) {
#pragma omp critical
                uerr = e;
            }
        }
    }
    free(hit);
    free(bidx);
    free(L.b);
    if (err != OV_OK) return err;
    return uerr;
}

/* Touched voxels of one keyframe at one pose, without changing the volume.
 * Writes up to `cap` records: voxel coordinates n (x,y,z), pixel index,
 * quantised weight, FP64 signed distance and the FP32 camera point.  Returns
 * the total count (which may exceed cap), or a negative error. */
int64_t ov_record(const ovol* v, const float* Z, const float* Wk, int W, int H, const float* intr,
                  const double* R, const double* t, int64_t cap, int32_t* n_out, int32_t* pix_out,
                  float* w_out, double* d_out, float* p_out)
{
    oop P;
    memset(&P, 0, sizeof(P));
    P.Z = Z;
    P.Wk = Wk;
    P.W = W;
    P.H = H;
    P.fx = intr[0];
    P.fy = intr[1];
    P.cx = intr[2];
    P.cy = intr[3];
    memcpy(P.R, R, sizeof(P.R));
    memcpy(P.t, t, sizeof(P.t));
    oop_setup(&P, v);
    blist L = {0, 0, NULL};
    if (candidates_sparse(v, &P, &L) != OV_OK) return OV_ENOMEM;
    int64_t cnt = 0;
    for (int64_t i = 0; i < L.n; ++i)
        for (int k = 0; k < BVOX; ++k) {
            int64_t n[3];
            touch_t T;
            voxel_of(L.b + 3 * i, k, n);
            if (!touch(v, &P, n, &T)) continue;
            if (cnt < cap) {
                n_out[3 * cnt + 0] = (int32_t)n[0];
                n_out[3 * cnt + 1] = (int32_t)n[1];
                n_out[3 * cnt + 2] = (int32_t)n[2];
                pix_out[cnt] = T.pix;
                w_out[cnt] = T.w;
                d_out[cnt] = T.d;
                p_out[3 * cnt + 0] = T.pf[0];
                p_out[3 * cnt + 1] = T.pf[1];
                p_out[3 * cnt + 2] = T.pf[2];
            }
            cnt++;
        }
    free(L.b);
    return cnt;
}

/* The decision for one voxel: returns 1 and the pixel if touched. */
int ov_touch_one(const ovol* v, const float* Z, const float* Wk, int W, int H, const float* intr, const double* R,
                 const double* t, const int64_t* n, int32_t* pix, float* pf)
{
    oop P;
    memset(&P, 0, sizeof(P));
    P.Z = Z;
    P.Wk = Wk;
    P.W = W;
    P.H = H;
    P.fx = intr[0];
    P.fy = intr[1];
    P.cx = intr[2];
    P.cy = intr[3];
    memcpy(P.R, R, sizeof(P.R));
    memcpy(P.t, t, sizeof(P.t));
    oop_setup(&P, v);
    float p[3];
    cam_point_f32(v, &P, n, p);
    if (pf) {
        pf[0] = p[0];
        pf[1] = p[1];
        pf[2] = p[2];
    }
    int iu, iv;
    if (!nearest_pixel(&P, p, &iu, &iv)) return 0;
    int px = iv * W + iu;
    if (!(qweight(Wk[px]) > 0.0f)) return 0;
    if (!(fabsf(Z[px] - p[2]) <= v->mu)) return 0;
    if (pix) *pix = px;
    return 1;
}

/* One voxel through a sequence of operations, from the empty state: the
 * plain per-voxel definition used to check large volumes on samples.
 * ops: n_ops keyframe indices, signs (+1 integrate, -1 de-integrate) and
 * poses (R n_ops x 9, t n_ops x 3); keyframes: arrays of pointers.  Returns
 * the number of operations that touched the voxel, or a negative error;
 * out_D/out_W/out_C receive the final state (C: 3 values). */
int ov_voxel_sequence(const ovol* v, const float* const* Z, const float* const* Wk, const uint8_t* const* rgba,
                      int W, int H, const float* intr, int n_ops, const int* kf, const int* sign, const double* R,
                      const double* t, const int64_t* n, double* out_D, double* out_W, double* out_C)
{
    ovol tmp = *v;
    tmp.color_f32 = 0;
    tmp.n = 0;
    tmp.cap = 0;
    tmp.bxyz = NULL;
    tmp.D = tmp.W = tmp.C = NULL;
    if (omap_init(&tmp.map, 16) != OV_OK) return OV_ENOMEM;
    int64_t b[3] = {floor_div8(n[0]), floor_div8(n[1]), floor_div8(n[2])};
    int k = (int)((n[0] - 8 * b[0]) + 8 * (n[1] - 8 * b[1]) + 64 * (n[2] - 8 * b[2]));
    int64_t bi = ov_alloc_block(&tmp, b[0], b[1], b[2]);
    int touched = 0, err = OV_OK;
    for (int o = 0; o < n_ops && bi >= 0; ++o) {
        oop P;
        memset(&P, 0, sizeof(P));
        P.Z = Z[kf[o]];
        P.Wk = Wk[kf[o]];
        P.rgba = rgba[kf[o]];
        P.W = W;
        P.H = H;
        P.fx = intr[0];
        P.fy = intr[1];
        P.cx = intr[2];
        P.cy = intr[3];
        memcpy(P.R, R + 9 * o, sizeof(P.R));
        memcpy(P.t, t + 3 * o, sizeof(P.t));
        oop_setup(&P, &tmp);
        touch_t T;
        if (!touch(&tmp, &P, n, &T)) continue;
        touched++;
        int e = update_voxel(&tmp, bi, k, &T, sign[o]);
        if (e != OV_OK && err == OV_OK) err = e;
    }
    if (bi >= 0) {
        *out_D = tmp.D[BVOX * bi + k];
        *out_W = tmp.W[BVOX * bi + k];
        for (int c = 0; c < 3; ++c) out_C[c] = tmp.C[(BVOX * bi + k) * 3 + c];
    }
    omap_free(&tmp.map);
    free(tmp.bxyz);
    free(tmp.D);
    free(tmp.W);
    free(tmp.C);
    if (bi < 0) return OV_ENOMEM;
    return err != OV_OK ? err : touched;
}

/* Export sorted by block key order of insertion is not stable across
 * implementations, so the caller sorts.  Writes n x 3 block coordinates and
 * the per-voxel D, W (n x 512) and colour (n x 512 x 3). */
int64_t ov_export(const ovol* v, int64_t cap, int64_t* bxyz, double* D, double* W, double* C)
{
    int64_t n = v->n < cap ? v->n : cap;
    if (bxyz) memcpy(bxyz, v->bxyz, sizeof(int64_t) * 3 * n);
    if (D) memcpy(D, v->D, sizeof(double) * BVOX * n);
    if (W) memcpy(W, v->W, sizeof(double) * BVOX * n);
    if (C) memcpy(C, v->C, sizeof(double) * BVOX * 3 * n);
    return v->n;
}

/* Import a field (for tests that start from a given state). */
int ov_import(ovol* v, int64_t n, const int64_t* bxyz, const double* D, const double* W, const double* C)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t bi = ov_alloc_block(v, bxyz[3 * i], bxyz[3 * i + 1], bxyz[3 * i + 2]);
        if (bi < 0) return OV_ENOMEM;
        memcpy(v->D + BVOX * bi, D + BVOX * i, sizeof(double) * BVOX);
        memcpy(v->W + BVOX * bi, W + BVOX * i, sizeof(double) * BVOX);
        memcpy(v->C + BVOX * 3 * bi, C + BVOX * 3 * i, sizeof(double) * BVOX * 3);
    }
    return OV_OK;
}

/* ------------------------------------------------------------------------- */
/* keyframe fusion (Sec. 3 "Keyframe Fusion", Eq. 1)                          */
/* ------------------------------------------------------------------------- */

static int zvalid(float z, float zmin, float zmax) { return z >= zmin && z <= zmax; }

static void backproject(float u, float v, float z, const float* intr, float P[3])
{
    P[0] = ((u - intr[2]) * z) / intr[0];
    P[1] = ((v - intr[3]) * z) / intr[1];
    P[2] = z;
}

/*
 * Per-pixel depth weight w_z = cos(theta) * Z^-2 (Sec. 3, Keyframe Fusion),
 * theta the angle between the depth normal and the camera axis, quantised to
 * the 2^-10 grid; 0 marks a rejected pixel.  The normal is the cross product
 * of central differences of back-projected neighbours; a pixel is rejected
 * near a depth discontinuity, i.e. when a 4-neighbour is invalid, out of the
 * image, or differs by more than disc_rel * Z.
 */
void of_depth_weight(const float* Z, int W, int H, const float* intr, float zmin, float zmax, float disc_rel,
                     float* wz)
{
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            float out = 0.0f;
            float z = Z[v * W + u];
            if (zvalid(z, zmin, zmax) && u >= 1 && u <= W - 2 && v >= 1 && v <= H - 2) {
                float zl = Z[v * W + u - 1], zr = Z[v * W + u + 1];
                float zu = Z[(v - 1) * W + u], zd = Z[(v + 1) * W + u];
                int ok = zvalid(zl, zmin, zmax) && zvalid(zr, zmin, zmax) && zvalid(zu, zmin, zmax) &&
                         zvalid(zd, zmin, zmax);
                float th = disc_rel * z;
                if (ok && !(fabsf(zl - z) > th) && !(fabsf(zr - z) > th) && !(fabsf(zu - z) > th) &&
                    !(fabsf(zd - z) > th)) {
                    float Pl[3], Pr[3], Pu[3], Pd[3];
                    backproject((float)(u - 1), (float)v, zl, intr, Pl);
                    backproject((float)(u + 1), (float)v, zr, intr, Pr);
                    backproject((float)u, (float)(v - 1), zu, intr, Pu);
                    backproject((float)u, (float)(v + 1), zd, intr, Pd);
                    float a[3] = {Pr[0] - Pl[0], Pr[1] - Pl[1], Pr[2] - Pl[2]};
                    float b[3] = {Pd[0] - Pu[0], Pd[1] - Pu[1], Pd[2] - Pu[2]};
                    float nx = a[1] * b[2] - a[2] * b[1];
                    float ny = a[2] * b[0] - a[0] * b[2];
                    float nz = a[0] * b[1] - a[1] * b[0];
                    float nn = (nx * nx + ny * ny) + nz * nz;
                    if (nn > 0.0f) {
                        float c = fabsf(nz) / sqrtf(nn);
                        float w = c / (z * z);
                        out = qweight(w);
                    }
                }
            }
            wz[v * W + u] = out;
        }
}

/* relative pose A^-1 B in FP64 (rows of A^T times B), written order */
static void rel_pose(const double* RA, const double* tA, const double* RB, const double* tB, float Rr[9], float tr[3])
{
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
            double x = (RA[0 * 3 + r] * RB[0 * 3 + c] + RA[1 * 3 + r] * RB[1 * 3 + c]) + RA[2 * 3 + r] * RB[2 * 3 + c];
            Rr[3 * r + c] = (float)x;
        }
        double y = (RA[0 * 3 + r] * (tB[0] - tA[0]) + RA[1 * 3 + r] * (tB[1] - tA[1])) + RA[2 * 3 + r] * (tB[2] - tA[2]);
        tr[r] = (float)y;
    }
}

static void xform_f32(const float Rr[9], const float tr[3], const float P[3], float q[3])
{
    for (int r = 0; r < 3; ++r) q[r] = ((Rr[3 * r + 0] * P[0] + Rr[3 * r + 1] * P[1]) + Rr[3 * r + 2] * P[2]) + tr[r];
}

static int px_nearest(const float* intr, int W, int H, const float q[3], float* uf, float* vf, int* iu, int* iv)
{
    if (!(q[2] > 0.0f)) return 0;
    float u = (intr[0] * q[0]) / q[2] + intr[2];
    float v = (intr[1] * q[1]) / q[2] + intr[3];
    *uf = u;
    *vf = v;
    float fu = floorf(u + 0.5f), fv = floorf(v + 0.5f);
    if (!(fu >= 0.0f && fu <= (float)(W - 1) && fv >= 0.0f && fv <= (float)(H - 1))) return 0;
    *iu = (int)fu;
    *iv = (int)fv;
    return 1;
}

/*
 * Depth fusion, Eq. (1): every surviving pixel of every frame is warped into
 * the keyframe, p* = g(T*^-1, g(T_i, pi^-1(x, Z_i(x)))), and averaged at the
 * nearest pixel of pi(p*) with weight w_z.  Eq. (1) is a running weighted
 * mean; its result equals sum(w z) / sum(w), accumulated here in exact
 * integers (w on the 2^-10 grid, z on the 2^-20 m grid) so that the order of
 * contributions cannot matter.  Outputs W* (on the 2^-10 grid) and Z*.
 */
void of_fuse_depth(const float* Z, const float* wz, int n, int W, int H, const float* intr, const double* R,
                   const double* t, int ref, float* Zs, float* Ws)
{
    int64_t* KW = (int64_t*)calloc((size_t)W * H, sizeof(int64_t));
    int64_t* KZ = (int64_t*)calloc((size_t)W * H, sizeof(int64_t));
    for (int i = 0; i < n; ++i) {
        float Rr[9], tr[3];
        rel_pose(R + 9 * ref, t + 3 * ref, R + 9 * i, t + 3 * i, Rr, tr);
        const float* Zi = Z + (size_t)i * W * H;
        const float* wi = wz + (size_t)i * W * H;
        for (int v = 0; v < H; ++v)
            for (int u = 0; u < W; ++u) {
                float w = wi[v * W + u];
                if (!(w > 0.0f)) continue;
                float P[3], q[3];
                backproject((float)u, (float)v, Zi[v * W + u], intr, P);
                xform_f32(Rr, tr, P, q);
                float uf, vf;
                int iu, iv;
                if (!px_nearest(intr, W, H, q, &uf, &vf, &iu, &iv)) continue;
                int64_t wk = (int64_t)rintf(w * WQ_SCALE);
                int64_t zk = (int64_t)rintf(q[2] * 1048576.0f);
                KW[iv * W + iu] += wk;
                KZ[iv * W + iu] += wk * zk;
            }
    }
    for (int p = 0; p < W * H; ++p) {
        if (KW[p] > 0) {
            Ws[p] = (float)((double)KW[p] / 1024.0);
            Zs[p] = (float)(((double)KZ[p] / (double)KW[p]) * 0x1p-20);
        } else {
            Ws[p] = 0.0f;
            Zs[p] = 0.0f;
        }
    }
    free(KW);
    free(KZ);
}

static int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/*
 * Unsharp masking of an RGB image (Sec. 3, colour fusion): Cs = C + (C - G*C)
 * with G the separable binomial [1 4 6 4 1]/16 kernel and clamp-to-edge
 * borders.  Evaluated exactly in integers and returned in units of 1/256:
 * out = clamp(512 C - sum g g C, 0, 255 * 256).
 */
void of_sharpen(const uint8_t* rgb, int W, int H, uint16_t* out)
{
    static const int g[5] = {1, 4, 6, 4, 1};
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u)
            for (int c = 0; c < 3; ++c) {
                int64_t S = 0;
                for (int j = -2; j <= 2; ++j)
                    for (int i = -2; i <= 2; ++i) {
                        int uu = clampi(u + i, 0, W - 1), vv = clampi(v + j, 0, H - 1);
                        S += (int64_t)g[i + 2] * g[j + 2] * rgb[3 * (vv * W + uu) + c];
                    }
                int64_t val = 512 * (int64_t)rgb[3 * (v * W + u) + c] - S;
                if (val < 0) val = 0;
                if (val > 65280) val = 65280;
                out[3 * (v * W + u) + c] = (uint16_t)val;
            }
}

/*
 * No-reference blur measure of a frame (the paper's blurriness w_b, citation
 * unresolved in the text; read here as the re-blur metric of Crete et al.,
 * SPIE 2007).  On integer luminance Y = (77R + 150G + 29B + 128) >> 8, each
 * direction compares neighbour differences of Y with those of Y re-blurred by
 * a 1x9 box (kept as 9x sums so that every quantity is an exact integer):
 *   sF = sum 9|dY|, sV = sum max(0, 9|dY| - |dB|), blur = (sF - sV) / sF.
 * Returns blur = max(blur_h, blur_v) in [0,1]; sums[4] = sF_h, sV_h, sF_v, sV_v.
 * Parity unpinned against the paper's own measure (which the text does not
 * identify): the tests pin this reading by its closed forms and invariants
 * only.
 */
double of_blur(const uint8_t* rgb, int W, int H, int64_t* sums)
{
    int* Y = (int*)malloc(sizeof(int) * (size_t)W * H);
    for (int p = 0; p < W * H; ++p)
        Y[p] = (77 * rgb[3 * p] + 150 * rgb[3 * p + 1] + 29 * rgb[3 * p + 2] + 128) >> 8;
    int64_t sFh = 0, sVh = 0, sFv = 0, sVv = 0;
    for (int v = 0; v < H; ++v)
        for (int u = 1; u < W; ++u) {
            int64_t b1 = 0, b0 = 0;
            for (int j = -4; j <= 4; ++j) {
                b1 += Y[v * W + clampi(u + j, 0, W - 1)];
                b0 += Y[v * W + clampi(u - 1 + j, 0, W - 1)];
            }
            int64_t dF = 9 * (int64_t)abs(Y[v * W + u] - Y[v * W + u - 1]);
            int64_t dB = b1 > b0 ? b1 - b0 : b0 - b1;
            sFh += dF;
            sVh += dF > dB ? dF - dB : 0;
        }
    for (int v = 1; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int64_t b1 = 0, b0 = 0;
            for (int j = -4; j <= 4; ++j) {
                b1 += Y[clampi(v + j, 0, H - 1) * W + u];
                b0 += Y[clampi(v - 1 + j, 0, H - 1) * W + u];
            }
            int64_t dF = 9 * (int64_t)abs(Y[v * W + u] - Y[(v - 1) * W + u]);
            int64_t dB = b1 > b0 ? b1 - b0 : b0 - b1;
            sFv += dF;
            sVv += dF > dB ? dF - dB : 0;
        }
    free(Y);
    if (sums) {
        sums[0] = sFh;
        sums[1] = sVh;
        sums[2] = sFv;
        sums[3] = sVv;
    }
    double bh = sFh > 0 ? (double)(sFh - sVh) / (double)sFh : 0.0;
    double bv = sFv > 0 ? (double)(sFv - sVv) / (double)sFv : 0.0;
    return bh > bv ? bh : bv;
}

typedef struct {
    float c;
    int i;
    int64_t w;
} obs_t;

static int obs_cmp(const void* a, const void* b)
{
    const obs_t* x = (const obs_t*)a;
    const obs_t* y = (const obs_t*)b;
    if (x->c < y->c) return -1;
    if (x->c > y->c) return 1;
    return (x->i > y->i) - (x->i < y->i);
}

/*
 * Colour fusion (Sec. 3, Keyframe Fusion): each keyframe pixel with fused
 * depth is warped back into every input frame i,
 *   x_i = pi(g(T_i^-1, g(T*, pi^-1(x*, Z*(x*))))),
 * and the sharpened colour is sampled bilinearly.  An observation is valid
 * when it lies in front of the camera, its nearest pixel has a positive depth
 * weight w_z in frame i and a depth within occ_rel * z of the warped depth
 * (visibility), and its 2x2 footprint is in the image.  Its weight is
 * w_b,i * w_z (quantised to 2^-20 so the cumulative sums are exact).  The
 * keyframe colour is the per-channel lower weighted median: values sorted
 * ascending (ties by frame index), the first whose cumulative weight reaches
 * half the total.  A pixel without observations is invalidated (Z* = W* = 0).
 * Colour output is RGBA8 with alpha 255 on valid pixels.
 */
void of_fuse_color(const float* Z, const float* wz, const uint16_t* cs, const double* wb, int n, int W, int H,
                   const float* intr, const double* R, const double* t, int ref, float occ_rel, float* Zs,
                   float* Ws, uint8_t* rgba)
{
    float (*Rr)[9] = malloc(sizeof(float[9]) * n);
    float (*tr)[3] = malloc(sizeof(float[3]) * n);
    for (int i = 0; i < n; ++i) rel_pose(R + 9 * i, t + 3 * i, R + 9 * ref, t + 3 * ref, Rr[i], tr[i]);
    obs_t* obs = (obs_t*)malloc(sizeof(obs_t) * n * 3);
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int p = v * W + u;
            uint8_t* out = rgba + 4 * p;
            out[0] = out[1] = out[2] = out[3] = 0;
            if (!(Ws[p] > 0.0f)) continue;
            float P[3];
            backproject((float)u, (float)v, Zs[p], intr, P);
            int m = 0;
            float cval[64][3];
            int fidx[64];
            int64_t wq[64];
            for (int i = 0; i < n && m < 64; ++i) {
                float q[3], uf, vf;
                int iu, iv;
                xform_f32(Rr[i], tr[i], P, q);
                if (!px_nearest(intr, W, H, q, &uf, &vf, &iu, &iv)) continue;
                const float* Zi = Z + (size_t)i * W * H;
                float wzi = wz[(size_t)i * W * H + iv * W + iu];
                if (!(wzi > 0.0f)) continue;
                if (!(fabsf(Zi[iv * W + iu] - q[2]) <= occ_rel * q[2])) continue;
                float x0 = floorf(uf), y0 = floorf(vf);
                if (!(x0 >= 0.0f && x0 + 1.0f <= (float)(W - 1) && y0 >= 0.0f && y0 + 1.0f <= (float)(H - 1))) continue;
                float ax = uf - x0, ay = vf - y0;
                int ix = (int)x0, iy = (int)y0;
                const uint16_t* C = cs + (size_t)i * W * H * 3;
                float wc = (float)wb[i] * wzi;
                float wcs = rintf(wc * 1048576.0f);
                if (!(wcs > 0.0f)) continue;
                for (int c = 0; c < 3; ++c) {
                    float c00 = (float)C[3 * (iy * W + ix) + c], c10 = (float)C[3 * (iy * W + ix + 1) + c];
                    float c01 = (float)C[3 * ((iy + 1) * W + ix) + c], c11 = (float)C[3 * ((iy + 1) * W + ix + 1) + c];
                    float top = c00 + ax * (c10 - c00);
                    float bot = c01 + ax * (c11 - c01);
                    cval[m][c] = top + ay * (bot - top);
                }
                fidx[m] = i;
                wq[m] = (int64_t)wcs;
                m++;
            }
            if (m == 0) {
                Zs[p] = 0.0f;
                Ws[p] = 0.0f;
                continue;
            }
            for (int c = 0; c < 3; ++c) {
                int64_t total = 0;
                for (int j = 0; j < m; ++j) {
                    obs[j].c = cval[j][c];
                    obs[j].i = fidx[j];
                    obs[j].w = wq[j];
                    total += wq[j];
                }
                qsort(obs, (size_t)m, sizeof(obs_t), obs_cmp);
                int64_t cum = 0;
                float pick = obs[m - 1].c;
                for (int j = 0; j < m; ++j) {
                    cum += obs[j].w;
                    if (2 * cum >= total) {
                        pick = obs[j].c;
                        break;
                    }
                }
                float val = rintf(pick / 256.0f);
                if (val < 0.0f) val = 0.0f;
                if (val > 255.0f) val = 255.0f;
                out[c] = (uint8_t)val;
            }
            out[3] = 255;
        }
    free(Rr);
    free(tr);
    free(obs);
}

/* Sets the OpenMP thread count used by the oracle's parallel loops (for
 * timing it on one core or on all of them); returns the new maximum. */
int ov_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int ov_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
