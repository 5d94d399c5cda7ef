/*
 * hexfc_oracle.c -- plain, slow, FP64 CPU oracle of the focus+context hex-mesh
 * render path (Neuhauser, Wang, Westermann, "Interactive Focus+Context
 * Rendering for Hexahedral Mesh Inspection", arXiv 2009.06574).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or table with the HIP library; the
 * two implement the same written definitions independently.
 *
 * What it computes, per frame, for a chosen set of pixels:
 *   1. the mesh attributes (Section 3: per-cell deformation, vertex and edge
 *      importance as maxima over incident cells; faces deduplicated),
 *   2. the exact integer vertex transform and snap, coverage of every face
 *      triangle (two per face, Section 4) and the exact depth key,
 *   3. each pixel's fragment list sorted front to back (Section 3 / Section 6:
 *      sorted by distance to the camera; ties by triangle id),
 *   4. each fragment's colour by Eq. 1-4 with the focus of Section 4,
 *   5. front-to-back alpha compositing (Section 4.2).
 * Floating point is FP64 throughout; geometry is exact integer arithmetic.
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - integer geometry contract (quantisation, snap, fill rule, depth key),
 *   - object-space spherical lens distance, Eq. 3's dist clamped to 1,
 *   - halo/darkening constants are parameters; nearest-edge colour = TF(t_e),
 *   - importance = normalised (1 - scaled Jacobian) unless a scalar is given.
 *
 * Pins: see tests/test_oracle_*.py (closed forms, brute force, invariants).
 * The edge colour (TF of the nearest visible edge's importance, darkened in
 * focus), the halo band and its white colour, and the accent brightening are
 * pinned on a two-cell orthographic setup whose distances and importances are
 * known by construction (tests/test_oracle_edges.py); their default values
 * (halo width, darkening, brightening) are parameters the paper leaves open.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERANGE = -2, ORC_ENOMEM = -3 };

/* ---------------------------------------------------------------- contract */
/* positions: X_q = rint(x * 2^16), |x| < 4                                   */
/* matrix:    M_q = rint(M * 2^20), |M_ij| < 8; rows 0, 1, 3 are used          */
/* clip:      c = M_q * (X_q, 2^16)   (scale 2^36)                             */
/* screen:    4 sub-pixel bits; pixel (i,j) centre at (16i+8, 16j+8)           */
/* near:      w_q < 2^32 (w < 1/16) culls; guard band |s| >= 2^17 culls        */
/* depth:     q = floor(2^56 / w_q) <= 2^24, key = floor(sum E_i q_i / sum E_i) */
#define ORC_POS_SCALE 65536.0
#define ORC_MAT_SCALE 1048576.0
#define ORC_W_NEAR (((int64_t)1) << 32)
#define ORC_GUARD (((int64_t)1) << 17)
#define ORC_QNUM (((int64_t)1) << 56)
#define ORC_KMAX (((int64_t)1) << 24)

/* VTK hexahedron faces and the local edge table of cell_edge_level */
static const int FACE_CORNERS[6][4] = {
    {0, 4, 7, 3}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 7, 6, 2}, {0, 3, 2, 1}, {4, 5, 6, 7}};
static const int CELL_EDGE[12][2] = {
    {0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6}, {6, 7}, {7, 4},
    {0, 4}, {1, 5}, {2, 6}, {3, 7}};
/* the three neighbours of each corner, ordered so that the unit cube has
 * det = +1 at every corner (right-handed frame) */
static const int CORNER_NB[8][3] = {
    {1, 3, 4}, {2, 0, 5}, {3, 1, 6}, {0, 2, 7}, {7, 5, 0}, {4, 6, 1}, {5, 7, 2}, {6, 4, 3}};

/* style vector layout (doubles) */
enum {
    ST_W_BASE, ST_K_FOCUS, ST_HALO_W, ST_HALO_A, ST_DARKEN, ST_S, ST_BRIGHT, ST_DELTA, ST_LOD,
    ST_TF_LO, ST_TF_LO_G, ST_TF_LO_B, ST_TF_HI, ST_TF_HI_G, ST_TF_HI_B, ST_A_LO, ST_A_HI,
    ST_BG, ST_BG_G, ST_BG_B, ST_LENS_MODE, ST_DESAT, ST_SIL_A, ST_SIL_TAU, ST_COUNT
};

/* ---------------------------------------------------------------- mesh */
typedef struct orc_mesh {
    int64_t V, C, F;
    int32_t *pos_q;    /* V*3 */
    double *t_cell;    /* C   */
    double *t_v;       /* V   */
    int32_t *face_v;   /* F*4 */
    uint8_t *face_lvl; /* F*4 */
    double *face_te;   /* F*4 */
    uint8_t *face_bnd; /* F: 1 if the face belongs to one cell only (mesh boundary) */
} orc_mesh;

typedef struct { int64_t a, b; int lvl; double t; } edge_ent;
typedef struct { int32_t key[4]; int64_t idx; } face_ent;

static int cmp_edge(const void *x, const void *y) {
    const edge_ent *p = (const edge_ent *)x, *q = (const edge_ent *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return 0;
}
static int cmp_face(const void *x, const void *y) {
    const face_ent *p = (const face_ent *)x, *q = (const face_ent *)y;
    for (int i = 0; i < 4; ++i)
        if (p->key[i] != q->key[i]) return p->key[i] < q->key[i] ? -1 : 1;
    if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;
    return 0;
}
static int cmp_i64(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return a < b ? -1 : (a > b);
}
static int cmp_u64(const void *x, const void *y) {
    uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return a < b ? -1 : (a > b);
}

/* Scaled Jacobian of one hexahedron (corners in VTK order, 8x3 doubles): the
 * minimum over the 8 corners of det[e1,e2,e3] of the unit edge vectors to the
 * corner's three neighbours (the Verdict-style corner measure, Section 3). */
double orc_scaled_jacobian(const double *c) {
    double best = INFINITY;
    for (int k = 0; k < 8; ++k) {
        double e[3][3];
        for (int m = 0; m < 3; ++m) {
            const double *a = c + 3 * k, *b = c + 3 * CORNER_NB[k][m];
            double v0 = b[0] - a[0], v1 = b[1] - a[1], v2 = b[2] - a[2];
            double len = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
            if (len == 0.0) return 0.0;
            e[m][0] = v0 / len; e[m][1] = v1 / len; e[m][2] = v2 / len;
        }
        double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1])
                   - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0])
                   + e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        if (det < best) best = det;
    }
    return best;
}

void orc_mesh_free(orc_mesh *m) {
    if (!m) return;
    free(m->pos_q); free(m->t_cell); free(m->t_v);
    free(m->face_v); free(m->face_lvl); free(m->face_te); free(m->face_bnd);
    free(m);
}

static int64_t find_edge(const edge_ent *u, int64_t n, int64_t a, int64_t b) {
    int64_t lo = 0, hi = n - 1;
    if (a > b) { int64_t t = a; a = b; b = t; }
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (u[mid].a == a && u[mid].b == b) return mid;
        if (u[mid].a < a || (u[mid].a == a && u[mid].b < b)) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Mesh attributes (Section 3 and Section 4):
 *  - positions quantised to the integer contract,
 *  - per-cell importance: the given scalar, or 1 - scaled Jacobian; normalised
 *    to [0,1] over the mesh,
 *  - vertex importance = max over incident cells; edge importance = max over
 *    cells sharing the edge,
 *  - faces deduplicated (first-seen order, corner order of the first cell),
 *  - per face edge k = (corner k, corner k+1): LoD level and importance. */
int orc_mesh_build(const float *xyz, int64_t V, const int32_t *hex, int64_t C,
                   const float *scalar, const uint8_t *lvl, orc_mesh **out) {
    *out = NULL;
    if (V <= 0 || C < 0 || !xyz || (C > 0 && !hex)) return ORC_EINVAL;
    for (int64_t i = 0; i < 3 * V; ++i)
        if (!(fabs((double)xyz[i]) < 4.0)) return ORC_ERANGE;
    for (int64_t i = 0; i < 8 * C; ++i)
        if (hex[i] < 0 || hex[i] >= V) return ORC_ERANGE;
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    if (!m) return ORC_ENOMEM;
    m->V = V; m->C = C;
    m->pos_q = (int32_t *)malloc(sizeof(int32_t) * 3 * V);
    m->t_cell = (double *)malloc(sizeof(double) * (C ? C : 1));
    m->t_v = (double *)calloc(V, sizeof(double));
    if (!m->pos_q || !m->t_cell || !m->t_v) { orc_mesh_free(m); return ORC_ENOMEM; }
    for (int64_t i = 0; i < 3 * V; ++i) m->pos_q[i] = (int32_t)rint((double)xyz[i] * ORC_POS_SCALE);

    /* importance */
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t c = 0; c < C; ++c) {
        double raw;
        if (scalar) {
            raw = (double)scalar[c];
        } else {
            double corners[24];
            for (int k = 0; k < 8; ++k)
                for (int a = 0; a < 3; ++a)
                    corners[3 * k + a] = (double)m->pos_q[3 * (int64_t)hex[8 * c + k] + a] / ORC_POS_SCALE;
            raw = 1.0 - orc_scaled_jacobian(corners);
        }
        m->t_cell[c] = raw;
        if (raw < lo) lo = raw;
        if (raw > hi) hi = raw;
    }
    for (int64_t c = 0; c < C; ++c)
        m->t_cell[c] = (hi > lo) ? (m->t_cell[c] - lo) / (hi - lo) : 0.0;
    for (int64_t c = 0; c < C; ++c)
        for (int k = 0; k < 8; ++k) {
            int64_t v = hex[8 * c + k];
            if (m->t_cell[c] > m->t_v[v]) m->t_v[v] = m->t_cell[c];
        }

    /* edges */
    edge_ent *E = (edge_ent *)malloc(sizeof(edge_ent) * (12 * C + 1));
    if (!E) { orc_mesh_free(m); return ORC_ENOMEM; }
    for (int64_t c = 0; c < C; ++c)
        for (int e = 0; e < 12; ++e) {
            int64_t a = hex[8 * c + CELL_EDGE[e][0]], b = hex[8 * c + CELL_EDGE[e][1]];
            if (a == b) { free(E); orc_mesh_free(m); return ORC_EINVAL; }
            edge_ent *x = &E[12 * c + e];
            x->a = a < b ? a : b; x->b = a < b ? b : a;
            x->lvl = lvl ? lvl[12 * c + e] : 0;
            x->t = m->t_cell[c];
        }
    qsort(E, 12 * C, sizeof(edge_ent), cmp_edge);
    int64_t nE = 0;
    for (int64_t i = 0; i < 12 * C; ++i) {
        if (nE > 0 && E[nE - 1].a == E[i].a && E[nE - 1].b == E[i].b) {
            if (E[nE - 1].lvl != E[i].lvl) { free(E); orc_mesh_free(m); return ORC_EINVAL; }
            if (E[i].t > E[nE - 1].t) E[nE - 1].t = E[i].t;
        } else {
            E[nE++] = E[i];
        }
    }

    /* faces */
    face_ent *Fe = (face_ent *)malloc(sizeof(face_ent) * (6 * C + 1));
    if (!Fe) { free(E); orc_mesh_free(m); return ORC_ENOMEM; }
    for (int64_t c = 0; c < C; ++c)
        for (int f = 0; f < 6; ++f) {
            face_ent *x = &Fe[6 * c + f];
            int32_t k[4];
            for (int i = 0; i < 4; ++i) k[i] = hex[8 * c + FACE_CORNERS[f][i]];
            for (int i = 1; i < 4; ++i) /* insertion sort of 4 ids */
                for (int j = i; j > 0 && k[j - 1] > k[j]; --j) { int32_t t = k[j]; k[j] = k[j - 1]; k[j - 1] = t; }
            memcpy(x->key, k, sizeof k);
            x->idx = 6 * c + f;
        }
    qsort(Fe, 6 * C, sizeof(face_ent), cmp_face);
    int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (6 * C + 1));
    int64_t *single = (int64_t *)malloc(sizeof(int64_t) * (6 * C + 1));  /* first ids of faces of one cell */
    int64_t nF = 0, nS = 0;
    for (int64_t i = 0; i < 6 * C; ++i)
        if (i == 0 || memcmp(Fe[i].key, Fe[i - 1].key, sizeof Fe[i].key) != 0) {
            first[nF++] = Fe[i].idx;
            if (i + 1 >= 6 * C || memcmp(Fe[i].key, Fe[i + 1].key, sizeof Fe[i].key) != 0) single[nS++] = Fe[i].idx;
        }
    qsort(first, nF, sizeof(int64_t), cmp_i64);
    qsort(single, nS, sizeof(int64_t), cmp_i64);
    m->F = nF;
    m->face_v = (int32_t *)malloc(sizeof(int32_t) * 4 * (nF ? nF : 1));
    m->face_lvl = (uint8_t *)malloc(4 * (nF ? nF : 1));
    m->face_te = (double *)malloc(sizeof(double) * 4 * (nF ? nF : 1));
    m->face_bnd = (uint8_t *)calloc(nF ? nF : 1, 1);
    for (int64_t f = 0, q = 0; f < nF; ++f) {  /* both lists ascending: merge */
        while (q < nS && single[q] < first[f]) ++q;
        m->face_bnd[f] = q < nS && single[q] == first[f];
    }
    for (int64_t f = 0; f < nF; ++f) {
        int64_t c = first[f] / 6, lf = first[f] % 6;
        for (int i = 0; i < 4; ++i) m->face_v[4 * f + i] = hex[8 * c + FACE_CORNERS[lf][i]];
        for (int k = 0; k < 4; ++k) {
            int64_t e = find_edge(E, nE, m->face_v[4 * f + k], m->face_v[4 * f + (k + 1) % 4]);
            m->face_lvl[4 * f + k] = (uint8_t)E[e].lvl;
            m->face_te[4 * f + k] = E[e].t;
        }
    }
    free(first); free(single); free(Fe); free(E);
    *out = m;
    return ORC_OK;
}

void orc_mesh_sizes(const orc_mesh *m, int64_t *out3) { out3[0] = m->V; out3[1] = m->C; out3[2] = m->F; }
void orc_mesh_boundary(const orc_mesh *m, uint8_t *out) { memcpy(out, m->face_bnd, (size_t)m->F); }

void orc_mesh_export(const orc_mesh *m, int32_t *pos_q, double *t_cell, double *t_v,
                     int32_t *face_v, uint8_t *face_lvl, double *face_te) {
    if (pos_q) memcpy(pos_q, m->pos_q, sizeof(int32_t) * 3 * m->V);
    if (t_cell) memcpy(t_cell, m->t_cell, sizeof(double) * m->C);
    if (t_v) memcpy(t_v, m->t_v, sizeof(double) * m->V);
    if (face_v) memcpy(face_v, m->face_v, sizeof(int32_t) * 4 * m->F);
    if (face_lvl) memcpy(face_lvl, m->face_lvl, 4 * m->F);
    if (face_te) memcpy(face_te, m->face_te, sizeof(double) * 4 * m->F);
}

/* ---------------------------------------------------------------- frame */
typedef struct orc_frame {
    const orc_mesh *m;
    int W, H;
    int64_t Mq[16];
    double wrow[4];    /* row 3 (clip w) of the float camera matrix */
    double w0, w1;     /* clip-w range of the corners of the mesh bbox */
    int32_t *sx, *sy, *q;
    uint8_t *vflag;
    int64_t npix;
    int32_t *pix;      /* sample pixels, row-major index y*W+x */
    uint32_t *count;   /* per sample */
    uint64_t *off;     /* npix+1 */
    uint64_t *rec;     /* sorted records */
    /* shading candidates (pixels with ambiguous discontinuities) */
    int64_t *cand_off; /* npix+1, or NULL */
    double *cand;
    int64_t ncand;
} orc_frame;

static int64_t floor_div(int64_t n, int64_t d) { /* d > 0 */
    int64_t q = n / d, r = n % d;
    return (r != 0 && r < 0) ? q - 1 : q;
}

/* edge function of directed edge a->b at p (cross product z of (b-a) x (p-a)) */
static int64_t edgef(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py) {
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}
/* fill rule: a pixel centre exactly on an edge belongs to the triangle iff the
 * edge (oriented with the interior on its left) has dy < 0, or dy == 0 and
 * dx > 0.  This equals sampling at the centre nudged by (+eps, +eps*delta). */
static int on_edge_owned(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
    int64_t dx = bx - ax, dy = by - ay;
    return dy < 0 || (dy == 0 && dx > 0);
}

static void tri_vertices(const orc_mesh *m, int64_t tri, int64_t v[3]) {
    int64_t f = tri >> 1;
    const int32_t *c = m->face_v + 4 * f;
    v[0] = c[0];
    if ((tri & 1) == 0) { v[1] = c[1]; v[2] = c[2]; }
    else { v[1] = c[2]; v[2] = c[3]; }
}

void orc_frame_free(orc_frame *fr) {
    if (!fr) return;
    free(fr->sx); free(fr->sy); free(fr->q); free(fr->vflag); free(fr->pix);
    free(fr->count); free(fr->off); free(fr->rec); free(fr->cand_off); free(fr->cand);
    free(fr);
}

/* Covers (exactly) pixel centre (px,py) by the triangle with snapped vertices?
 * If so returns 1 and the depth key. */
static int cover_key(const orc_frame *fr, const int64_t v[3], int64_t px, int64_t py, int64_t *key) {
    int64_t x[3], y[3], qq[3];
    for (int i = 0; i < 3; ++i) { x[i] = fr->sx[v[i]]; y[i] = fr->sy[v[i]]; qq[i] = fr->q[v[i]]; }
    int64_t area = edgef(x[0], y[0], x[1], y[1], x[2], y[2]);
    if (area == 0) return 0;
    int o[3] = {0, 1, 2};
    if (area < 0) { o[1] = 2; o[2] = 1; }
    /* oriented edges: o0->o1, o1->o2, o2->o0; edge opposite vertex o2, o0, o1 */
    int64_t e_opp[3]; /* barycentric weight of oriented vertex k */
    for (int k = 0; k < 3; ++k) {
        int a = o[k], b = o[(k + 1) % 3];
        int64_t e = edgef(x[a], y[a], x[b], y[b], px, py);
        if (e < 0 || (e == 0 && !on_edge_owned(x[a], y[a], x[b], y[b]))) return 0;
        e_opp[(k + 2) % 3] = e; /* edge a->b is opposite the third vertex */
    }
    int64_t D = e_opp[0] + e_opp[1] + e_opp[2];
    int64_t N = e_opp[0] * qq[o[0]] + e_opp[1] * qq[o[1]] + e_opp[2] * qq[o[2]];
    *key = N / D; /* N >= 0, D > 0 */
    return 1;
}

int orc_frame_raster(const orc_mesh *m, const float *vp, int W, int H, int64_t npix,
                     const int32_t *pix, orc_frame **out) {
    *out = NULL;
    if (W < 1 || H < 1 || W > 8192 || H > 8192) return ORC_ERANGE;
    for (int i = 0; i < 16; ++i)
        if (!(fabs((double)vp[i]) < 8.0)) return ORC_ERANGE;
    orc_frame *fr = (orc_frame *)calloc(1, sizeof(orc_frame));
    if (!fr) return ORC_ENOMEM;
    fr->m = m; fr->W = W; fr->H = H;
    for (int i = 0; i < 16; ++i) fr->Mq[i] = (int64_t)rint((double)vp[i] * ORC_MAT_SCALE);
    for (int i = 0; i < 4; ++i) fr->wrow[i] = (double)vp[12 + i];
    {   /* view-depth range of the mesh bbox (normalises the depth cue) */
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t v = 0; v < m->V; ++v)
            for (int a = 0; a < 3; ++a) {
                double x = (double)m->pos_q[3 * v + a] / ORC_POS_SCALE;
                if (x < lo[a]) lo[a] = x;
                if (x > hi[a]) hi[a] = x;
            }
        fr->w0 = 1e300;
        fr->w1 = -1e300;
        for (int c = 0; c < 8; ++c) {
            double x[3] = {(c & 1) ? hi[0] : lo[0], (c & 2) ? hi[1] : lo[1], (c & 4) ? hi[2] : lo[2]};
            double w = fr->wrow[0] * x[0] + fr->wrow[1] * x[1] + fr->wrow[2] * x[2] + fr->wrow[3];
            if (w < fr->w0) fr->w0 = w;
            if (w > fr->w1) fr->w1 = w;
        }
        if (!(fr->w1 > fr->w0)) fr->w1 = fr->w0 + 1.0;
    }
    int64_t V = m->V;
    fr->sx = (int32_t *)calloc(V, 4); fr->sy = (int32_t *)calloc(V, 4);
    fr->q = (int32_t *)calloc(V, 4); fr->vflag = (uint8_t *)calloc(V, 1);
    /* vertex transform and snap */
    for (int64_t v = 0; v < V; ++v) {
        int64_t X[4] = {m->pos_q[3 * v], m->pos_q[3 * v + 1], m->pos_q[3 * v + 2], 65536};
        int64_t c[4];
        for (int r = 0; r < 4; ++r) {
            c[r] = 0;
            if (r == 2) continue;
            for (int j = 0; j < 4; ++j) c[r] += fr->Mq[4 * r + j] * X[j];
        }
        int64_t cx = c[0], cy = c[1], cw = c[3];
        if (cw < ORC_W_NEAR) { fr->vflag[v] = 1; continue; }
        int64_t sx = floor_div((cx + cw) * (int64_t)W * 16 + cw, 2 * cw);
        int64_t sy = floor_div((cw - cy) * (int64_t)H * 16 + cw, 2 * cw);
        if (sx >= ORC_GUARD || sx <= -ORC_GUARD || sy >= ORC_GUARD || sy <= -ORC_GUARD) { fr->vflag[v] = 2; continue; }
        fr->sx[v] = (int32_t)sx; fr->sy[v] = (int32_t)sy;
        fr->q[v] = (int32_t)(ORC_QNUM / cw);
    }
    /* sample set */
    int64_t P = (int64_t)W * H;
    fr->npix = pix ? npix : P;
    fr->pix = (int32_t *)malloc(sizeof(int32_t) * (fr->npix + 1));
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * P);
    for (int64_t i = 0; i < P; ++i) map[i] = -1;
    for (int64_t s = 0; s < fr->npix; ++s) {
        int32_t p = pix ? pix[s] : (int32_t)s;
        if (p < 0 || p >= P) { free(map); orc_frame_free(fr); return ORC_ERANGE; }
        if (map[p] >= 0) { free(map); orc_frame_free(fr); return ORC_EINVAL; } /* repeated sample pixel */
        fr->pix[s] = p;
        map[p] = (int32_t)s;
    }
    fr->count = (uint32_t *)calloc(fr->npix + 1, 4);
    fr->off = (uint64_t *)calloc(fr->npix + 1, 8);
    /* two passes over all triangles: count, then store */
    for (int pass = 0; pass < 2; ++pass) {
        uint32_t *fillc = NULL;
        if (pass == 1) {
            for (int64_t s = 0; s < fr->npix; ++s) fr->off[s + 1] = fr->off[s] + fr->count[s];
            fr->rec = (uint64_t *)malloc(8 * (fr->off[fr->npix] + 1));
            fillc = (uint32_t *)calloc(fr->npix + 1, 4);
        }
        for (int64_t tri = 0; tri < 2 * m->F; ++tri) {
            int64_t v[3];
            tri_vertices(m, tri, v);
            if (fr->vflag[v[0]] | fr->vflag[v[1]] | fr->vflag[v[2]]) continue;
            int64_t xmin = fr->sx[v[0]], xmax = xmin, ymin = fr->sy[v[0]], ymax = ymin;
            for (int i = 1; i < 3; ++i) {
                if (fr->sx[v[i]] < xmin) xmin = fr->sx[v[i]];
                if (fr->sx[v[i]] > xmax) xmax = fr->sx[v[i]];
                if (fr->sy[v[i]] < ymin) ymin = fr->sy[v[i]];
                if (fr->sy[v[i]] > ymax) ymax = fr->sy[v[i]];
            }
            int64_t i0 = -floor_div(-(xmin - 8), 16), i1 = floor_div(xmax - 8, 16);
            int64_t j0 = -floor_div(-(ymin - 8), 16), j1 = floor_div(ymax - 8, 16);
            if (i0 < 0) i0 = 0;
            if (j0 < 0) j0 = 0;
            if (i1 > W - 1) i1 = W - 1;
            if (j1 > H - 1) j1 = H - 1;
            for (int64_t j = j0; j <= j1; ++j)
                for (int64_t i = i0; i <= i1; ++i) {
                    int32_t s = map[j * W + i];
                    if (s < 0) continue;
                    int64_t key;
                    if (!cover_key(fr, v, 16 * i + 8, 16 * j + 8, &key)) continue;
                    if (pass == 0) {
                        fr->count[s]++;
                    } else {
                        uint64_t depth = (uint64_t)(ORC_KMAX - key);
                        fr->rec[fr->off[s] + fillc[s]++] = (depth << 32) | (uint64_t)tri;
                    }
                }
        }
        free(fillc);
    }
    free(map);
    /* sort each list ascending: front to back, ties by triangle id */
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t s = 0; s < fr->npix; ++s)
        qsort(fr->rec + fr->off[s], fr->count[s], 8, cmp_u64);
    *out = fr;
    return ORC_OK;
}

int64_t orc_frame_nfrag(const orc_frame *fr) { return (int64_t)fr->off[fr->npix]; }

void orc_frame_lists(const orc_frame *fr, uint32_t *count, uint64_t *off, uint64_t *rec) {
    if (count) memcpy(count, fr->count, 4 * fr->npix);
    if (off) memcpy(off, fr->off, 8 * (fr->npix + 1));
    if (rec) memcpy(rec, fr->rec, 8 * fr->off[fr->npix]);
}

void orc_frame_vertices(const orc_frame *fr, int32_t *sx, int32_t *sy, int32_t *q, uint8_t *flags) {
    int64_t V = fr->m->V;
    if (sx) memcpy(sx, fr->sx, 4 * V);
    if (sy) memcpy(sy, fr->sy, 4 * V);
    if (q) memcpy(q, fr->q, 4 * V);
    if (flags) memcpy(flags, fr->vflag, V);
}

/* ---------------------------------------------------------------- shading */
double orc_smoothstep(double e0, double e1, double x) {
    double u = (x - e0) / (e1 - e0);
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
    return u * u * (3.0 - 2.0 * u);
}

static double seg_dist(const double p[3], const double a[3], const double b[3]) {
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double l2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
    double t = l2 > 0.0 ? (ap[0] * ab[0] + ap[1] * ab[1] + ap[2] * ab[2]) / l2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double d[3] = {ap[0] - t * ab[0], ap[1] - t * ab[1], ap[2] - t * ab[2]};
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* predicate bits used for the ambiguity bookkeeping */
enum { B_EF = 0, B_HALO = 1, B_EC = 2, B_ACC = 3, B_ARGF = 4, B_ARGC = 5, B_MEM = 6 /* ..9 */ };

typedef struct { double c[3]; double a; } frag;

/* One fragment's premultiplied colour and opacity (Eq. 1 with halo, Eq. 2,
 * Eq. 3, Eq. 4).  `flip` inverts the listed discontinuous predicates; with
 * flip == 0, *amb receives the predicates whose FP64 margin is below the FP32
 * error bound (their other outcome is also a correct result). */
static void shade(const orc_frame *fr, int64_t px_i, int64_t px_j, uint64_t tri,
                  const double *hot, const double *st, unsigned flip, frag *out, unsigned *amb) {
    const orc_mesh *m = fr->m;
    int64_t v[3];
    tri_vertices(m, (int64_t)tri, v);
    int64_t f = (int64_t)(tri >> 1);
    int64_t px = 16 * px_i + 8, py = 16 * px_j + 8;
    /* perspective-correct barycentrics: lambda_i ~ E_i(p) q_i */
    double w[3], sum = 0.0;
    for (int i = 0; i < 3; ++i) {
        int a = (i + 1) % 3, b = (i + 2) % 3;
        int64_t e = edgef(fr->sx[v[a]], fr->sy[v[a]], fr->sx[v[b]], fr->sy[v[b]], px, py);
        w[i] = (double)e * (double)fr->q[v[i]];
        sum += w[i];
    }
    double p[3] = {0, 0, 0}, tf = 0.0;
    for (int i = 0; i < 3; ++i) {
        double l = w[i] / sum;
        for (int a = 0; a < 3; ++a) p[a] += l * (double)m->pos_q[3 * v[i] + a] / ORC_POS_SCALE;
        tf += l * m->t_v[v[i]];
    }
    /* focus: distance to the lens centre, 0 at the centre, 1 at the border:
       object-space sphere (lens mode 0) or screen-space circle in pixels
       (lens mode 1, Section 4: centre hot[0], hot[1], radius hot[3]) */
    double dist;
    if (st[ST_LENS_MODE] == 1.0) {
        double ex = (double)px_i + 0.5 - hot[0], ey = (double)px_j + 0.5 - hot[1];
        dist = sqrt(ex * ex + ey * ey) / hot[3];
    } else {
        double dx = p[0] - hot[0], dy = p[1] - hot[1], dz = p[2] - hot[2];
        dist = sqrt(dx * dx + dy * dy + dz * dz) / hot[3];
    }
    double focus = 1.0 - orc_smoothstep(0.7, 1.0, dist);
    /* distances to the four face edges */
    double P[4][3], d[4], L = 0.0;
    for (int k = 0; k < 4; ++k)
        for (int a = 0; a < 3; ++a) P[k][a] = (double)m->pos_q[3 * (int64_t)m->face_v[4 * f + k] + a] / ORC_POS_SCALE;
    for (int k = 1; k < 4; ++k) {
        double e0 = P[k][0] - P[0][0], e1 = P[k][1] - P[0][1], e2 = P[k][2] - P[0][2];
        double l = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        if (l > L) L = l;
    }
    for (int k = 0; k < 4; ++k) d[k] = seg_dist(p, P[k], P[(k + 1) % 4]);
    const double wb = st[ST_W_BASE], kf = st[ST_K_FOCUS], hw = st[ST_HALO_W], ha = st[ST_HALO_A];
    const double delta = st[ST_DELTA];
    const int lod = (int)st[ST_LOD];
    const double tau_d = 1e-5 * (L + wb * (1.0 + kf) + hw), tau_t = 1e-6;
    unsigned A = 0;
    /* visible edge sets (Eq. 1): F = focus edges, C = contextual edges */
    int inF[4], inC[4];
    for (int k = 0; k < 4; ++k) {
        int lv = m->face_lvl[4 * f + k];
        double te = m->face_te[4 * f + k];
        inC[k] = lv >= lod;
        int imp = te >= delta;
        if (!inC[k] && fabs(te - delta) < tau_t) A |= 1u << (B_MEM + k);
        if (flip & (1u << (B_MEM + k))) imp = !imp;
        inF[k] = inC[k] || imp;
    }
    int aF = -1, aF2 = -1, aC = -1, aC2 = -1, aAll = 0;
    for (int k = 0; k < 4; ++k) {
        if (d[k] < d[aAll]) aAll = k;
        if (inF[k]) {
            if (aF < 0 || d[k] < d[aF]) { aF2 = aF; aF = k; }
            else if (aF2 < 0 || d[k] < d[aF2]) aF2 = k;
        }
        if (inC[k]) {
            if (aC < 0 || d[k] < d[aC]) { aC2 = aC; aC = k; }
            else if (aC2 < 0 || d[k] < d[aC2]) aC2 = k;
        }
    }
    double dF = aF >= 0 ? d[aF] : INFINITY, dC = aC >= 0 ? d[aC] : INFINITY, dAll = d[aAll];
    double wd = (1.0 + kf * focus) * wb;
    int eF = dF <= wd, eC = dC <= wd;
    if (aF >= 0 && focus > 0 && fabs(dF - wd) < tau_d) A |= 1u << B_EF;
    if (aC >= 0 && focus < 1 && fabs(dC - wd) < tau_d) A |= 1u << B_EC;
    if (flip & (1u << B_EF)) eF = !eF;
    if (flip & (1u << B_EC)) eC = !eC;
    int hin = dF <= wd + hw * focus;
    if (aF >= 0 && focus > 0 && hw * focus > 0 && ha > 0 && !eF && fabs(dF - (wd + hw * focus)) < tau_d) A |= 1u << B_HALO;
    if (flip & (1u << B_HALO)) hin = !hin;
    int h = !eF && hin;
    /* nearest-edge colour (ties: lower local edge index) */
    if (aF2 >= 0 && eF && focus > 0 && d[aF2] - dF < tau_d &&
        m->face_te[4 * f + aF2] != m->face_te[4 * f + aF]) A |= 1u << B_ARGF;
    if (aC2 >= 0 && eC && focus < 1 && d[aC2] - dC < tau_d &&
        m->face_te[4 * f + aC2] != m->face_te[4 * f + aC]) A |= 1u << B_ARGC;
    int cF = aF, cC = aC;
    if ((flip & (1u << B_ARGF)) && aF2 >= 0) cF = aF2;
    if ((flip & (1u << B_ARGC)) && aC2 >= 0) cC = aC2;
    double teF = cF >= 0 ? m->face_te[4 * f + cF] : 0.0, teC = cC >= 0 ? m->face_te[4 * f + cC] : 0.0;
    double CF[3], CC[3], Cf[3];
    for (int a = 0; a < 3; ++a) {
        double lo = st[ST_TF_LO + a], hi = st[ST_TF_HI + a];
        CF[a] = (lo + (hi - lo) * teF) * (1.0 - st[ST_DARKEN] * focus);
        CC[a] = lo + (hi - lo) * teC;
        Cf[a] = lo + (hi - lo) * tf;
    }
    /* Eq. 1 with the focus-edge halo */
    double AF = eF ? 1.0 : (h ? ha : 0.0);
    double PF[3];
    for (int a = 0; a < 3; ++a) PF[a] = eF ? CF[a] : (h ? ha : 0.0);
    double ae = (1.0 - focus) * (double)eC + focus * AF;
    double aeCe[3];
    for (int a = 0; a < 3; ++a) aeCe[a] = (1.0 - focus) * (double)eC * CC[a] + focus * PF[a];
    /* Eq. 2 (accentuation) and Eq. 3 (face opacity) */
    int acc = dAll <= (2.0 / 3.0) * wb;
    double s = st[ST_S];
    double ahat = st[ST_A_LO] + (st[ST_A_HI] - st[ST_A_LO]) * tf;
    double dc = dist < 1.0 ? dist : 1.0;
    double af = ahat * dc * dc * dc * dc;
    if (s != 1.0 && af > 0 && ae < 1.0 && fabs(dAll - (2.0 / 3.0) * wb) < tau_d) A |= 1u << B_ACC;
    if (flip & (1u << B_ACC)) acc = !acc;
    double se = acc ? s : 1.0;
    if (se != 1.0)
        for (int a = 0; a < 3; ++a) {
            Cf[a] *= 1.0 + st[ST_BRIGHT];
            if (Cf[a] > 1.0) Cf[a] = 1.0;
        }
    double afs = se * af;
    if (afs > 1.0) afs = 1.0;
    /* Eq. 4 (premultiplied) */
    for (int a = 0; a < 3; ++a) out->c[a] = aeCe[a] + (1.0 - ae) * afs * Cf[a];
    out->a = ae + (1.0 - ae) * afs;
    /* depth cue in the focus region: desaturate towards the luminance with
       the normalised view depth of the fragment */
    if (st[ST_DESAT] > 0.0) {
        double w = fr->wrow[0] * p[0] + fr->wrow[1] * p[1] + fr->wrow[2] * p[2] + fr->wrow[3];
        double z = (w - fr->w0) / (fr->w1 - fr->w0);
        if (z < 0.0) z = 0.0;
        if (z > 1.0) z = 1.0;
        double sd = st[ST_DESAT] * focus * z;
        double lum = 0.2126 * out->c[0] + 0.7152 * out->c[1] + 0.0722 * out->c[2];
        for (int a = 0; a < 3; ++a) out->c[a] = (1.0 - sd) * out->c[a] + sd * lum;
    }
    if (amb) *amb = A;
}

static void blend(const frag *fs, int64_t n, const double *bg, double *rgba) {
    double C[3] = {0, 0, 0}, A = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = 1.0 - A;
        for (int a = 0; a < 3; ++a) C[a] += t * fs[i].c[a];
        A += t * fs[i].a;
    }
    for (int a = 0; a < 3; ++a) rgba[a] = C[a] + (1.0 - A) * bg[a];
    rgba[3] = A;
}

/* ---------------------------------------------------------------- silhouettes
 * White exterior and interior screen-space silhouettes (Section 4.2, the
 * final look): the depth buffer of the mesh boundary surface (per pixel, the
 * nearest fragment of a face that belongs to one cell only) is searched for
 * sharp edges.  A pixel is a silhouette pixel when it sees the boundary
 * surface and a 4-neighbour inside the image sees none (exterior) or sees it
 * farther than (1 + tau) times its own view depth (interior; view depth
 * ratio = inverse ratio of the depth keys, tau taken as the FP32 value).
 * Silhouette pixels get white of opacity sil_a composited on top:
 * rgb' = (1 - a) rgb + a, A' = a + (1 - a) A.  Needs every pixel of the frame
 * (sample set = all pixels in row-major order). */
static int silhouettes(orc_frame *fr, const double *st, double *rgba) {
    const int64_t W = fr->W, H = fr->H, P = W * H;
    if (P <= 0 || fr->npix != P) return ORC_EINVAL;
    for (int64_t s = 0; s < P; ++s)
        if (fr->pix[s] != s) return ORC_EINVAL;
    const orc_mesh *m = fr->m;
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);  /* boundary surface key, 0: none */
    uint8_t *sil = (uint8_t *)calloc((size_t)P, 1);
    if (!key || !sil) { free(key); free(sil); return ORC_ENOMEM; }
    for (int64_t s = 0; s < P; ++s) {
        key[s] = 0;
        for (uint64_t k = fr->off[s]; k < fr->off[s + 1]; ++k) {  /* sorted: the first boundary fragment is the nearest */
            uint64_t r = fr->rec[k];
            if (m->face_bnd[(r & 0xffffffffu) >> 1]) { key[s] = ORC_KMAX - (int64_t)(r >> 32); break; }
        }
    }
    const double tau = (double)(float)st[ST_SIL_TAU];
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            int64_t kp = key[y * W + x];
            if (kp == 0) continue;
            const int64_t nb[4][2] = {{x - 1, y}, {x + 1, y}, {x, y - 1}, {x, y + 1}};
            for (int q = 0; q < 4; ++q) {
                int64_t nx = nb[q][0], ny = nb[q][1];
                if (nx < 0 || ny < 0 || nx >= W || ny >= H) continue;
                int64_t kn = key[ny * W + nx];
                if (kn == 0 || (double)kp > (1.0 + tau) * (double)kn) { sil[y * W + x] = 1; break; }
            }
        }
    const double a = st[ST_SIL_A];
    for (int64_t s = 0; s < P; ++s) {
        if (!sil[s]) continue;
        double *px = rgba + 4 * s;
        for (int c = 0; c < 3; ++c) px[c] = (1.0 - a) * px[c] + a;
        px[3] = a + (1.0 - a) * px[3];
        if (fr->cand_off)
            for (int64_t c = fr->cand_off[s]; c < fr->cand_off[s + 1]; ++c) {
                double *q = fr->cand + 4 * c;
                for (int ch = 0; ch < 3; ++ch) q[ch] = (1.0 - a) * q[ch] + a;
                q[3] = a + (1.0 - a) * q[3];
            }
    }
    free(key); free(sil);
    return ORC_OK;
}

#define ORC_MAX_COMBOS 64

/* Shade + composite every sample pixel.  ncand[s] = 0: unambiguous;
 * > 0: number of alternative results stored for the pixel; -1: too many
 * ambiguous fragments to enumerate (pixel excluded from strict checks). */
int orc_frame_shade(orc_frame *fr, const double *hot, const double *st, double *rgba, int32_t *ncand) {
    if (!(hot[3] > 0.0)) return ORC_EINVAL;
    int64_t np = fr->npix;
    free(fr->cand_off); free(fr->cand);
    fr->cand_off = (int64_t *)calloc(np + 1, 8);
    double **pc = (double **)calloc(np, sizeof(double *));
    const double *bg = st + ST_BG;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < np; ++s) {
        int64_t n = fr->count[s];
        int64_t i = fr->pix[s] % fr->W, j = fr->pix[s] / fr->W;
        frag *fs = (frag *)malloc(sizeof(frag) * (n + 1));
        unsigned *am = (unsigned *)malloc(sizeof(unsigned) * (n + 1));
        int64_t combos = 1;
        for (int64_t k = 0; k < n; ++k) {
            shade(fr, i, j, fr->rec[fr->off[s] + k] & 0xffffffffu, hot, st, 0, &fs[k], &am[k]);
            if (am[k]) {
                int bits = __builtin_popcount(am[k]);
                if (combos <= ORC_MAX_COMBOS) combos <<= bits;
            }
        }
        blend(fs, n, bg, rgba + 4 * s);
        ncand[s] = 0;
        if (combos > ORC_MAX_COMBOS) {
            ncand[s] = -1;
        } else if (combos > 1) {
            /* enumerate every combination of the ambiguous predicates */
            double *cands = (double *)malloc(sizeof(double) * 4 * combos);
            frag *alt = (frag *)malloc(sizeof(frag) * (n + 1));
            for (int64_t cmb = 0; cmb < combos; ++cmb) {
                int64_t rest = cmb;
                memcpy(alt, fs, sizeof(frag) * n);
                for (int64_t k = 0; k < n; ++k) {
                    if (!am[k]) continue;
                    int bits = __builtin_popcount(am[k]);
                    int64_t pick = rest & ((1 << bits) - 1);
                    rest >>= bits;
                    unsigned sub = 0;
                    int bi = 0;
                    for (int b = 0; b < 32; ++b)
                        if (am[k] & (1u << b)) { if (pick & (1 << bi)) sub |= 1u << b; ++bi; }
                    if (sub) shade(fr, i, j, fr->rec[fr->off[s] + k] & 0xffffffffu, hot, st, sub, &alt[k], NULL);
                }
                blend(alt, n, bg, cands + 4 * cmb);
            }
            free(alt);
            pc[s] = cands;
            ncand[s] = (int32_t)combos;
        }
        free(fs); free(am);
    }
    for (int64_t s = 0; s < np; ++s) fr->cand_off[s + 1] = fr->cand_off[s] + (ncand[s] > 0 ? ncand[s] : 0);
    fr->ncand = fr->cand_off[np];
    fr->cand = (double *)malloc(sizeof(double) * 4 * (fr->ncand + 1));
    for (int64_t s = 0; s < np; ++s)
        if (pc[s]) { memcpy(fr->cand + 4 * fr->cand_off[s], pc[s], sizeof(double) * 4 * ncand[s]); free(pc[s]); }
    free(pc);
    if (st[ST_SIL_A] > 0.0) return silhouettes(fr, st, rgba);
    return ORC_OK;
}

int64_t orc_frame_ncand(const orc_frame *fr) { return fr->ncand; }
void orc_frame_cands(const orc_frame *fr, int64_t *cand_off, double *cand) {
    if (cand_off) memcpy(cand_off, fr->cand_off, 8 * (fr->npix + 1));
    if (cand) memcpy(cand, fr->cand, sizeof(double) * 4 * fr->ncand);
}

/* Single-fragment access for the closed-form pins. */
void orc_shade_one(const orc_frame *fr, int64_t i, int64_t j, uint32_t tri, const double *hot,
                   const double *st, unsigned flip, double *out5) {
    frag fo;
    unsigned amb = 0;
    shade(fr, i, j, tri, hot, st, flip, &fo, &amb);
    out5[0] = fo.c[0]; out5[1] = fo.c[1]; out5[2] = fo.c[2]; out5[3] = fo.a; out5[4] = (double)amb;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the oracle's parallel loops from here on (n >= 1). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- learned tail
 * Head/tail split of a sorted list (the approximate-compositing direction of
 * Section 8): the first K fragments are blended exactly (head); the tail
 * (fragments K..n-1) is summarised by 9 features computed from a cheap proxy
 * shading, and its exact composite is the regression target.
 *   proxy fragment: alpha~ = ahat(tbar) * min(|c_face - h| / r, 1)^4,
 *                   colour~ = TF(tbar), with c_face the mean of the face's
 *                   corners and tbar the mean corner importance;
 *   depth z = (w - w0) / (w1 - w0) clamped to [0,1], w = 2^20 / key the view
 *   depth of the fragment, [w0, w1] the view-depth range of the mesh bbox;
 *   features: log1p(n_tail), sum alpha~, sum alpha~ z^k / sum alpha~ (k=1,2),
 *   the premultiplied RGBA of the proxies composited front to back in depth
 *   order (4), and z of the first tail fragment.
 * Outputs per sample pixel with n > K (others get has = 0):
 *   head[4] (premultiplied head composite), feat[9], target[4] (exact
 *   premultiplied tail composite). */
int orc_frame_tail(orc_frame *fr, const double *hot, const double *st, int K, double w0, double w1,
                   double *head, double *feat, double *target, uint8_t *has) {
    if (!(hot[3] > 0.0) || K < 1 || !(w1 > w0)) return ORC_EINVAL;
    const orc_mesh *m = fr->m;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < fr->npix; ++s) {
        int64_t n = fr->count[s];
        int64_t i = fr->pix[s] % fr->W, j = fr->pix[s] / fr->W;
        has[s] = n > K;
        for (int a = 0; a < 4; ++a) head[4 * s + a] = target[4 * s + a] = 0.0;
        for (int a = 0; a < 9; ++a) feat[9 * s + a] = 0.0;
        if (n <= K) continue;
        double Ch[3] = {0, 0, 0}, Ah = 0.0, Ct[3] = {0, 0, 0}, At = 0.0;
        double sa = 0.0, sz[2] = {0, 0}, P[3] = {0, 0, 0}, PA = 0.0, zf = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            uint64_t r = fr->rec[fr->off[s] + k];
            uint32_t tri = (uint32_t)(r & 0xffffffffu);
            frag f;
            shade(fr, i, j, tri, hot, st, 0, &f, NULL);
            if (k < K) {
                double t = 1.0 - Ah;
                for (int a = 0; a < 3; ++a) Ch[a] += t * f.c[a];
                Ah += t * f.a;
                continue;
            }
            double t = 1.0 - At;
            for (int a = 0; a < 3; ++a) Ct[a] += t * f.c[a];
            At += t * f.a;
            /* proxy shading of the tail fragment: its face's centre and mean
               corner importance */
            int64_t fc = tri >> 1;
            double ctr[3] = {0, 0, 0}, tbar = 0.0;
            for (int c = 0; c < 4; ++c) {
                int64_t v = m->face_v[4 * fc + c];
                for (int a = 0; a < 3; ++a) ctr[a] += 0.25 * (double)m->pos_q[3 * v + a] / ORC_POS_SCALE;
                tbar += 0.25 * m->t_v[v];
            }
            double dx = ctr[0] - hot[0], dy = ctr[1] - hot[1], dz = ctr[2] - hot[2];
            double dist = sqrt(dx * dx + dy * dy + dz * dz) / hot[3];
            if (dist > 1.0) dist = 1.0;
            double al = (st[ST_A_LO] + (st[ST_A_HI] - st[ST_A_LO]) * tbar) * dist * dist * dist * dist;
            double key = (double)(ORC_KMAX - (int64_t)(r >> 32));
            double w = 1048576.0 / key;
            double z = (w - w0) / (w1 - w0);
            if (z < 0.0) z = 0.0;
            if (z > 1.0) z = 1.0;
            if (k == K) zf = z;
            sa += al;
            sz[0] += al * z;
            sz[1] += al * z * z;
            /* front-to-back composite of the proxies */
            double tp = 1.0 - PA;
            for (int a = 0; a < 3; ++a) P[a] += tp * al * (st[ST_TF_LO + a] + (st[ST_TF_HI + a] - st[ST_TF_LO + a]) * tbar);
            PA += tp * al;
        }
        for (int a = 0; a < 3; ++a) { head[4 * s + a] = Ch[a]; target[4 * s + a] = Ct[a]; }
        head[4 * s + 3] = Ah;
        target[4 * s + 3] = At;
        double *F = feat + 9 * s;
        F[0] = log1p((double)(n - K));
        F[1] = sa;
        F[2] = sa > 0.0 ? sz[0] / sa : 0.0;
        F[3] = sa > 0.0 ? sz[1] / sa : 0.0;
        for (int a = 0; a < 3; ++a) F[4 + a] = P[a];
        F[7] = PA;
        F[8] = zf;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- approximate resolves
 * Two order-independent approximations of the sorted blend, on the same
 * fragment lists (the paper's future work names approximate transparency
 * without per-pixel sorting; these are the published non-learned methods):
 *
 * method 1, multi-layer alpha blending (Salvi and Vaidyanathan, 2014):
 *   k blending nodes (premultiplied colour, transmittance, depth key) per
 *   pixel, kept in depth order.  Fragments arrive in primitive order
 *   (ascending triangle id); each is inserted at its depth (after nodes of
 *   equal depth); when k+1 nodes exist the last two merge:
 *   (c, T) = (c_a + T_a c_b, T_a T_b), depth of the front one.  The nodes are
 *   then blended front to back.  With k >= n this is the exact blend.
 *
 * method 2, moment-based order-independent transparency (Muenstermann,
 *   Krumpen, Klein, Peters, 2018) with four power moments:
 *   absorbance a_i = -ln(1 - alpha_i) (alpha clamped to 1 - 1e-6), warped
 *   depth x_i = 2 clamp((w_i - w0) / (w1 - w0), 0, 1) - 1, moments
 *   b_j = sum a_i x_i^j (j = 0..4).  For each fragment the absorbance in
 *   front of it is b_0 F(x_i), F from the 4-moment (Hamburger) bound: the
 *   normalised moments m_j = b_j / b_0, blended towards (0, 0.375, 0, 0.375)
 *   by beta, are matched by a distribution on three points {x, z2, z3}; z2,
 *   z3 are the roots of P(t) / (t - x) where P is the monic cubic with
 *   E[P(X)] = E[X P(X)] = 0 and P(x) = 0; weights by Lagrange
 *   interpolation; F = (weight of the support points in front of x)
 *   + eta * (weight at x).  Then C = sum T_i alpha_i c_i with
 *   T_i = exp(-b_0 F(x_i)), rescaled so that the total opacity is the exact
 *   1 - exp(-b_0).
 */
typedef struct { double c[3], T; int64_t z; } mlab_node;

static void mlab_resolve(const double *fc, const double *fa, const int64_t *fz, int64_t n, int k, double *out) {
    mlab_node nd[9];
    int cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        mlab_node x;
        for (int a = 0; a < 3; ++a) x.c[a] = fc[3 * i + a];
        x.T = 1.0 - fa[i];
        x.z = fz[i];
        int p = cnt;
        while (p > 0 && nd[p - 1].z > x.z) --p;  /* after nodes of equal depth */
        for (int q = cnt; q > p; --q) nd[q] = nd[q - 1];
        nd[p] = x;
        ++cnt;
        if (cnt > k) {  /* merge the last two */
            mlab_node *a = &nd[cnt - 2], *b = &nd[cnt - 1];
            for (int c = 0; c < 3; ++c) a->c[c] += a->T * b->c[c];
            a->T *= b->T;
            --cnt;
        }
    }
    double C[3] = {0, 0, 0}, T = 1.0;
    for (int q = 0; q < cnt; ++q) {
        for (int a = 0; a < 3; ++a) C[a] += T * nd[q].c[a];
        T *= nd[q].T;
    }
    for (int a = 0; a < 3; ++a) out[a] = C[a];
    out[3] = 1.0 - T;
}

/* fraction of the total absorbance in front of x, from normalised moments m[1..4] */
static double moment_bound(const double *m, double x, double eta) {
    /* P(t) = t^3 + p2 t^2 + p1 t + p0 with E[P] = 0, E[X P] = 0, P(x) = 0 */
    double A[3][4] = {{1.0, m[1], m[2], -m[3]}, {m[1], m[2], m[3], -m[4]}, {1.0, x, x * x, -x * x * x}};
    for (int c = 0; c < 3; ++c) {  /* Gaussian elimination with partial pivoting */
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c)
            for (int q = 0; q < 4; ++q) { double t = A[c][q]; A[c][q] = A[piv][q]; A[piv][q] = t; }
        if (A[c][c] == 0.0) return eta;  /* degenerate: no information */
        for (int r = c + 1; r < 3; ++r) {
            double f = A[r][c] / A[c][c];
            for (int q = c; q < 4; ++q) A[r][q] -= f * A[c][q];
        }
    }
    double p[3];
    for (int c = 2; c >= 0; --c) {
        double s = A[c][3];
        for (int q = c + 1; q < 3; ++q) s -= A[c][q] * p[q];
        p[c] = s / A[c][c];
    }
    /* P(t) / (t - x) = t^2 + (p2 + x) t + (p1 + x (p2 + x)) */
    double bq = p[2] + x, cq = p[1] + x * bq;
    double disc = bq * bq - 4.0 * cq;
    if (disc < 0.0) disc = 0.0;
    double sq = sqrt(disc);
    double z2 = 0.5 * (-bq - sq), z3 = 0.5 * (-bq + sq);
    /* weights by Lagrange interpolation: w_k = E[prod_{l != k} (X - x_l) / (x_k - x_l)] */
    double d2 = (z2 - x) * (z2 - z3), d3 = (z3 - x) * (z3 - z2);
    double w2 = d2 != 0.0 ? (m[2] - m[1] * (x + z3) + x * z3) / d2 : 0.0;
    double w3 = d3 != 0.0 ? (m[2] - m[1] * (x + z2) + x * z2) / d3 : 0.0;
    double w1 = 1.0 - w2 - w3;
    double F = (z2 < x ? w2 : 0.0) + (z3 < x ? w3 : 0.0) + eta * w1;
    if (F < 0.0) F = 0.0;
    if (F > 1.0) F = 1.0;
    return F;
}

static void mboit_resolve(const double *fc, const double *fa, const double *fx, int64_t n, double beta, double eta,
                          double *out) {
    double b[5] = {0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        double al = fa[i] < 1.0 - 1e-6 ? fa[i] : 1.0 - 1e-6;
        double a = -log1p(-al), xp = 1.0;
        for (int j = 0; j < 5; ++j) { b[j] += a * xp; xp *= fx[i]; }
    }
    for (int a = 0; a < 4; ++a) out[a] = 0.0;
    if (!(b[0] > 0.0)) return;
    const double ref[5] = {1.0, 0.0, 0.375, 0.0, 0.375};
    double m[5];
    for (int j = 0; j < 5; ++j) m[j] = (1.0 - beta) * (b[j] / b[0]) + beta * ref[j];
    double C[3] = {0, 0, 0}, W = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double T = exp(-b[0] * moment_bound(m, fx[i], eta));
        for (int a = 0; a < 3; ++a) C[a] += T * fc[3 * i + a];
        W += T * fa[i];
    }
    double A = -expm1(-b[0]);
    double s = W > 0.0 ? A / W : 0.0;
    for (int a = 0; a < 3; ++a) out[a] = C[a] * s;
    out[3] = A;
}

static int cmp_tri(const void *a, const void *b) {
    uint32_t x = (uint32_t)(*(const uint64_t *)a & 0xffffffffu), y = (uint32_t)(*(const uint64_t *)b & 0xffffffffu);
    return x < y ? -1 : x > y;
}

/* method 1: param = k (1..8); method 2: beta, eta (param unused).  rgba: final
 * colour over the background, as orc_frame_shade. */
int orc_frame_approx(orc_frame *fr, const double *hot, const double *st, int method, int param, double beta,
                     double eta, double w0, double w1, double *rgba) {
    if (!(hot[3] > 0.0) || (method != 1 && method != 2) || (method == 1 && (param < 1 || param > 8)) ||
        !(w1 > w0))
        return ORC_EINVAL;
    const double *bg = st + ST_BG;
    int err = 0;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < fr->npix; ++s) {
        int64_t n = fr->count[s];
        int64_t i = fr->pix[s] % fr->W, j = fr->pix[s] / fr->W;
        double out[4] = {0, 0, 0, 0};
        if (n > 0) {
            uint64_t *r = (uint64_t *)malloc(sizeof(uint64_t) * n);
            double *fc = (double *)malloc(sizeof(double) * 3 * n), *fa = (double *)malloc(sizeof(double) * n);
            double *fx = (double *)malloc(sizeof(double) * n);
            int64_t *fz = (int64_t *)malloc(sizeof(int64_t) * n);
            if (!r || !fc || !fa || !fx || !fz) {
                #pragma omp atomic write
                err = 1;
            } else {
                memcpy(r, fr->rec + fr->off[s], sizeof(uint64_t) * n);
                if (method == 1) qsort(r, (size_t)n, sizeof(uint64_t), cmp_tri);  /* primitive order */
                for (int64_t q = 0; q < n; ++q) {
                    frag f;
                    shade(fr, i, j, r[q] & 0xffffffffu, hot, st, 0, &f, NULL);
                    for (int a = 0; a < 3; ++a) fc[3 * q + a] = f.c[a];
                    fa[q] = f.a;
                    fz[q] = (int64_t)(r[q] >> 32);
                    double w = 1048576.0 / (double)(ORC_KMAX - (int64_t)(r[q] >> 32));
                    double z = (w - w0) / (w1 - w0);
                    if (z < 0.0) z = 0.0;
                    if (z > 1.0) z = 1.0;
                    fx[q] = 2.0 * z - 1.0;
                }
                if (method == 1) mlab_resolve(fc, fa, fz, n, param, out);
                else mboit_resolve(fc, fa, fx, n, beta, eta, out);
            }
            free(r); free(fc); free(fa); free(fx); free(fz);
        }
        for (int a = 0; a < 3; ++a) rgba[4 * s + a] = out[a] + (1.0 - out[3]) * bg[a];
        rgba[4 * s + 3] = out[3];
    }
    return err ? ORC_ENOMEM : ORC_OK;
}
