// geom.hip -- geometry half of the per-frame path on gfx950: exact integer
// vertex transform and snap, triangle binning to screen tiles, the coverage
// count, the prefix scan, pass planning and the fragment-list fill.
//
// The paper renders every hex face as two triangles and appends one fragment
// per covered pixel to a per-pixel list (Section 4, Section 6).  Here the
// rasteriser is an integer edge-function test over screen tiles (one
// workgroup per tile, one lane per pixel), and the lists are built in two
// passes over the same bins -- count, exclusive scan, fill -- into one
// contiguous 8-byte record per fragment, instead of atomically linked nodes.
#include "kern.h"

namespace hexfc {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ long long floordiv_pos(long long n, long long d) {  // d > 0
    long long q = n / d;
    long long r = n - q * d;
    return (r < 0) ? q - 1 : q;
}

// Vertex transform (exact): clip = M_q (X_q, 2^16); screen position with 4
// sub-pixel bits, round half up; inverse depth q = floor(2^56 / w_q).
__global__ void __launch_bounds__(256) k_transform(const int4 *__restrict__ posq, int64_t V, int64_t NVV,
                                                   const ViewParams *__restrict__ views, int W, int H,
                                                   VertRec *__restrict__ vert, int4 *__restrict__ vscr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NVV) return;
    const int64_t view = i / V, v = i - view * V;
    const Mat3q &M = views[view].M;
    int4 p = posq[v];
    long long X = p.x, Y = p.y, Z = p.z, O = 65536;
    long long cx = M.m[0][0] * X + M.m[0][1] * Y + M.m[0][2] * Z + M.m[0][3] * O;
    long long cy = M.m[1][0] * X + M.m[1][1] * Y + M.m[1][2] * Z + M.m[1][3] * O;
    long long cw = M.m[2][0] * X + M.m[2][1] * Y + M.m[2][2] * Z + M.m[2][3] * O;
    int4 out = make_int4(0, 0, 0, 0);
    if (cw < W_NEAR_Q) {
        out.w = 1;
    } else {
        long long d = 2 * cw;
        long long sx = floordiv_pos((cx + cw) * (long long)(W * SUB) + cw, d);
        long long sy = floordiv_pos((cw - cy) * (long long)(H * SUB) + cw, d);
        if (sx >= GUARD || sx <= -GUARD || sy >= GUARD || sy <= -GUARD) {
            out.w = 2;
        } else {
            out.x = (int)sx;
            out.y = (int)sy;
            out.z = (int)(QNUM / cw);
        }
    }
    vert[i].scr = out;  // for shading
    vscr[i] = out;      // dense copy for the rasteriser
}

// Triangle t of the face list: corners (c0,c1,c2) or (c0,c2,c3).
__device__ __forceinline__ void tri_ids(const int4 c, int t, int &a, int &b, int &d) {
    a = c.x;
    b = t ? c.z : c.y;
    d = t ? c.w : c.z;
}

// Screen-tile range of a triangle's pixel-centre bounding box; false when the
// triangle is culled (flagged vertex, zero snapped area, nothing on screen).
__device__ __forceinline__ bool tri_tile_range(const int4 a, const int4 b, const int4 d, const Tiling &tl, int &tx0,
                                               int &tx1, int &ty0, int &ty1) {
    static_assert(SUB == 16, "sub-pixel shifts");
    if (a.w | b.w | d.w) return false;
    long long area = (long long)(b.x - a.x) * (d.y - a.y) - (long long)(b.y - a.y) * (d.x - a.x);
    if (area == 0) return false;
    int xmin = min(a.x, min(b.x, d.x)), xmax = max(a.x, max(b.x, d.x));
    int ymin = min(a.y, min(b.y, d.y)), ymax = max(a.y, max(b.y, d.y));
    // pixel i is a candidate iff xmin <= 16 i + 8 <= xmax: i from
    // ceil((xmin - 8) / 16) to floor((xmax - 8) / 16) (arithmetic shifts floor)
    int i0 = -((8 - xmin) >> 4);
    int i1 = (xmax - 8) >> 4;
    int j0 = -((8 - ymin) >> 4);
    int j1 = (ymax - 8) >> 4;
    i0 = max(i0, 0);
    j0 = max(j0, 0);
    i1 = min(i1, tl.W - 1);
    j1 = min(j1, tl.H - 1);
    if (i0 > i1 || j0 > j1) return false;
    // (tile sides are powers of two)
    const int sx = __builtin_ctz((unsigned)tl.TW), sy = __builtin_ctz((unsigned)tl.TH);
    tx0 = i0 >> sx;
    tx1 = i1 >> sx;
    ty0 = j0 >> sy;
    ty1 = j1 >> sy;
    return true;
}

// Triangle binning, one lane per face (its two triangles share the corner
// loads).  Each triangle adds itself to every screen tile its pixel-centre
// bounding box overlaps.  Consecutive faces are mesh neighbours, so the 64
// faces of a wave hit few distinct tiles: the lanes that hit the same tile
// are merged into one atomic (leader election by ballot), and each gets its
// rank inside the merged group.  The grouping uses ballots only; the group
// leaders then issue their atomics together, so their latencies overlap.
// The order of a tile's entries is not fixed; nothing downstream depends on
// it.
//
// The counting pass keeps, for the first BIN_SLOTS tiles of every face, the
// slot it reserved in the tile (counter `lo`); the scatter pass writes those
// entries there with no atomic.  A face's further tiles reserve from a second
// counter (`hi`) and are placed by atomics in the scatter pass, after the
// tile's `lo` entries.
constexpr int BIN_SLOTS = 4;

template <bool SCATTER>
__global__ void __launch_bounds__(256) k_tri_bin(const int4 *__restrict__ face_c,
                                                 const uint32_t *__restrict__ face_ord, int64_t F, int64_t NVF,
                                                 const int4 *__restrict__ vscr, int64_t V, Tiling tl,
                                                 uint32_t *__restrict__ tile_ctr, const uint64_t *__restrict__ tile_off,
                                                 uint32_t *__restrict__ bins, uint64_t cap,
                                                 int4 *__restrict__ fscr, uint32_t *__restrict__ bslot,
                                                 const uint32_t *__restrict__ tile_lo, int64_t NT,
                                                 int4 *__restrict__ frange) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (view, position in binning order)
    // (view = i / F: none for one view, in 32 bits while the views' faces count below 2^32)
    const int64_t view = (NVF <= F || i >= NVF) ? 0
                         : NVF <= 0xffffffffll ? (int64_t)((uint32_t)i / (uint32_t)F)
                                               : i / F;
    const int64_t fo = i - view * F;
    // bin entries name triangles by binning position (2 fo + t): the count and
    // fill passes then read the screen vertices in binning order too; the fill
    // takes the canonical face id for the records from the w of corner 0
    const int64_t f = fo;
    int r0[4] = {0, -1, 0, -1}, r1[4] = {0, -1, 0, -1};  // tile ranges of triangles 0 and 1: x0, x1, y0, y1
    bool ok0 = false, ok1 = false;
    if (SCATTER && i < NVF) {
        // the count pass stored both triangles' tile ranges (16 B instead of
        // the 64 B of screen vertices they come from)
        const int4 rg = frange[i];
        ok0 = rg.x != -1;
        ok1 = rg.z != -1;
        r0[0] = rg.x & 0xffff;
        r0[1] = (int)((uint32_t)rg.x >> 16);
        r0[2] = rg.y & 0xffff;
        r0[3] = (int)((uint32_t)rg.y >> 16);
        r1[0] = rg.z & 0xffff;
        r1[1] = (int)((uint32_t)rg.z >> 16);
        r1[2] = rg.w & 0xffff;
        r1[3] = (int)((uint32_t)rg.w >> 16);
    } else if (i < NVF) {
        int4 p0, p1, p2, p3;
        int4 *fs = fscr + 4 * i;  // (view, binning position) record of the four screen vertices
        {
            const int4 c = face_c[fo];
            const int4 *vs = vscr + view * V;
            p0 = vs[c.x];
            p1 = vs[c.y];
            p2 = vs[c.z];
            p3 = vs[c.w];
            // corner 0's flag gives way to the canonical face id (-1: culled corner)
            fs[0] = make_int4(p0.x, p0.y, p0.z, p0.w ? -1 : (int)face_ord[fo]);
            fs[1] = p1;
            fs[2] = p2;
            fs[3] = p3;
        }
        ok0 = tri_tile_range(p0, p1, p2, tl, r0[0], r0[1], r0[2], r0[3]);
        ok1 = tri_tile_range(p0, p2, p3, tl, r1[0], r1[1], r1[2], r1[3]);
        frange[i] = make_int4(ok0 ? r0[0] | (r0[1] << 16) : -1, ok0 ? r0[2] | (r0[3] << 16) : 0,
                              ok1 ? r1[0] | (r1[1] << 16) : -1, ok1 ? r1[2] | (r1[3] << 16) : 0);
    }
    const int64_t tile0 = view * tl.ntiles;
    // union of the two ranges; a tile of it takes the face's triangles that overlap it
    int u[4] = {0, -1, 0, -1};
    if (ok0 || ok1) {
        u[0] = min(ok0 ? r0[0] : r1[0], ok1 ? r1[0] : r0[0]);
        u[1] = max(ok0 ? r0[1] : r1[1], ok1 ? r1[1] : r0[1]);
        u[2] = min(ok0 ? r0[2] : r1[2], ok1 ? r1[2] : r0[2]);
        u[3] = max(ok0 ? r0[3] : r1[3], ok1 ? r1[3] : r0[3]);
    }
    const int nx = u[1] - u[0] + 1;
    const int n = (ok0 || ok1) ? nx * (u[3] - u[2] + 1) : 0;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int kx = -1, ky = 0;  // tile k of the range, row-major: (u[0] + kx, u[2] + ky)
    for (int k = 0; __any(k < n); ++k) {
        if (++kx >= nx) {
            kx = 0;
            ++ky;
        }
        int64_t tile = -1;
        bool h0 = false, h1 = false;
        if (k < n) {
            const int x = u[0] + kx, y = u[2] + ky;
            h0 = ok0 && x >= r0[0] && x <= r0[1] && y >= r0[2] && y <= r0[3];
            h1 = ok1 && x >= r1[0] && x <= r1[1] && y >= r1[2] && y <= r1[3];
            if (h0 || h1) tile = tile0 + (int64_t)y * tl.ntx + x;
        }
        if (SCATTER && k < BIN_SLOTS) {  // (k is the same on every lane)
            if (tile >= 0) {
                uint64_t idx = tile_off[tile] + bslot[i * BIN_SLOTS + k];
                if (h0) {
                    if (idx < cap) bins[idx] = (uint32_t)(2 * f);
                    ++idx;
                }
                if (h1 && idx < cap) bins[idx] = (uint32_t)(2 * f + 1);
            }
            continue;
        }
        // group the lanes by tile (ballots only), then one atomic per group,
        // all groups' atomics in flight together
        unsigned long long pend = __ballot(tile >= 0);
        int my_leader = lane;
        unsigned my_rank = 0, lead_count = 0;
        while (pend) {
            const int leader = __ffsll((long long)pend) - 1;
            const int64_t lead_tile = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(tile >> 32), leader)
                                                 << 32) |
                                                (uint32_t)__builtin_amdgcn_readlane((int)tile, leader));
            const bool mine = tile == lead_tile;
            const unsigned long long m0 = __ballot(mine && h0), m1 = __ballot(mine && h1);
            if (mine) {
                my_leader = leader;
                my_rank = (unsigned)(__popcll(m0 & below) + __popcll(m1 & below));
            }
            if (lane == leader) lead_count = (unsigned)(__popcll(m0) + __popcll(m1));
            pend &= ~__ballot(mine);
        }
        unsigned base = 0;
        // count pass: the first slots' counter, or the second one past them
        uint32_t *ctr = (SCATTER || k < BIN_SLOTS) ? tile_ctr : tile_ctr + NT;
        if (tile >= 0 && my_leader == lane) base = atomicAdd(&ctr[tile], lead_count);
        base = __shfl(base, my_leader);
        if (!SCATTER && tile >= 0 && k < BIN_SLOTS) bslot[i * BIN_SLOTS + k] = base + my_rank;
        if (SCATTER && tile >= 0) {
            uint64_t idx = tile_off[tile] + tile_lo[tile] + base + my_rank;
            if (h0) {
                if (idx < cap) bins[idx] = (uint32_t)(2 * f);
                ++idx;
            }
            if (h1 && idx < cap) bins[idx] = (uint32_t)(2 * f + 1);
        }
    }
}

// ------------------------------------------------------------------ per-tile triangle setup

// Coverage of one triangle over one tile, as three edge tests
//   E'(dx, dy) = c + a*dx + b*dy >= 0
// in int32, where (dx, dy) is the sub-pixel offset of the pixel centre from
// the tile's first pixel centre.  The half-open rule is folded into c (-1 on
// edges that do not own their centres).  An edge that passes everywhere on
// the tile becomes (0,0,0); a triangle that misses the tile gets c = -1.
struct CovSetup {
    int a0, b0, c0, a1;
    int b1, c1, a2, b2;
    int c2;
    int pad0;  // candidate pixel box in the tile: x0 | x1 << 8 | y0 << 16 | y1 << 24
    int pad1;  // candidate rows of the box (0: the triangle misses the tile)
    int pad2;
};
// Depth key of the same triangle: N(dx, dy) = n0 + na*dx + nb*dy (exact
// int64), key = floor(N / D) with D = twice the oriented area.
struct KeySetup {
    long long n0, na, nb, D;
    double rD;
    unsigned tri;
    unsigned pad;
};

// Twice the oriented area of the triangle v, and its three edge tests over
// the tile (see CovSetup), in an integer type T that holds their products;
// returns true if an edge rejects the whole tile.
template <class T>
__device__ __forceinline__ T tri_area(const int4 (&v)[3]) {
    return (T)(v[1].x - v[0].x) * (v[2].y - v[0].y) - (T)(v[1].y - v[0].y) * (v[2].x - v[0].x);
}
struct TriEdges {
    int a0, b0, c0, a1, b1, c1, a2, b2, c2;
    bool reject;
};
template <class T>
__device__ __forceinline__ void edge_test(const int4 &p, const int4 &q, int ox, int oy, int ex, int ey, int &ea,
                                          int &eb, int &ec, bool &reject) {
    const int A = p.y - q.y, B = q.x - p.x;  // E(x,y) = A (x - px) + B (y - py)
    const T Eo = (T)A * (ox - p.x) + (T)B * (oy - p.y);
    const bool owned = (A > 0) || (A == 0 && B > 0);  // dy < 0, or dy == 0 and dx > 0
    const T Eb = owned ? Eo : Eo - 1;
    const T ax = (T)A * ex, by = (T)B * ey;
    const T emin = Eb + min((T)0, ax) + min((T)0, by);
    const T emax = Eb + max((T)0, ax) + max((T)0, by);
    if (emax < 0) reject = true;
    const bool all = emin >= 0;  // passes on the whole tile
    ea = all ? 0 : A;
    eb = all ? 0 : B;
    ec = all ? 0 : (int)Eb;
}
template <class T>
__device__ __forceinline__ TriEdges tri_edges(const int4 &v0, const int4 &v1, const int4 &v2, int ox, int oy, int ex,
                                              int ey) {
    TriEdges e;
    e.reject = false;
    edge_test<T>(v0, v1, ox, oy, ex, ey, e.a0, e.b0, e.c0, e.reject);
    edge_test<T>(v1, v2, ox, oy, ex, ey, e.a1, e.b1, e.c1, e.reject);
    edge_test<T>(v2, v0, ox, oy, ex, ey, e.a2, e.b2, e.c2, e.reject);
    return e;
}

__device__ __forceinline__ void tri_setup(const int4 *__restrict__ fscr, uint32_t tri, int ox, int oy, int ex,
                                          int ey, CovSetup &cs) {
    const int4 *fs = fscr + 4 * (size_t)(tri >> 1);  // the face's four screen vertices
    const int t1 = (int)(tri & 1);
    int4 v[3] = {fs[0], fs[1 + t1], fs[2 + t1]};
    cs.pad0 = cs.pad1 = cs.pad2 = 0;
    // Vertices within 2^13 sub-pixels of the tile origin (nearly every
    // triangle) keep every product below in 32 bits: edge deltas below 2^14,
    // offsets below 2^13, extents ex, ey below 2^9, so |E| < 2^28 + 2^24.
    // The wave takes the 64-bit path only if one of its triangles needs it.
    int reach = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) reach = max(reach, max(abs(v[k].x - ox), abs(v[k].y - oy)));
    const bool narrow = !__any(!(reach < (1 << 13) && ex < (1 << 9) && ey < (1 << 9)));
    long long area = narrow ? (long long)tri_area<int>(v) : tri_area<long long>(v);
    if (v[0].w < 0 || (v[1].w | v[2].w) || area == 0) {  // (culled triangles are never binned)
        cs.a0 = cs.b0 = cs.a1 = cs.b1 = cs.a2 = cs.b2 = 0;
        cs.c0 = -1;
        cs.c1 = cs.c2 = 0;
        return;
    }
    if (area < 0) {  // orient so the interior is on the left of every edge
        int4 t = v[1];
        v[1] = v[2];
        v[2] = t;
        area = -area;
    }
    const TriEdges e = narrow ? tri_edges<int>(v[0], v[1], v[2], ox, oy, ex, ey)
                              : tri_edges<long long>(v[0], v[1], v[2], ox, oy, ex, ey);
    bool reject = e.reject;
    // candidate pixels of the tile: centres inside the triangle's bounding box
    const int mnx = min(v[0].x, min(v[1].x, v[2].x)), mxx = max(v[0].x, max(v[1].x, v[2].x));
    const int mny = min(v[0].y, min(v[1].y, v[2].y)), mxy = max(v[0].y, max(v[1].y, v[2].y));
    const int x0 = max(0, -((ox - mnx) >> 4)), x1 = min(ex / SUB, (mxx - ox) >> 4);  // ceil / floor of /16
    const int y0 = max(0, -((oy - mny) >> 4)), y1 = min(ey / SUB, (mxy - oy) >> 4);
    if (x0 > x1 || y0 > y1) reject = true;
    if (reject) {
        cs.a0 = cs.b0 = cs.a1 = cs.b1 = cs.a2 = cs.b2 = 0;
        cs.c0 = -1;
        cs.c1 = cs.c2 = 0;
        cs.pad0 = 0;
        cs.pad1 = 0;
    } else {
        cs.a0 = e.a0; cs.b0 = e.b0; cs.c0 = e.c0;
        cs.a1 = e.a1; cs.b1 = e.b1; cs.c1 = e.c1;
        cs.a2 = e.a2; cs.b2 = e.b2; cs.c2 = e.c2;
        cs.pad0 = x0 | (x1 << 8) | (y0 << 16) | (y1 << 24);
        cs.pad1 = y1 - y0 + 1;
    }
}

// Depth-key setup of a triangle for the fill (its coverage is already known,
// as masks): oriented like tri_setup, N(dx, dy) = sum over the edges of the
// edge function times the opposite vertex's q, D = twice the area.
__device__ __forceinline__ void key_setup(const int4 *__restrict__ fscr, uint32_t tri, int ox, int oy, KeySetup &ks) {
    const int4 *fs = fscr + 4 * (size_t)(tri >> 1);
    const int t1 = (int)(tri & 1);
    int4 v[3] = {fs[0], fs[1 + t1], fs[2 + t1]};
    ks.tri = ((uint32_t)v[0].w << 1) | (uint32_t)t1;  // the canonical triangle id (corner 0's w)
    long long area = (long long)(v[1].x - v[0].x) * (v[2].y - v[0].y) -
                     (long long)(v[1].y - v[0].y) * (v[2].x - v[0].x);
    if (area < 0) {
        int4 t = v[1];
        v[1] = v[2];
        v[2] = t;
        area = -area;
    }
    long long n0 = 0, na = 0, nb = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int4 p = v[k], q = v[(k + 1) % 3];
        const int A = p.y - q.y, B = q.x - p.x;
        const long long Eo = (long long)A * (ox - p.x) + (long long)B * (oy - p.y);
        const long long qo = v[(k + 2) % 3].z;  // edge k is opposite vertex k + 2
        n0 += Eo * qo;
        na += (long long)A * qo;
        nb += (long long)B * qo;
    }
    ks.n0 = n0;
    ks.na = na;
    ks.nb = nb;
    ks.D = area;
    ks.rD = 1.0 / (double)area;
    ks.pad = 0;
}

__device__ __forceinline__ bool covers(const CovSetup &s, int dx, int dy) {
    int e0 = s.c0 + __mul24(s.a0, dx) + __mul24(s.b0, dy);
    int e1 = s.c1 + __mul24(s.a1, dx) + __mul24(s.b1, dy);
    int e2 = s.c2 + __mul24(s.a2, dx) + __mul24(s.b2, dy);
    return (e0 | e1 | e2) >= 0;
}

__device__ __forceinline__ uint32_t depth_key(const KeySetup &k, int dx, int dy) {
    long long N = k.n0 + k.na * dx + k.nb * dy;
    long long q = (long long)((double)N * k.rD);
    long long r = N - q * k.D;
    if (r < 0) q -= 1;
    else if (r >= k.D) q += 1;
    return (uint32_t)q;
}

// ------------------------------------------------------------------ count / fill
// One workgroup of 512 lanes per screen tile: S = 512 / (TW*TH) groups of
// TW*TH lanes (lane = pixel), the tile's bin dealt to the groups in batches of
// TW*TH entries, round-robin, so that the densest tiles are not walked by one
// wave alone.  For each of its batches a group's lanes each set up one
// triangle into LDS, then the batch's candidates -- the rows of the tile
// inside each triangle's bounding box -- are tested one per lane (the count),
// or its covered pixels expanded one per lane (the fill).  The count pass
// also stores, per bin entry and wave, the 64-bit
// mask of covered pixels, and per group and pixel the fragments of the
// groups before it; the fill pass expands the masks instead of testing
// coverage again and places each group's records after those of the groups
// before it.

template <int TW, int TH>
struct RasterShape {
    static constexpr int NT = TW * TH, NW = NT / 64, S = RASTER_WG / NT;
    static_assert(NT % 64 == 0 && RASTER_WG % NT == 0 && 64 % TW == 0, "tile shape");
};

// Synchronise the lanes of one group (the NT lanes that work on one bin
// chunk).  A one-wave group needs its LDS stores ordered before the loads
// that follow and no code motion of LDS accesses across the point: a
// wavefront-scope release/acquire pair around the wave barrier gives both
// (the compiler may not move memory operations across the fences, and the
// release waits for the wave's outstanding LDS stores).  Wider groups need
// the workgroup barrier, and then every group of the workgroup must reach the
// same number of them.
template <int NW>
__device__ __forceinline__ void group_sync() {
    if constexpr (NW == 1) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// The batches of NT entries that group grp of S takes from the tile's bin
// range [b0, b1): batch k = [b0 + k NT, b0 + (k + 1) NT) goes to group k % S,
// so that every batch but the tile's last is full (the per-batch work of a
// group does not depend on how many of its lanes hold an entry).
struct Chunk {
    uint64_t b0, b1;
    int grp;
    int iters;  // batches per group (the same for every group of the workgroup)
};
template <int NT, int S>
__device__ __forceinline__ Chunk bin_chunk(uint64_t b0, uint64_t b1, int grp) {
    const uint64_t nb = (b1 - b0 + NT - 1) / NT;
    Chunk c;
    c.b0 = b0;
    c.b1 = b1;
    c.grp = grp;
    c.iters = (int)((nb + S - 1) / S);
    return c;
}
// first entry of iteration it of the group's batches
template <int NT, int S>
__device__ __forceinline__ uint64_t batch_base(const Chunk &c, int it) {
    return c.b0 + ((uint64_t)it * S + c.grp) * NT;
}

// Count: every batch of entries is expanded into its candidate (entry, row)
// pairs -- the rows of the tile that cross the triangle's bounding box --
// one lane per pair, which tests the row's pixels inside the box; LDS
// atomics accumulate the per-pixel counts and, one per row, the entries'
// coverage masks.
constexpr int RASTER_WINDOW = 1024;  // candidate pairs expanded at a time per group

template <int TW, int TH>
__global__ void __launch_bounds__(RASTER_WG) k_count(Tiling tl, const uint64_t *__restrict__ tile_off,
                                                     const uint32_t *__restrict__ bins,
                                                     const int4 *__restrict__ fscr, int64_t F,
                                                     uint32_t *__restrict__ count, uint64_t cap,
                                                     uint64_t *__restrict__ masks, uint32_t *__restrict__ gpre) {
    using RS = RasterShape<TW, TH>;
    constexpr int NT = RS::NT, NW = RS::NW, S = RS::S;
    static_assert(NT <= 256, "entry and pixel indices are packed in 8 bits each");
    __shared__ CovSetup s_cov[S][NT];
    __shared__ uint32_t s_cnt[S][NT];
    __shared__ unsigned long long s_macc[S][NT * NW];
    __shared__ uint32_t s_wsum[S][NW];
    __shared__ uint16_t s_cand[S][RASTER_WINDOW];
    const int grp = threadIdx.x / NT, t = threadIdx.x % NT;
    const int64_t g = blockIdx.x;  // global tile
    const int64_t view = g / tl.ntiles;
    const int tile = (int)(g - view * tl.ntiles);
    fscr += view * 4 * F;
    const int tx = tile % tl.ntx, ty = tile / tl.ntx;
    const int lane = t & 63, wave = t >> 6;
    const int ox = SUB * (tx * TW) + SUB / 2, oy = SUB * (ty * TH) + SUB / 2;
    const int vw = tl.W - tx * TW, vh = tl.H - ty * TH;  // valid pixels: lx < vw, ly < vh
    // (bins beyond the capacity were not stored; the caller grows and redoes the frame)
    const uint64_t b0 = min(tile_off[g], cap), b1 = min(tile_off[g + 1], cap);
    const Chunk ch = bin_chunk<NT, S>(b0, b1, grp);
    s_cnt[grp][t] = 0;
    for (int it = 0; it < ch.iters; ++it) {
        const uint64_t base = batch_base<NT, S>(ch, it);
        const int m = base < ch.b1 ? (int)min((uint64_t)NT, ch.b1 - base) : 0;
        uint32_t c = 0;
        int box = 0;
        if (t < m) {
            CovSetup cs;
            tri_setup(fscr, bins[base + t], ox, oy, SUB * (TW - 1), SUB * (TH - 1), cs);
            s_cov[grp][t] = cs;
            c = (uint32_t)cs.pad1;
            box = cs.pad0;
#pragma unroll
            for (int w = 0; w < NW; ++w) s_macc[grp][t * NW + w] = 0ull;
        }
        uint32_t incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_wsum[grp][wave] = incl;
        group_sync<NW>();
        uint32_t carry = 0, total = 0, most = 0;
        if constexpr (NW == 1) {
            total = s_wsum[grp][0];
            most = total;  // (a one-wave group runs its own number of windows)
        } else {
#pragma unroll
            for (int q = 0; q < S; ++q) {
                uint32_t tq = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const uint32_t ws = s_wsum[q][w];
                    if (q == grp) carry += w < wave ? ws : 0u;
                    tq += ws;
                }
                if (q == grp) total = tq;
                most = max(most, tq);
            }
        }
        const uint32_t cb = carry + incl - c;
        // (wider groups all run the same number of windows: the loop holds barriers)
        for (uint32_t w0 = 0; w0 < most; w0 += RASTER_WINDOW) {
            if (c && cb < w0 + RASTER_WINDOW && cb + c > w0) {
                const int y0 = (box >> 16) & 255;
                for (uint32_t pos = max(cb, w0); pos < min(cb + c, w0 + RASTER_WINDOW); ++pos)
                    s_cand[grp][pos - w0] = (uint16_t)((t << 8) | (y0 + (int)(pos - cb)));
            }
            group_sync<NW>();
            const uint32_t nf = w0 < total ? min((uint32_t)RASTER_WINDOW, total - w0) : 0u;
            for (uint32_t f = t; f < nf; f += NT) {
                const uint32_t pr = s_cand[grp][f];
                const int j = (int)(pr >> 8), ly = (int)(pr & 255u);
                if (ly >= vh) continue;
                const CovSetup &cs = s_cov[grp][j];
                const int x0 = cs.pad0 & 255, x1 = min((cs.pad0 >> 8) & 255, vw - 1);
                // the row's pixels x0..x1 (a row lies in one 64-bit mask word: TW divides 64)
                unsigned long long bits = 0ull;
                for (int lx = x0; lx <= x1; ++lx) {
                    if (covers(cs, SUB * lx, SUB * ly)) {
                        const int pp = ly * TW + lx;
                        atomicAdd(&s_cnt[grp][pp], 1u);
                        bits |= 1ull << (pp & 63);
                    }
                }
                if (bits) atomicOr(&s_macc[grp][j * NW + ((ly * TW) >> 6)], bits);
            }
            group_sync<NW>();
        }
        if (t < m) {
#pragma unroll
            for (int w = 0; w < NW; ++w) masks[(base + t) * NW + w] = s_macc[grp][t * NW + w];
        }
        group_sync<NW>();  // s_cov, s_macc and s_wsum are rewritten by the next batch
    }
    __syncthreads();
    uint32_t before = 0, tot = 0;  // fragments of the groups before this one, and of all
#pragma unroll
    for (int q = 0; q < S; ++q) {
        before += q < grp ? s_cnt[q][t] : 0u;
        tot += s_cnt[q][t];
    }
    gpre[(size_t)g * RASTER_WG + threadIdx.x] = before;
    if (grp == 0) count[(size_t)g * NT + t] = tot;
}

// Fill: every batch of entries is expanded into a compact list of (entry,
// pixel) fragments in LDS, and the group's lanes
// take one fragment each (instead of one entry per wave step, which left most
// lanes idle: an entry covers a few pixels of the tile).  Slots within a
// pixel's list come from LDS counters, so records of one group may land in
// any order within the group's range; every consumer sorts the list.
constexpr int FILL_WINDOW = 512;  // fragments expanded at a time per group (fewer than candidates: LDS for occupancy)

template <int TW, int TH>
__global__ void __launch_bounds__(RASTER_WG) k_fill(Tiling tl, const uint64_t *__restrict__ pass_tiles,
                                                    const uint64_t *__restrict__ tile_off,
                                                    const uint32_t *__restrict__ bins,
                                                    const int4 *__restrict__ fscr, int64_t F,
                                                    const uint64_t *__restrict__ off, uint64_t *__restrict__ rec,
                                                    uint64_t rec_cap, uint64_t cap,
                                                    const uint64_t *__restrict__ masks,
                                                    const uint32_t *__restrict__ gpre) {
    using RS = RasterShape<TW, TH>;
    constexpr int NT = RS::NT, NW = RS::NW, S = RS::S;
    static_assert(NT <= 256, "entry and pixel indices are packed in 8 bits each");
    __shared__ KeySetup s_key[S][NT];
    __shared__ uint64_t s_mask[S][NT * NW];
    __shared__ uint32_t s_pos[S][NT];   // per pixel: next slot of the group
    __shared__ uint32_t s_wsum[S][NW];  // per wave: fragments (scan carry)
    __shared__ uint16_t s_frag[S][FILL_WINDOW];
    __shared__ uint64_t s_first[NT];
    const int64_t g0 = (int64_t)pass_tiles[0], g1 = (int64_t)pass_tiles[1];
    const int64_t g = g0 + blockIdx.x;  // global tile
    if (g >= g1) return;  // (uniform) outside this pass
    const int grp = threadIdx.x / NT, t = threadIdx.x % NT;
    const int64_t view = g / tl.ntiles;
    const int tile = (int)(g - view * tl.ntiles);
    fscr += view * 4 * F;
    const int tx = tile % tl.ntx, ty = tile / tl.ntx;
    const int lane = t & 63, wave = t >> 6;
    const int ox = SUB * (tx * TW) + SUB / 2, oy = SUB * (ty * TH) + SUB / 2;
    const uint64_t pass_base = off[(size_t)g0 * NT];
    if (grp == 0) s_first[t] = off[(size_t)g * NT + t] - pass_base;
    const uint64_t b0 = min(tile_off[g], cap), b1 = min(tile_off[g + 1], cap);
    const Chunk ch = bin_chunk<NT, S>(b0, b1, grp);
    // the group's first slot per pixel (the fragments of the groups before it, from the count pass)
    s_pos[grp][t] = gpre[(size_t)g * RASTER_WG + threadIdx.x];
    __syncthreads();
    // expand each batch into fragments, one lane per fragment; a lane's bin
    // entry and masks for the next batch are loaded while this one is worked
    // on (its triangle's screen vertices too measured slower: registers)
    uint32_t bin = 0;
    uint64_t mk[NW];
    auto load_entry = [&](int it2) {
        const uint64_t b = batch_base<NT, S>(ch, it2) + t;
        if (it2 < ch.iters && b < ch.b1) {
            bin = bins[b];
#pragma unroll
            for (int w = 0; w < NW; ++w) mk[w] = masks[b * NW + w];
        }
    };
    load_entry(0);
    for (int it = 0; it < ch.iters; ++it) {
        const uint64_t base = batch_base<NT, S>(ch, it);
        const int m = base < ch.b1 ? (int)min((uint64_t)NT, ch.b1 - base) : 0;
        uint32_t c = 0;
        uint32_t tri = 0;
        if (t < m) {
            tri = bin;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                s_mask[grp][t * NW + w] = mk[w];
                c += (uint32_t)__popcll(mk[w]);
            }
        }
        if (c) {  // (a covered triangle is not culled: its area is not zero)
            KeySetup ks;
            key_setup(fscr, tri, ox, oy, ks);
            s_key[grp][t] = ks;
        }
        load_entry(it + 1);
        // exclusive scan of the entries' fragment counts over the group
        uint32_t incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_wsum[grp][wave] = incl;
        __syncthreads();
        uint32_t carry = 0, total = 0, most = 0;  // most: the largest total of the workgroup's groups
#pragma unroll
        for (int q = 0; q < S; ++q) {
            uint32_t tq = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t ws = s_wsum[q][w];
                if (q == grp) carry += w < wave ? ws : 0u;
                tq += ws;
            }
            if (q == grp) total = tq;
            most = max(most, tq);
        }
        const uint32_t fb = carry + incl - c;
        // (every group runs the same number of windows: the loop holds barriers.  Keeping
        // the groups of a tile in step measured faster here than wave-level
        // synchronisation: their record stores to the tile's lists meet in the caches.)
        for (uint32_t w0 = 0; w0 < most; w0 += FILL_WINDOW) {
            // entries write their fragments that fall into this window
            if (c && fb < w0 + FILL_WINDOW && fb + c > w0) {
                uint32_t pos = fb;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    uint64_t mk = s_mask[grp][t * NW + w];
                    while (mk && pos < w0 + FILL_WINDOW) {
                        const int b = __ffsll((long long)mk) - 1;
                        mk &= mk - 1;
                        if (pos >= w0) s_frag[grp][pos - w0] = (uint16_t)((t << 8) | (w * 64 + b));
                        ++pos;
                    }
                }
            }
            __syncthreads();
            const uint32_t nf = w0 < total ? min((uint32_t)FILL_WINDOW, total - w0) : 0u;
            for (uint32_t f = t; f < nf; f += NT) {
                const uint32_t fr = s_frag[grp][f];
                const int j = (int)(fr >> 8), pp = (int)(fr & 255u);
                const KeySetup &ks = s_key[grp][j];
                const uint32_t key = depth_key(ks, SUB * (pp % TW), SUB * (pp / TW));
                const uint32_t slot = atomicAdd(&s_pos[grp][pp], 1u);
                const uint64_t first = s_first[pp];
                if (first < rec_cap && slot < rec_cap - first)
                    rec[first + slot] = ((uint64_t)(KMAX - key) << 32) | (uint64_t)ks.tri;
            }
            __syncthreads();
        }
        __syncthreads();  // s_wsum, s_mask and s_key are rewritten by the next batch
    }
}

// ------------------------------------------------------------------ scan (u32 -> u64 exclusive)
constexpr int SCAN_BS = 256, SCAN_IT = 8, SCAN_CHUNK = SCAN_BS * SCAN_IT;

__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *sh, uint64_t &total) {
    // Hillis-Steele over 256 threads in LDS
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_BS; o <<= 1) {
        uint64_t x = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    total = sh[SCAN_BS - 1];
    uint64_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(SCAN_BS) k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                         uint64_t *__restrict__ part) {
    __shared__ uint64_t sh[SCAN_BS];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_IT;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_IT; ++i)
        if (base + i < n) s += in[base + i];
    uint64_t tot;
    block_excl_scan(s, sh, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_BS) k_scan_parts(uint64_t *__restrict__ part, int64_t nparts,
                                                        uint64_t *__restrict__ out_total,
                                                        uint64_t *__restrict__ stat) {
    __shared__ uint64_t sh[SCAN_BS];
    uint64_t carry = 0;
    for (int64_t c = 0; c < nparts; c += SCAN_BS) {
        int64_t i = c + threadIdx.x;
        uint64_t v = i < nparts ? part[i] : 0;
        uint64_t tot;
        uint64_t ex = block_excl_scan(v, sh, tot);
        if (i < nparts) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *out_total = carry;
        if (stat) *stat = carry;
    }
}

__global__ void __launch_bounds__(SCAN_BS) k_scan_apply(const uint32_t *__restrict__ in, int64_t n,
                                                        const uint64_t *__restrict__ part,
                                                        uint64_t *__restrict__ out) {
    __shared__ uint64_t sh[SCAN_BS];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_IT;
    uint32_t v[SCAN_IT];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_IT; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan(s, sh, tot) + part[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_IT; ++i) {
        if (base + i < n) out[base + i] = ex;
        ex += v[i];
    }
}

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + SCAN_CHUNK - 1) / SCAN_CHUNK) + 1; }

void launch_scan_u32_u64(const uint32_t *in, int64_t n, uint64_t *out, uint64_t *tmp, uint64_t *stat,
                         hipStream_t s) {
    int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nb > 0) k_scan_reduce<<<dim3((unsigned)nb), dim3(SCAN_BS), 0, s>>>(in, n, tmp);
    k_scan_parts<<<1, SCAN_BS, 0, s>>>(tmp, nb, out + n, stat);
    if (nb > 0) k_scan_apply<<<dim3((unsigned)nb), dim3(SCAN_BS), 0, s>>>(in, n, tmp, out);
}

// ------------------------------------------------------------------ pass planning
// Greedy split of the tile sequence into passes whose fragments fit the
// workspace (the paper assumes the lists fit, Section 6, and meets a buffer
// cap at its largest viewport, Section 7, Table 2).  One thread; binary search over
// the tile prefix sums.
__global__ void k_plan(int ntiles, int tp, const uint64_t *__restrict__ off, uint64_t budget,
                       uint64_t *__restrict__ stats) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int np = 0;
    int start = 0;
    stats[ST_PASS] = 0;
    stats[ST_PLAN_ERR] = 0;
    while (start < ntiles) {
        uint64_t s0 = off[(size_t)start * tp];
        int lo = start, hi = ntiles;  // largest end with off[end*tp] - s0 <= budget
        while (lo < hi) {
            int mid = lo + (hi - lo + 1) / 2;
            if (off[(size_t)mid * tp] - s0 <= budget) lo = mid;
            else hi = mid - 1;
        }
        if (lo == start || np >= MAX_PASSES) {
            stats[ST_PLAN_ERR] = 1;
            break;
        }
        stats[ST_PASS + (++np)] = (uint64_t)lo;
        start = lo;
    }
    stats[ST_NPASS] = (uint64_t)np;
}

void launch_plan(const Tiling &tl, const uint64_t *off, uint64_t budget_recs, uint64_t *stats, hipStream_t s) {
    k_plan<<<1, 64, 0, s>>>(tl.ntiles, tl.TW * tl.TH, off, budget_recs, stats);
}

__global__ void k_single_pass(int64_t ntiles, uint64_t *__restrict__ stats) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    stats[ST_NPASS] = 1;
    stats[ST_PASS] = 0;
    stats[ST_PASS + 1] = (uint64_t)ntiles;
}

void launch_single_pass(int64_t ntiles, uint64_t *stats, hipStream_t s) { k_single_pass<<<1, 64, 0, s>>>(ntiles, stats); }

// ------------------------------------------------------------------ closing kernel of a frame
// Flags what went wrong (the frame's output is then invalid), keeps the
// largest needs seen across frames and copies them to host-mapped memory, so
// that the host can size later frames without waiting on this one.  One thread.
__global__ void k_finish(uint64_t *__restrict__ stats, uint64_t *__restrict__ persist,
                         volatile uint64_t *__restrict__ published, uint64_t bin_cap, int passes_launched,
                         uint64_t ws_recs, int single_pass) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t flags = 0;
    if (stats[ST_BINS] > bin_cap) flags |= FRAME_BINS;
    if (single_pass) {
        if (stats[ST_FRAGS] > ws_recs) flags |= FRAME_WORKSPACE;
    } else if (stats[ST_PLAN_ERR]) {
        flags |= FRAME_PLAN;
    } else if (stats[ST_NPASS] > (uint64_t)passes_launched) {
        flags |= FRAME_PASSES;
    }
    stats[ST_FLAGS] = flags;
    persist[PS_MAX_BINS] = max(persist[PS_MAX_BINS], stats[ST_BINS]);
    persist[PS_MAX_PASSES] = max(persist[PS_MAX_PASSES], stats[ST_NPASS]);
    persist[PS_FRAMES] += 1;
    persist[PS_FLAGGED] += flags ? 1 : 0;
    persist[PS_LAST_FLAGS] = flags;
    persist[PS_LAST_FRAGS] = stats[ST_FRAGS];
    const uint64_t np = min(stats[ST_NPASS], (uint64_t)MAX_PASSES);
    for (int c = 0; c < NCLASS; ++c) {
        uint64_t m = 0;
        for (uint64_t k = 0; k < np; ++k) m = max(m, stats[ST_PCLASS + k * NCLASS + c]);
        persist[PS_CLASS + c] = m;
    }
    if (published) {
        for (int i = 0; i < PS_COUNT; ++i) published[1 + i] = persist[i];
        __threadfence_system();
        published[0] = persist[PS_FRAMES];
        __threadfence_system();
    }
}

void launch_finish(uint64_t *stats, uint64_t *persist, uint64_t *published, uint64_t bin_cap, int passes_launched,
                   uint64_t ws_recs, bool single_pass, hipStream_t s) {
    k_finish<<<1, 64, 0, s>>>(stats, persist, published, bin_cap, passes_launched, ws_recs, single_pass ? 1 : 0);
}

__global__ void k_set_view(ViewParams vp, ViewParams *__restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = vp;
}

void launch_set_view(const ViewParams &vp, ViewParams *dst, hipStream_t s) { k_set_view<<<1, 64, 0, s>>>(vp, dst); }

// ------------------------------------------------------------------ length classes
// Each block classifies CLS_PPT * 256 consecutive pixels (coalesced rows of
// 256).  Class counts are aggregated per wave (lanes of one class take one
// LDS atomic), per block in LDS, and then with one global atomic per class
// and block: the class counters are the most contended addresses of the frame.
constexpr int CLS_PPT = 8;

__global__ void __launch_bounds__(256) k_classify(Tiling tl, int k, const uint32_t *__restrict__ count, int t_sort,
                                                  uint32_t *__restrict__ lists, int64_t cap,
                                                  uint64_t *__restrict__ stats) {
    __shared__ unsigned s_n[NCLASS];
    __shared__ unsigned long long s_f[NCLASS], s_base[NCLASS];
    const int64_t TPX = (int64_t)tl.TW * tl.TH;
    const int64_t p0 = (int64_t)stats[ST_PASS + k] * TPX, p1 = (int64_t)stats[ST_PASS + k + 1] * TPX;
    if (p0 + (int64_t)blockIdx.x * (256 * CLS_PPT) >= p1) return;  // (uniform) outside this pass
    if (threadIdx.x < NCLASS) {
        s_n[threadIdx.x] = 0;
        s_f[threadIdx.x] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int TP = tl.TW * tl.TH;
    const int64_t blk0 = p0 + (int64_t)blockIdx.x * (256 * CLS_PPT);
    int cls[CLS_PPT];
    unsigned rank[CLS_PPT];
    unsigned long long fsum[NCLASS];
#pragma unroll
    for (int c = 0; c < NCLASS; ++c) fsum[c] = 0;
#pragma unroll
    for (int i = 0; i < CLS_PPT; ++i) {
        const int64_t p = blk0 + i * 256 + threadIdx.x;
        cls[i] = -1;
        rank[i] = 0;
        if (p < p1) {
            const int64_t lp = p % ((int64_t)tl.ntiles * TP);  // pixel within its view
            const int tile = (int)(lp / TP), l = (int)(lp % TP);
            const int x = (tile % tl.ntx) * tl.TW + l % tl.TW;
            const int y = (tile / tl.ntx) * tl.TH + l / tl.TW;
            if (x < tl.W && y < tl.H) {
                const uint32_t n = count[p];
                cls[i] = length_class(n, t_sort);
#pragma unroll
                for (int c = 0; c < NCLASS; ++c) fsum[c] += cls[i] == c ? n : 0u;
            }
        }
        // one LDS atomic per class present in the wave
        unsigned long long pend = __ballot(cls[i] >= 0);
        while (pend) {
            const int leader = __ffsll((long long)pend) - 1;
            const int lc = __shfl(cls[i], leader);
            const unsigned long long m = __ballot(cls[i] == lc);
            unsigned base = 0;
            if (lane == leader) base = atomicAdd(&s_n[lc], (unsigned)__popcll(m));
            base = __shfl(base, leader);
            if (cls[i] == lc) rank[i] = base + (unsigned)__popcll(m & below);
            pend &= ~m;
        }
    }
#pragma unroll
    for (int c = 0; c < NCLASS; ++c) {
        unsigned long long v = fsum[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0 && v) atomicAdd(&s_f[c], v);
    }
    __syncthreads();
    if (threadIdx.x < NCLASS) {
        const int c = threadIdx.x;
        s_base[c] = s_n[c] ? atomicAdd((unsigned long long *)&stats[ST_PCLASS + k * NCLASS + c],
                                       (unsigned long long)s_n[c])
                           : 0ull;
        if (s_n[c]) atomicAdd((unsigned long long *)&stats[ST_CLASS + c], (unsigned long long)s_n[c]);
        if (s_f[c]) atomicAdd((unsigned long long *)&stats[ST_CLASSF + c], s_f[c]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CLS_PPT; ++i)
        if (cls[i] >= 0) lists[(int64_t)cls[i] * cap + s_base[cls[i]] + rank[i]] = (uint32_t)(blk0 + i * 256 + threadIdx.x);
}

void launch_classify(const Tiling &tl, int nv, int k, const uint32_t *count, int t_sort, uint32_t *cls_lists,
                     int64_t cls_cap, uint64_t *stats, hipStream_t s) {
    const int64_t n = (int64_t)tl.ntiles * nv * tl.TW * tl.TH;
    if (n <= 0) return;
    const int64_t per = 256 * CLS_PPT;
    k_classify<<<dim3((unsigned)((n + per - 1) / per)), 256, 0, s>>>(tl, k, count, t_sort, cls_lists, cls_cap, stats);
}

// ------------------------------------------------------------------ small utilities
__global__ void k_zero_u64(uint64_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
__global__ void k_zero_u32(uint32_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
void launch_zero_u64(uint64_t *p, int64_t n, hipStream_t s) {
    if (n > 0) k_zero_u64<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(p, n);
}
void launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s) {
    if (n > 0) k_zero_u32<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(p, n);
}

__global__ void k_rowmajor_counts(Tiling tl, const uint32_t *__restrict__ ctm, uint32_t *__restrict__ crm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)tl.W * tl.H) return;
    int x = (int)(i % tl.W), y = (int)(i / tl.W);
    int tile = (y / tl.TH) * tl.ntx + x / tl.TW;
    int l = (y % tl.TH) * tl.TW + x % tl.TW;
    crm[i] = ctm[(int64_t)tile * tl.TW * tl.TH + l];
}
void launch_rowmajor_counts(const Tiling &tl, const uint32_t *count_tm, uint32_t *count_rm, hipStream_t s) {
    int64_t n = (int64_t)tl.W * tl.H;
    k_rowmajor_counts<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(tl, count_tm, count_rm);
}

// ------------------------------------------------------------------ launchers
void launch_transform(const int4 *posq, int64_t V, int nv, const ViewParams *views, int W, int H, VertRec *vert,
                      int4 *vscr, hipStream_t s) {
    const int64_t n = V * nv;
    if (n > 0) k_transform<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(posq, V, n, views, W, H, vert, vscr);
}
__global__ void k_tile_totals(uint32_t *__restrict__ ctr, int64_t NT) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < NT) ctr[NT + g] += ctr[g];
}

void launch_tri_bin_count(const int4 *face_c, const uint32_t *face_ord, int64_t F, int nv, const int4 *vscr,
                          int64_t V, const Tiling &tl, uint32_t *tile_cnt, int4 *fscr, uint32_t *bslot,
                          int4 *frange, hipStream_t s) {
    const int64_t n = F * nv, NT = (int64_t)tl.ntiles * nv;
    if (n > 0)
        k_tri_bin<false><<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(face_c, face_ord, F, n, vscr, V, tl,
                                                                          tile_cnt,
                                                                          nullptr, nullptr, 0, fscr, bslot, nullptr,
                                                                          NT, frange);
    if (NT > 0) k_tile_totals<<<dim3((unsigned)((NT + 255) / 256)), 256, 0, s>>>(tile_cnt, NT);
}
void launch_tri_bin_scatter(const int4 *frange, int64_t F, int nv, const Tiling &tl, const uint64_t *tile_off,
                            const uint32_t *tile_lo, uint32_t *tile_fill, uint32_t *bins, uint64_t bin_cap,
                            const uint32_t *bslot, hipStream_t s) {
    const int64_t n = F * nv, NT = (int64_t)tl.ntiles * nv;
    if (n > 0)
        k_tri_bin<true><<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(
            nullptr, nullptr, F, n, nullptr, 0, tl, tile_fill, tile_off, bins, bin_cap, nullptr,
            const_cast<uint32_t *>(bslot), tile_lo, NT, const_cast<int4 *>(frange));
}

#define HEXFC_TILE_DISPATCH(TWv, THv, CALL) \
    if (tl.TW == TWv && tl.TH == THv) { CALL; return; }

void launch_count(const Tiling &tl, int nv, const uint64_t *tile_off, const uint32_t *bins, uint64_t cap,
                  const int4 *fscr, int64_t F, uint32_t *count, uint64_t *masks, uint32_t *gpre, hipStream_t s) {
    dim3 g((unsigned)((int64_t)tl.ntiles * nv));
#define ARGS tl, tile_off, bins, fscr, F, count, cap, masks, gpre
    HEXFC_TILE_DISPATCH(8, 8, (k_count<8, 8><<<g, RASTER_WG, 0, s>>>(ARGS)));
    HEXFC_TILE_DISPATCH(16, 8, (k_count<16, 8><<<g, RASTER_WG, 0, s>>>(ARGS)));
    HEXFC_TILE_DISPATCH(16, 16, (k_count<16, 16><<<g, RASTER_WG, 0, s>>>(ARGS)));
    HEXFC_TILE_DISPATCH(32, 8, (k_count<32, 8><<<g, RASTER_WG, 0, s>>>(ARGS)));
#undef ARGS
}

void launch_fill(const Tiling &tl, int nv, const uint64_t *pass_tiles, const uint64_t *tile_off,
                 const uint32_t *bins, uint64_t cap, const int4 *fscr, int64_t F, const uint64_t *off, uint64_t *rec,
                 uint64_t rec_cap, const uint64_t *masks, const uint32_t *gpre, hipStream_t s) {
    const int64_t nt = (int64_t)tl.ntiles * nv;
    if (nt <= 0) return;
    dim3 g((unsigned)nt);
#define ARGS tl, pass_tiles, tile_off, bins, fscr, F, off, rec, rec_cap, cap, masks, gpre
    HEXFC_TILE_DISPATCH(8, 8, (k_fill<8, 8><<<g, RASTER_WG, 0, s>>>(ARGS)));
    HEXFC_TILE_DISPATCH(16, 8, (k_fill<16, 8><<<g, RASTER_WG, 0, s>>>(ARGS)));
    HEXFC_TILE_DISPATCH(16, 16, (k_fill<16, 16><<<g, RASTER_WG, 0, s>>>(ARGS)));
    HEXFC_TILE_DISPATCH(32, 8, (k_fill<32, 8><<<g, RASTER_WG, 0, s>>>(ARGS)));
#undef ARGS
}

}  // namespace hexfc
