// resolve.hip -- per-pixel sort, focus+context shading and front-to-back
// compositing on gfx950.
//
// The paper sorts each per-pixel list by distance to the camera with a GPU
// priority queue and alpha-blends the fragments in that order (Section 3,
// Section 6); each fragment's colour comes from Eq. 1-4 (Section 4).  Here the
// shading is deferred until after the sort (lists then do not depend on lens
// or style), and lists are sorted by length class:
//   * short lists (n <= t_sort): one lane per pixel, insertion sort in an LDS
//     column private to the lane, then a sequential front-to-back blend;
//   * long lists: one wave per pixel, bitonic sort of 64*R keys held R per
//     lane in registers (cross-lane stages by lane shuffles), every lane
//     shading its R fragments in parallel, then an ordered wave reduction
//     with the associative "over" operator.
#include <algorithm>

#include "kern.h"

namespace hexfc {

// Sort key order: record = (depth field << 32) | triangle id, ascending.

// x as held by lane ^ m, for m a power of two below 64 (a constant once the
// callers' loops are unrolled), without the LDS round trip of a general lane
// permutation where the hardware has a fixed one: quad permutations (m = 1,
// 2) and the rotation of a 16-lane row by 8 (m = 8) as DPP operand
// modifiers, gfx950's swaps of 16-lane row pairs (m = 16) and of wave halves
// (m = 32), and the swizzle of the LDS crossbar for m = 4.
__device__ __forceinline__ uint32_t xor_lane(uint32_t x, int m, int lane) {
    switch (m) {
    // (every lane has a source in these patterns: no old value to keep)
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);   // quad_perm 1,0,3,2
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);   // quad_perm 2,3,0,1
    case 4: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x1f | (4 << 10));               // and 31, xor 4
    case 8: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true);  // row_ror 8
    case 16: {
        // rows 1, 3 of the first operand trade places with rows 0, 2 of the second
        const auto s = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (lane & 16) ? s[0] : s[1];
    }
    default: {
        // lanes 32..63 of the first operand trade places with lanes 0..31 of the second
        const auto s = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (lane & 32) ? s[0] : s[1];
    }
    }
}
__device__ __forceinline__ uint64_t xor_lane(uint64_t x, int m, int lane) {
    return ((uint64_t)xor_lane((uint32_t)(x >> 32), m, lane) << 32) | xor_lane((uint32_t)x, m, lane);
}
__device__ __forceinline__ float xor_lane(float x, int m, int lane) {
    return __uint_as_float(xor_lane(__float_as_uint(x), m, lane));
}
__device__ __forceinline__ float lane0(float x) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(x), 0));
}

struct Frag {
    float r, g, b, a;
};

// Squared distance from p to the segment a-b (the shading compares distances
// with thresholds and with each other only, so their squares serve).
__device__ __forceinline__ float segdist2(float px, float py, float pz, float ax, float ay, float az, float bx,
                                          float by, float bz) {
    float ux = bx - ax, uy = by - ay, uz = bz - az;
    float wx = px - ax, wy = py - ay, wz = pz - az;
    float l2 = ux * ux + uy * uy + uz * uz;
    float t = l2 > 0.f ? (wx * ux + wy * uy + wz * uz) * __builtin_amdgcn_rcpf(l2) : 0.f;
    t = fminf(fmaxf(t, 0.f), 1.f);
    float dx = wx - t * ux, dy = wy - t * uy, dz = wz - t * uz;
    return dx * dx + dy * dy + dz * dz;
}

// a b - c d for integers a, b, c, d below 2^19 in magnitude (exact in FP32),
// to within 2 ulp: the rounding error of c d is recovered with an FMA
// (Kahan's 2 x 2 determinant).
__device__ __forceinline__ float det2(float a, float b, float c, float d) {
    const float w = c * d;
    const float e = fmaf(-c, d, w);
    return fmaf(a, b, -w) + e;
}

// Premultiplied colour and opacity of one fragment: triangle `tri` at pixel
// (x, y).  Eq. 1 (edges, with the focus-edge halo and darkening), Eq. 2
// (accentuation), Eq. 3 (face opacity), Eq. 4 (edge/face blend).
__device__ __forceinline__ Frag shade(const DevMesh &m, const VertRec *__restrict__ vert, const ShadeParams &sp,
                                      uint32_t tri, int x, int y) {
    const uint32_t f = tri >> 1;
    const bool t1 = tri & 1;
    const FaceRec F = m.face[f];
    const int4 c = F.c;
    // the triangle's screen vertices: corners 0, 1 + t, 2 + t
    const int4 s0 = vert[c.x].scr, s1 = vert[t1 ? c.z : c.y].scr, s2 = vert[t1 ? c.w : c.z].scr;
    // perspective-correct barycentrics: weight of vertex i = E_opp(i) * q_i,
    // the edge functions from integer screen coordinates (below 2^18 in
    // magnitude: every difference is exact in FP32) to within 2 ulp, the
    // weights in FP32 (positive inside the triangle: no cancellation)
    const float X = (float)(SUB * x + SUB / 2), Y = (float)(SUB * y + SUB / 2);
    const float x0 = (float)s0.x, y0 = (float)s0.y, x1 = (float)s1.x, y1 = (float)s1.y;
    const float x2 = (float)s2.x, y2 = (float)s2.y;
    const float e0 = det2(x2 - x1, Y - y1, y2 - y1, X - x1);
    const float e1 = det2(x0 - x2, Y - y2, y0 - y2, X - x2);
    const float e2 = det2(x1 - x0, Y - y0, y1 - y0, X - x0);
    const float w0 = e0 * (float)s0.z, w1 = e1 * (float)s1.z, w2 = e2 * (float)s2.z;
    const float inv = __builtin_amdgcn_rcpf(w0 + w1 + w2);
    const float l0 = w0 * inv, l1 = w1 * inv, l2 = w2 * inv;
    // corners relative to corner 0 (exact: all are multiples of 2^-16)
    const float4 P0 = vert[c.x].world, P1 = vert[c.y].world, P2 = vert[c.z].world, P3 = vert[c.w].world;
    const float r1x = P1.x - P0.x, r1y = P1.y - P0.y, r1z = P1.z - P0.z;
    const float r2x = P2.x - P0.x, r2y = P2.y - P0.y, r2z = P2.z - P0.z;
    const float r3x = P3.x - P0.x, r3y = P3.y - P0.y, r3z = P3.z - P0.z;
    const float bx = t1 ? r2x : r1x, by = t1 ? r2y : r1y, bz = t1 ? r2z : r1z;
    const float cx = t1 ? r3x : r2x, cy = t1 ? r3y : r2y, cz = t1 ? r3z : r2z;
    const float px = l1 * bx + l2 * cx, py = l1 * by + l2 * cy, pz = l1 * bz + l2 * cz;
    const float tb = t1 ? P2.w : P1.w, tc = t1 ? P3.w : P2.w;
    const float tf = l0 * P0.w + l1 * tb + l2 * tc;
    // focus: object-space sphere, or the screen-space circle of Section 4
    // (centre hc[0], hc[1] and radius in pixels)
    float dist;
    if (sp.lens_mode == 1) {
        const float ex = ((float)x + 0.5f) - sp.hc[0], ey = ((float)y + 0.5f) - sp.hc[1];
        dist = __builtin_amdgcn_sqrtf(ex * ex + ey * ey) * sp.inv_r;
    } else {
        const float hx = (P0.x - sp.hc[0]) + px, hy = (P0.y - sp.hc[1]) + py, hz = (P0.z - sp.hc[2]) + pz;
        dist = __builtin_amdgcn_sqrtf(hx * hx + hy * hy + hz * hz) * sp.inv_r;
    }
    float u = fminf(fmaxf((dist - 0.7f) * (1.0f / 0.3f), 0.f), 1.f);
    const float focus = 1.f - u * u * (3.f - 2.f * u);
    // squared distances to the four face edges
    float d[4];
    d[0] = segdist2(px, py, pz, 0.f, 0.f, 0.f, r1x, r1y, r1z);
    d[1] = segdist2(px, py, pz, r1x, r1y, r1z, r2x, r2y, r2z);
    d[2] = segdist2(px, py, pz, r2x, r2y, r2z, r3x, r3y, r3z);
    d[3] = segdist2(px, py, pz, r3x, r3y, r3z, 0.f, 0.f, 0.f);
    const uint32_t lv = F.lvl;
    const float4 te4 = F.te;
    const float te[4] = {te4.x, te4.y, te4.z, te4.w};
    // nearest visible edge of each set (ties: lower local edge index)
    float dF = INFINITY, dC = INFINITY, dA = d[0], tF = 0.f, tC = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool inC = (int)((lv >> (8 * k)) & 0xffu) >= sp.lod;
        const bool inF = inC || te[k] >= sp.delta;
        if (inF && d[k] < dF) { dF = d[k]; tF = te[k]; }
        if (inC && d[k] < dC) { dC = d[k]; tC = te[k]; }
        dA = fminf(dA, d[k]);
    }
    // (distances squared: thresholds squared)
    const float w = (1.f + sp.k_focus * focus) * sp.w_base, wh = w + sp.halo_w * focus;
    const bool eF = dF <= w * w, eC = dC <= w * w;
    const bool h = !eF && dF <= wh * wh;
    const float dk = 1.f - sp.darken * focus;
    const float AF = eF ? 1.f : (h ? sp.halo_a : 0.f);
    const float fe = eC ? 1.f - focus : 0.f;  // (1 - focus) * e_C
    float Ce[3];
    Frag o;
    const float ae = fe + focus * AF;
    const float wa = (2.f / 3.f) * sp.w_base;
    const bool acc = dA <= wa * wa;
    const float se = acc ? sp.s : 1.f;
    const float ahat = sp.a_lo + (sp.a_hi - sp.a_lo) * tf;
    const float dc = fminf(dist, 1.f);
    const float dc2 = dc * dc;
    const float afs = fminf(se * (ahat * dc2 * dc2), 1.f);
    const float gain = (se != 1.f) ? 1.f + sp.bright : 1.f;
    const float wf = (1.f - ae) * afs;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float lo = sp.lo[ch], span = sp.hi[ch] - sp.lo[ch];
        const float PF = eF ? (lo + span * tF) * dk : (h ? sp.halo_a : 0.f);
        const float cf = fminf((lo + span * tf) * gain, se != 1.f ? 1.f : INFINITY);
        Ce[ch] = fe * (lo + span * tC) + focus * PF + wf * cf;
    }
    if (sp.desat > 0.f) {  // depth cue in the focus region: desaturate with the view depth
        const float wv = sp.wrow[0] * (P0.x + px) + sp.wrow[1] * (P0.y + py) + sp.wrow[2] * (P0.z + pz) + sp.wrow[3];
        const float z = fminf(fmaxf((wv - sp.zw0) * sp.zinv, 0.f), 1.f);
        const float sd = sp.desat * focus * z;
        const float lum = 0.2126f * Ce[0] + 0.7152f * Ce[1] + 0.0722f * Ce[2];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) Ce[ch] = (1.f - sd) * Ce[ch] + sd * lum;
    }
    o.r = Ce[0];
    o.g = Ce[1];
    o.b = Ce[2];
    o.a = ae + wf;
    return o;
}

constexpr float T_EPS = 9.5367431640625e-07f;  // 2^-20: stop once 1 - A is below it

// ------------------------------------------------------------------ resolve by length class
// The pixels of a pass are resolved by one kernel per length class, each
// specialised for its lists: a lane per pixel (insertion sort in LDS) for the
// short lists, a wave per pixel (bitonic sort in registers) up to 2048
// fragments, a workgroup per pixel (sorted in place) beyond.  Every kernel
// strides over its class list, whose size it reads from device memory, so
// its grid needs no exact count: the host sizes it from the counts it knows
// (exact after a statistics read-back, else those of the last finished
// frame).  The classes above 256 fragments run on a second stream next to
// the others, longest first on both, so that the few long lists do not form
// a tail of their own (see the frame orchestration).

constexpr int RT = 256;      // threads of the resolve workgroup (4 waves)
constexpr int LCAP = 2048;   // longest list a workgroup sorts in LDS; longer ones are sorted in place

// Records of a pass are stored relative to the offset of the pass's first pixel.
__device__ __forceinline__ uint64_t rec_base(const ResolveArgs &a) {
    const int64_t p0 = a.pass_tiles ? (int64_t)a.pass_tiles[0] * (a.tl.TW * a.tl.TH) : a.pass_p0;
    return a.off[p0];
}

__device__ __forceinline__ void write_rgba(const ResolveArgs &a, const PixelRef &pr, const ShadeParams &sp, float C0,
                                           float C1, float C2, float A) {
    const float T = 1.f - A;
    reinterpret_cast<float4 *>(a.rgba)[(pr.view * a.tl.H + pr.y) * (int64_t)a.tl.W + pr.x] =
        make_float4(C0 + T * sp.bg[0], C1 + T * sp.bg[1], C2 + T * sp.bg[2], A);
}

// Short list of pixel p (n <= TS): one lane, insertion sort in the lane's LDS
// column, then a sequential front-to-back blend.
template <int TS>
__device__ __forceinline__ void resolve_lane(const ResolveArgs &a, uint64_t base, uint32_t p,
                                             uint64_t (*__restrict__ col)[64], int lane) {
    uint32_t n = min(a.count[p], (uint32_t)TS);  // the class guarantees n <= t_sort <= TS
    const uint64_t first = a.off[p] - base;
    if (first + n > a.rec_cap) n = 0;  // overflowed workspace: records were not stored
    const uint64_t *src = a.rec + first;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t r = src[i];
        int j = (int)i;
        while (j > 0 && col[j - 1][lane] > r) {
            col[j][lane] = col[j - 1][lane];
            --j;
        }
        col[j][lane] = r;
    }
    const PixelRef pr = pixel_ref(a.tl, p);
    if (a.sorted_out) {
        uint64_t *dst = a.sorted_out + a.off_rm[(int64_t)pr.y * a.tl.W + pr.x];
        for (uint32_t i = 0; i < n; ++i) dst[i] = col[i][lane];
    }
    if (a.rgba) {
        const ShadeParams &sp = view_params(a.views, pr.view).sp;
        const VertRec *vert = a.mesh.vert + pr.view * a.mesh.V;
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
        for (uint32_t i = 0; i < n; ++i) {
            const float T = 1.f - A;
            if (T < T_EPS) break;
            const Frag fr = shade(a.mesh, vert, sp, (uint32_t)(col[i][lane] & 0xffffffffu), pr.x, pr.y);
            C0 += T * fr.r;
            C1 += T * fr.g;
            C2 += T * fr.b;
            A += T * fr.a;
        }
        write_rgba(a, pr, sp, C0, C1, C2, A);
    }
}

// One stage of the bitonic network within the lanes' registers: partners r
// and r | J (J < R, a constant: the registers stay statically indexed).
template <int J, int R, class K>
__device__ __forceinline__ void bitonic_inlane(K (&v)[R], int lane, int k) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if ((r & J) == 0) {
            const int r2 = r | J;
            const bool up = ((lane * R + r) & k) == 0;
            const K x = v[r], y = v[r2];
            const bool sw = up ? (x > y) : (x < y);
            v[r] = sw ? y : x;
            v[r2] = sw ? x : y;
        }
    }
}

// Element e = lane*R + r of the padded list lives in register v[r] of `lane`.
template <int R, class K>
__device__ __forceinline__ void bitonic_sort(K (&v)[R], int lane) {
    constexpr int N = 64 * R;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= R) {
                const int lm = j / R;
                const bool lower = (lane & lm) == 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const K o = xor_lane(v[r], lm, lane);
                    const bool up = ((lane * R + r) & k) == 0;
                    v[r] = (lower == up) ? (v[r] < o ? v[r] : o) : (v[r] < o ? o : v[r]);
                }
            } else if constexpr (R < 32) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if ((r & j) == 0) {
                        const int r2 = r | j;
                        const bool up = ((lane * R + r) & k) == 0;
                        const K x = v[r], y = v[r2];
                        const bool sw = up ? (x > y) : (x < y);
                        v[r] = sw ? y : x;
                        v[r2] = sw ? x : y;
                    }
                }
            } else {
                // (32 registers: the stage loops stay rolled, so j is not a
                // constant here; a register index from it would put v in
                // private memory)
                switch (j) {
                    case 1: bitonic_inlane<1>(v, lane, k); break;
                    case 2: bitonic_inlane<2>(v, lane, k); break;
                    case 4: bitonic_inlane<4>(v, lane, k); break;
                    case 8: bitonic_inlane<8>(v, lane, k); break;
                    default: bitonic_inlane<16>(v, lane, k); break;
                }
            }
        }
    }
}

// Ordered wave reduction of premultiplied fragments with the "over"
// operator: lane l's fragment lies in front of lane l + 1's; lane 0 ends with
// the composite of the whole wave.
__device__ __forceinline__ void over_reduce(float &C0, float &C1, float &C2, float &A, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        // (the lanes that combine, lane % 2o == 0, read lane + o = lane ^ o)
        const float q0 = xor_lane(C0, o, lane), q1 = xor_lane(C1, o, lane), q2 = xor_lane(C2, o, lane),
                    qa = xor_lane(A, o, lane);
        if ((lane & (2 * o - 1)) == 0) {
            const float T = 1.f - A;
            C0 += T * q0;
            C1 += T * q1;
            C2 += T * q2;
            A += T * qa;
        }
    }
}

// Shade the sorted list of pixel pr in rounds of 64 fragments (element 64k + l
// to lane l), blend each round with the ordered "over" reduction, and stop
// once the pixel is opaque to within 2^-20: the fragments behind add less
// than that to any channel.  tri_of(k) gives the lane's triangle of round k.
// Only the first `ordered` elements are known to be in list order: a round
// reaching past them returns false before writing anything.
template <int R, class TriOf>
__device__ __forceinline__ bool shade_rounds(const ResolveArgs &a, const PixelRef &pr, uint32_t n, int lane,
                                             uint32_t ordered, TriOf &&tri_of) {
    const ShadeParams &sp = view_params(a.views, pr.view).sp;
    const VertRec *vert = a.mesh.vert + pr.view * a.mesh.V;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;  // blended rounds (uniform over the wave)
    constexpr int UNROLL = R <= 8 ? R : 1;
#pragma unroll UNROLL
    for (int k = 0; k < R; ++k) {
        if (64u * k >= n) break;
        if (64u * (k + 1) > ordered) return false;
        const uint32_t e = 64u * k + lane;
        const uint32_t tri = tri_of(k);
        float c0 = 0.f, c1 = 0.f, c2 = 0.f, ca = 0.f;
        if (e < n) {
            const Frag fr = shade(a.mesh, vert, sp, tri, pr.x, pr.y);
            c0 = fr.r;
            c1 = fr.g;
            c2 = fr.b;
            ca = fr.a;
        }
        over_reduce(c0, c1, c2, ca, lane);
        c0 = lane0(c0);
        c1 = lane0(c1);
        c2 = lane0(c2);
        ca = lane0(ca);
        const float T = 1.f - A;
        C0 += T * c0;
        C1 += T * c1;
        C2 += T * c2;
        A += T * ca;
        if (1.f - A < T_EPS) break;
    }
    if (lane == 0) write_rgba(a, pr, sp, C0, C1, C2, A);
    return true;
}

// Keys (and triangle ids) a wave's LDS stash holds for lists of up to 64 R.
template <int R>
constexpr int STASH_KEYS = R <= 4 ? 256 : 64 * R;

// Wavefront-scope ordering of a wave's LDS stash accesses (stores by some
// lanes, loads by others) without a workgroup barrier.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// List of pixel p (n <= 64 R): one wave, bitonic sort in registers.  Up to
// 512 elements (R <= 8) the sorted keys go to `stash` (2 KB of LDS private to
// the wave, 4 KB for R = 8) for the shading rounds, so that they hold no
// registers across the shading; longer lists keep them in registers.
template <int R>
__device__ __forceinline__ void resolve_wave(const ResolveArgs &a, uint32_t p, uint32_t cnt, uint64_t first, int lane,
                                             uint32_t *__restrict__ stash) {
    uint32_t n = min(cnt, (uint32_t)(64 * R));  // the class guarantees n <= 64 R
    if (first + n > a.rec_cap) n = 0;  // overflowed workspace: records were not stored
    const uint64_t *src = a.rec + first;
    const PixelRef pr = pixel_ref(a.tl, p);
    if constexpr (R <= 8) {
        // Rendering only (no sorted export): sort 32-bit keys (depth << PB |
        // position in the list, PB = 8 position bits up to 256 elements; for
        // 512 the depth gives up its lowest bit to a ninth.  Depths stay below
        // 2^24 - 1, so the padding ~0 sorts last: a list without padding has
        // no key to collide with it); the triangle ids stay in the stash at
        // their list positions.  Equal key depths must be ordered by depth and
        // triangle id, which these keys do not hold: the rounds stop short of
        // the first such pair, and a pixel that needs fragments past it takes
        // the 64-bit sort below.
        constexpr int PB = R <= 4 ? 8 : 9, DROP = PB - 8;
        constexpr uint32_t PMASK = (1u << PB) - 1;
        uint32_t *skey = stash, *stri = stash + STASH_KEYS<R>;
        if (!a.sorted_out) {
            if (!a.rgba) return;
            uint32_t key[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t e = lane * R + r;
                const uint64_t rec = e < n ? src[e] : ~0ull;
                key[r] = e < n ? (((uint32_t)(rec >> 32) >> DROP) << PB) | e : ~0u;
                stri[e] = (uint32_t)rec;
            }
            bitonic_sort<R>(key, lane);
            // first position e with equal depths at e and e + 1
            const uint32_t nxt = __shfl_down(key[0], 1);
            uint32_t tie = ~0u;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t nk = r + 1 < R ? key[r + 1] : nxt;
                const bool t = (r + 1 < R || lane < 63) && lane * R + r + 1 < n && (key[r] >> PB) == (nk >> PB);
                const uint64_t b = __ballot(t);
                if (b) tie = min(tie, (uint32_t)__builtin_ctzll(b) * R + r);
                skey[lane * R + r] = key[r];
            }
            wave_lds_sync();
            const bool done = shade_rounds<R>(a, pr, n, lane, tie,
                                              [&](int k) { return stri[skey[64u * k + lane] & PMASK]; });
            wave_lds_sync();  // (the stash is rewritten next)
            if (done) return;
        }
        uint64_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t e = lane * R + r;
            v[r] = e < n ? src[e] : ~0ull;
        }
        bitonic_sort<R>(v, lane);
        if (a.sorted_out) {
            uint64_t *dst = a.sorted_out + a.off_rm[(int64_t)pr.y * a.tl.W + pr.x];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t e = lane * R + r;
                if (e < n) dst[e] = v[r];
            }
        }
        if (a.rgba) {
            // the sorted triangle ids to the stash, element e at position e
#pragma unroll
            for (int r = 0; r < R; ++r) stri[lane * R + r] = (uint32_t)v[r];
            wave_lds_sync();
            shade_rounds<R>(a, pr, n, lane, ~0u, [&](int k) { return stri[64u * k + lane]; });
            wave_lds_sync();  // (the stash is rewritten by the wave's next list)
        }
    } else {
        uint64_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t e = lane * R + r;
            v[r] = e < n ? src[e] : ~0ull;
        }
        bitonic_sort<R>(v, lane);
        if (a.sorted_out) {
            uint64_t *dst = a.sorted_out + a.off_rm[(int64_t)pr.y * a.tl.W + pr.x];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t e = lane * R + r;
                if (e < n) dst[e] = v[r];
            }
        }
        if (a.rgba)
            shade_rounds<R>(a, pr, n, lane, ~0u, [&](int k) {
                const uint32_t e = 64u * k + lane;
                uint64_t x = ~0ull;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const uint64_t t = __shfl(v[rr], (int)(e / R));
                    if ((int)(e % R) == rr) x = t;
                }
                return (uint32_t)(x & 0xffffffffu);
            });
    }
}

// Ascending compare-exchange of two 64-bit keys at lo < hi.
__device__ __forceinline__ void cmpx(uint64_t *__restrict__ k, uint32_t lo, uint32_t hi) {
    const uint64_t x = k[lo], y = k[hi];
    if (x > y) {
        k[lo] = y;
        k[hi] = x;
    }
}

// Bitonic sort of N (a power of two, <= LCAP) keys in LDS by the workgroup,
// ascending.
__device__ __forceinline__ void block_sort_lds(uint64_t *__restrict__ k, uint32_t N, int tid) {
    for (uint32_t size = 2; size <= N; size <<= 1)
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = tid; i < N / 2; i += RT) {
                const uint32_t lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1)), hi = lo + stride;
                const uint64_t x = k[lo], y = k[hi];
                const bool up = (lo & size) == 0;
                if ((x > y) == up) {
                    k[lo] = y;
                    k[hi] = x;
                }
            }
            __syncthreads();
        }
}

// Half-cleaner stages stride = from .. 1 (ascending) on LDS chunk k of LCAP keys.
__device__ __forceinline__ void block_half_cleaners_lds(uint64_t *__restrict__ k, uint32_t from, int tid) {
    for (uint32_t stride = from; stride > 0; stride >>= 1) {
        for (uint32_t i = tid; i < LCAP / 2; i += RT) {
            const uint32_t lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));
            cmpx(k, lo, lo + stride);
        }
        __syncthreads();
    }
}

// In-place ascending sort of a list of n > LCAP records in global memory by
// one workgroup: every LCAP chunk is sorted in LDS, then the sorted runs are
// merged by the bitonic merge in its ascending-only form (each merge starts by
// comparing element i of a block with its mirror image, then halves), which
// never moves an element past the end of the list: elements beyond n count as
// +infinity and are not touched, so the list needs no padding in memory.
// Strides of at least LCAP go through global memory (the workgroup owns the
// list; its barriers order the accesses), shorter ones through LDS chunks.
// Reordering the records within the list is harmless: every reader sorts.
__device__ void block_sort_global(uint64_t *__restrict__ g, uint32_t n, uint64_t *__restrict__ lds, int tid) {
    const uint32_t nch = (n + LCAP - 1) / LCAP;
    auto load_chunk = [&](uint32_t c) {
        const uint32_t b = c * LCAP, m = min((uint32_t)LCAP, n - b);
        for (uint32_t i = tid; i < LCAP; i += RT) lds[i] = i < m ? g[b + i] : ~0ull;
        __syncthreads();
        return m;
    };
    auto store_chunk = [&](uint32_t c, uint32_t m) {
        for (uint32_t i = tid; i < m; i += RT) g[c * LCAP + i] = lds[i];
        __syncthreads();
    };
    for (uint32_t c = 0; c < nch; ++c) {
        const uint32_t m = load_chunk(c);
        block_sort_lds(lds, LCAP, tid);
        store_chunk(c, m);
    }
    uint32_t N = LCAP;
    while (N < n) N <<= 1;
    for (uint32_t size = 2 * LCAP; size <= N; size <<= 1) {
        const uint32_t h = size >> 1;
        for (uint32_t i = tid; i < N / 2; i += RT) {  // mirror stage
            const uint32_t blk = i / h, r = i % h;
            const uint32_t lo = blk * size + r, hi = blk * size + size - 1 - r;
            if (hi < n) cmpx(g, lo, hi);
        }
        __syncthreads();
        for (uint32_t stride = size >> 2; stride >= LCAP; stride >>= 1) {
            for (uint32_t i = tid; i < N / 2; i += RT) {
                const uint32_t lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1)), hi = lo + stride;
                if (hi < n) cmpx(g, lo, hi);
            }
            __syncthreads();
        }
        for (uint32_t c = 0; c < nch; ++c) {
            const uint32_t m = load_chunk(c);
            block_half_cleaners_lds(lds, LCAP / 2, tid);
            store_chunk(c, m);
        }
    }
}

struct BlockLds {
    uint64_t keys[LCAP];
    float4 red[RT / 64];
};

// Very long list of pixel p (n > 2048): one workgroup sorts it in place and
// shades it in rounds of 256 fragments, the four waves' ordered composites
// being combined in wave order.
__device__ void resolve_block(const ResolveArgs &a, uint64_t base, uint32_t p, BlockLds &L, int tid) {
    uint32_t n = a.count[p];
    const uint64_t first = a.off[p] - base;
    if (first + n > a.rec_cap) n = 0;  // overflowed workspace: records were not stored
    uint64_t *src = a.rec + first;
    const bool in_lds = n <= (uint32_t)LCAP;
    if (in_lds) {
        uint32_t N = 64;
        while (N < n) N <<= 1;
        for (uint32_t i = tid; i < N; i += RT) L.keys[i] = i < n ? src[i] : ~0ull;
        __syncthreads();
        block_sort_lds(L.keys, N, tid);
    } else {
        block_sort_global(src, n, L.keys, tid);
    }
    const uint64_t *sorted = in_lds ? L.keys : src;
    const PixelRef pr = pixel_ref(a.tl, p);
    if (a.sorted_out) {
        uint64_t *dst = a.sorted_out + a.off_rm[(int64_t)pr.y * a.tl.W + pr.x];
        for (uint32_t i = tid; i < n; i += RT) dst[i] = sorted[i];
    }
    if (a.rgba) {
        const int lane = tid & 63, wave = tid >> 6;
        const ShadeParams &sp = view_params(a.views, pr.view).sp;
        const VertRec *vert = a.mesh.vert + pr.view * a.mesh.V;
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;  // uniform over the workgroup
        for (uint32_t r0 = 0; r0 < n; r0 += RT) {
            const uint32_t e = r0 + tid;
            float c0 = 0.f, c1 = 0.f, c2 = 0.f, ca = 0.f;
            if (e < n) {
                const Frag fr = shade(a.mesh, vert, sp, (uint32_t)(sorted[e] & 0xffffffffu), pr.x, pr.y);
                c0 = fr.r;
                c1 = fr.g;
                c2 = fr.b;
                ca = fr.a;
            }
            over_reduce(c0, c1, c2, ca, lane);
            if (lane == 0) L.red[wave] = make_float4(c0, c1, c2, ca);
            __syncthreads();
#pragma unroll
            for (int w = 0; w < RT / 64; ++w) {
                const float4 q = L.red[w];
                const float T = 1.f - A;
                C0 += T * q.x;
                C1 += T * q.y;
                C2 += T * q.z;
                A += T * q.w;
            }
            __syncthreads();  // L.red is rewritten by the next round
            if (1.f - A < T_EPS) break;
        }
        if (tid == 0) write_rgba(a, pr, sp, C0, C1, C2, A);
    }
    __syncthreads();  // L.keys is reused by the next item
}

__device__ __forceinline__ uint32_t class_size(const ClassWork &w) {
    return w.n_dev ? (uint32_t)*w.n_dev : w.n_host;
}

// Dynamic distribution of a class list over the resident waves (what a grid
// of one workgroup per list item would get from the hardware dispatcher,
// without knowing the list's size when the grid is launched).  The list is
// cut into 8 contiguous parts, one per XCD (workgroups are dealt to the XCDs
// round-robin, and an XCD's waves share an L2 in which neighbouring pixels
// find the faces they shade), each part into SEGS / 8 segments with a
// counter of their own (pops on one address serialise: the classes that pop
// one item at a time take more segments); a wave pops the next item of its
// home segment, with the next pop in flight while it works on the current
// one, then helps with what is left of its XCD's other segments and then of
// the other XCDs'.  `body(item)` is called by the whole wave with a
// wave-uniform item.
template <int PER_POP, int SEGS, class Body>
__device__ __forceinline__ void drain(uint32_t total, uint32_t *__restrict__ queue, int lane, Body &&body) {
    static_assert(SEGS % 8 == 0 && SEGS <= QUEUE_SEGS, "queue segments");
    constexpr int SUB = SEGS / 8;
    const int xcd = blockIdx.x & 7, sub = (blockIdx.x >> 3) % SUB;
#pragma unroll 1
    for (int h = 0; h < SEGS; ++h) {
        const int x = ((xcd + h / SUB) & 7) * SUB + (sub + h) % SUB;
        const uint32_t lo = (uint32_t)((uint64_t)total * x / SEGS),
                       hi = (uint32_t)((uint64_t)total * (x + 1) / SEGS);
        uint32_t *ctr = queue + x * QUEUE_STRIDE;
        if (lo == hi || (h && __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= hi - lo))
            continue;  // (an empty segment, or one already taken)
        uint32_t got = 0;
        if (lane == 0) got = atomicAdd(ctr, (uint32_t)PER_POP);
        uint32_t it = lo + __builtin_amdgcn_readfirstlane(got);
        while (it < hi) {
            uint32_t next = 0;
            if (lane == 0) next = atomicAdd(ctr, (uint32_t)PER_POP);  // (in flight during the items below)
#pragma unroll 1
            for (uint32_t j = it; j < min(it + PER_POP, hi); ++j) body(j);
            it = lo + __builtin_amdgcn_readfirstlane(next);
        }
    }
}

// Short lists (class 0): a lane per pixel, 64 pixels per workgroup; the grid
// covers a bound of the class size (most pixels are short: few workgroups
// find nothing to do), dealt to the XCDs in contiguous ranges of the true
// size, each workgroup a chunk as the hardware dispatches it.
template <int TS>
__global__ void __launch_bounds__(64) k_resolve_short(ClassWork w, ResolveArgs a) {
    __shared__ uint64_t col[TS][64];
    const int lane = threadIdx.x;
    const uint32_t total = class_size(w);
    const uint32_t chunks = (total + 63) / 64;
    if (blockIdx.x >= chunks && gridDim.x >= chunks) return;
    const uint64_t base = rec_base(a);
    // (a grid smaller than the list strides over it)
    for (uint32_t b = blockIdx.x; b < chunks; b += gridDim.x) {
        const uint32_t chunk = gridDim.x >= chunks ? xcd_contiguous(b, chunks) : b;
        const uint32_t idx = chunk * 64 + lane;
        if (idx >= total) continue;
        const uint32_t p = w.list[idx];
        if (p != PIX_SKIP) resolve_lane<TS>(a, base, p, col, lane);
    }
}

// Wave-per-pixel lists (classes 1..6).  Up to 8 keys per lane the kernel is
// held to a register budget that keeps WAVES_R waves per SIMD resident.
template <int R>
__device__ __forceinline__ void resolve_waves(const ClassWork &w, const ResolveArgs &a) {
    __shared__ uint32_t stash[RT / 64][R <= 8 ? 2 * STASH_KEYS<R> : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t total = class_size(w);
    if (!total) return;
    const uint64_t base = rec_base(a);
    // (short lists take several items per pop: their work would not hide its latency)
    drain<R == 1 ? 4 : R == 2 ? 2 : 1, R == 4 ? 64 : 8>(total, w.queue, lane, [&](uint32_t item) {
        const uint32_t p = w.list[item];
        if (p != PIX_SKIP) resolve_wave<R>(a, p, a.count[p], a.off[p] - base, lane, stash[wave]);
    });
}
template <int R>
constexpr int WAVES_R = R <= 2 ? 7 : R == 4 ? 6 : 5;
template <int R>
__global__ void __launch_bounds__(RT) __attribute__((amdgpu_waves_per_eu(WAVES_R<R>, 8))) k_resolve_wave(ClassWork w,
                                                                                                        ResolveArgs a) {
    resolve_waves<R>(w, a);
}
template <int R>
__global__ void __launch_bounds__(RT) k_resolve_wave_wide(ClassWork w, ResolveArgs a) {
    resolve_waves<R>(w, a);
}

// Lists longer than 2048 (class 7): a workgroup per pixel (few of them:
// dealt round-robin to the workgroups).
__global__ void __launch_bounds__(RT) k_resolve_block(ClassWork w, ResolveArgs a) {
    __shared__ BlockLds L;
    const uint32_t total = class_size(w);
    if (!total) return;
    const uint64_t base = rec_base(a);
    for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
        const uint32_t p = w.list[it];
        if (p != PIX_SKIP) resolve_block(a, base, p, L, threadIdx.x);
    }
}

// Workgroups of each class kernel the device holds at once (the grid is never
// smaller: a low estimate then costs the balance of a persistent grid, not
// a few workgroups striding over a long list), at most `cap` per CU: the
// wave-per-pixel kernels' workgroups hold one wave per SIMD each, and more
// resident waves than a class needs to hide its latency only compete for the
// caches and leave less room to the long classes on the second stream
// (measured best: 5 waves per SIMD for classes 1 and 2, 6 for class 3; their
// registers would allow 7).
template <class K>
static int resident(int device, K kernel, int threads, int cap = 1 << 20) {
    int cus = 0, per = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0);
    return std::max(1, cus) * std::max(1, std::min(per, cap));
}

void resolve_min_grids(int device, int out[NCLASS + 2]) {
    out[0] = resident(device, k_resolve_short<16>, 64);
    out[1] = resident(device, k_resolve_wave<1>, RT, 5);
    out[2] = resident(device, k_resolve_wave<2>, RT, 5);
    out[3] = resident(device, k_resolve_wave<4>, RT, 6);
    out[4] = resident(device, k_resolve_wave<8>, RT);
    out[5] = resident(device, k_resolve_wave_wide<16>, RT);
    out[6] = resident(device, k_resolve_wave_wide<32>, RT);
    out[7] = resident(device, k_resolve_block, RT);
    out[8] = resident(device, k_resolve_short<32>, 64);
    out[9] = resident(device, k_resolve_short<64>, 64);
}

void launch_resolve_class(int c, const ClassWork &w, uint32_t est, int t_sort, const int min_grid[NCLASS + 2],
                          const ResolveArgs &a, hipStream_t s) {
    // class 0: a workgroup per 64 pixels of est (here a bound of the class
    // size); classes 1..6 drain their lists dynamically on a resident grid,
    // smaller when the list is known to be short; class 7: a workgroup per list
    const unsigned per = c == 0 ? 64u : c == 7 ? 1u : 4u;  // pixels per workgroup
    const unsigned res = (unsigned)(c == 0 ? min_grid[t_sort <= 16 ? 0 : t_sort <= 32 ? 8 : 9] : min_grid[c]);
    const unsigned need = est == ~0u ? res : (est + per - 1) / per;
    const dim3 g(std::max(1u, c == 0   ? std::min(std::max(need, res), 1u << 22)
                              : c == 7 ? std::min(std::max(need, 64u), res)
                                       : std::min(need + 64u, res)));
    switch (c) {
        case 0:
            if (t_sort <= 16) k_resolve_short<16><<<g, 64, 0, s>>>(w, a);
            else if (t_sort <= 32) k_resolve_short<32><<<g, 64, 0, s>>>(w, a);
            else k_resolve_short<64><<<g, 64, 0, s>>>(w, a);
            break;
        case 1: k_resolve_wave<1><<<g, RT, 0, s>>>(w, a); break;
        case 2: k_resolve_wave<2><<<g, RT, 0, s>>>(w, a); break;
        case 3: k_resolve_wave<4><<<g, RT, 0, s>>>(w, a); break;
        case 4: k_resolve_wave<8><<<g, RT, 0, s>>>(w, a); break;
        case 5: k_resolve_wave_wide<16><<<g, RT, 0, s>>>(w, a); break;
        case 6: k_resolve_wave_wide<32><<<g, RT, 0, s>>>(w, a); break;
        default: k_resolve_block<<<g, RT, 0, s>>>(w, a); break;
    }
}

// ------------------------------------------------------------------ learned tail: head and tail features
// Wave per pixel, as the long-list resolve.  The head (the first K fragments
// in list order) is shaded exactly, one fragment per lane, and composited in
// order.  Every tail fragment gets the proxy shading of its face (opacity
// from the mean corner importance and the focus factor at the face centre,
// colour from the mean corner importance) from which the features are
// accumulated: tail length, proxy opacity sum, opacity-weighted mean depth
// and mean squared depth, the ordered composite of the proxies and the depth
// where the tail starts.
//   TAIL_FEATURES  every row gets its head and features (full sort)
//   TAIL_TRAIN     as TAIL_FEATURES, plus the exact composite of the tail
//                  (the regression target)
//   TAIL_RESOLVE   the learned resolve: the head comes from a selection of
//                  the K smallest records (no sort); a pixel whose head is opaque to
//                  within 2^-20 (and at least conf_min, so that its confidence
//                  accepts it whatever the network says) gets the head over
//                  the background as its final colour, mask 0 and no row
//                  (pix PIX_SKIP, zero features): its tail is invisible.  Only
//                  the other pixels sort the whole list for the ordered proxy.
enum { TAIL_FEATURES = 0, TAIL_TRAIN = 1, TAIL_RESOLVE = 2 };

__device__ __forceinline__ float wave_sum(float v) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += xor_lane(v, o, lane);
    return v;
}

// The head of a list without sorting it: the m = min(K, n) smallest records
// of the wave's 64 R keys (element e = lane R + r in v[r], padding ~0; the
// records of a list are distinct), ascending, one per lane: lane l < m gets
// the l-th smallest in `h`.  A bitwise search over the 25-bit high words
// (counting with ballots) finds the high word h* of the K-th smallest; the
// keys below it are in the head, and of those equal to it the ones with the
// smallest low words (a second search, only when more of them tie than there
// are places left).  The m chosen keys are compacted through the wave's LDS
// `stash` (2 KK words) and ranked by comparing each with all the others.
template <int R, int KK>
__device__ __forceinline__ uint32_t wave_head(const uint64_t (&v)[R], uint32_t n, int K, int lane,
                                              uint64_t *__restrict__ stash, uint64_t &h) {
    const uint32_t m = min((uint32_t)K, n);
    uint32_t hi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) hi[r] = (uint32_t)(v[r] >> 32);
    auto count_below = [&](uint32_t t) {  // keys whose high word is below t (wave-uniform)
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) c += (uint32_t)__popcll(__ballot(hi[r] < t));
        return c;
    };
    uint32_t hs = 0;
    for (int b = 24; b >= 0; --b) {
        const uint32_t t = hs | (1u << b);
        if (count_below(t) < m) hs = t;
    }
    // places left for keys with high word hs, and how many there are
    const uint32_t less = count_below(hs);
    uint32_t eq = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) eq += (uint32_t)__popcll(__ballot(hi[r] == hs));
    const uint32_t need = m - less;
    uint32_t lo_cut = 0xffffffffu;  // keys with high word hs and low word <= lo_cut are in
    if (eq > need) {
        uint32_t ls = 0;
        for (int b = 31; b >= 0; --b) {
            const uint32_t t = ls | (1u << b);
            uint32_t c = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) c += (uint32_t)__popcll(__ballot(hi[r] == hs && (uint32_t)v[r] < t));
            if (c < need) ls = t;
        }
        lo_cut = ls;  // the need-th smallest low word among the ties
    }
    // compact the chosen keys into stash[0..m-1] (any order)
    const uint64_t below = (1ull << lane) - 1;
    uint32_t base = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool in = hi[r] < hs || (hi[r] == hs && (uint32_t)v[r] <= lo_cut && (lane * R + r) < (int)n);
        const uint64_t bal = __ballot(in);
        if (in) stash[base + __popcll(bal & below)] = v[r];
        base += (uint32_t)__popcll(bal);
    }
    wave_lds_sync();
    // rank: lane l < m places its key at its position in ascending order
    uint64_t mine = ~0ull;
    uint32_t rank = 0;
    if ((uint32_t)lane < m) {
        mine = stash[lane];
        for (uint32_t j = 0; j < m; ++j) rank += stash[j] < mine;
    }
    if ((uint32_t)lane < m) stash[KK + rank] = mine;
    wave_lds_sync();
    h = (uint32_t)lane < m ? stash[KK + lane] : ~0ull;
    wave_lds_sync();  // (the stash is rewritten by the wave's next list)
    return m;
}

// Head composite of pixel pr from the head key h of lane l < m (element l
// in list order); the result is uniform over the wave.
__device__ __forceinline__ float4 head_composite(const ResolveArgs &a, const PixelRef &pr, uint64_t h, uint32_t m,
                                                 int lane) {
    float H0 = 0.f, H1 = 0.f, H2 = 0.f, HA = 0.f;
    if ((uint32_t)lane < m) {
        const ViewParams &vp = view_params(a.views, pr.view);
        const Frag fr = shade(a.mesh, a.mesh.vert + pr.view * a.mesh.V, vp.sp, (uint32_t)(h & 0xffffffffu), pr.x, pr.y);
        H0 = fr.r;
        H1 = fr.g;
        H2 = fr.b;
        HA = fr.a;
    }
    over_reduce(H0, H1, H2, HA, lane);
    return make_float4(lane0(H0), lane0(H1), lane0(H2), lane0(HA));
}

// Sorts the records v (element e = lane R + r, padding ~0) through 32-bit
// keys (depth << 8 | list position: exact depths, up to 256 elements)
// sorted in registers, the records gathered back from the wave's LDS stash
// in key order.  A list with equal depths takes the 64-bit sort instead: its
// order then depends on the triangle ids, which the keys do not hold.
template <int R>
__device__ __forceinline__ void sort_records(uint64_t (&v)[R], uint32_t n, int lane, uint64_t *__restrict__ rs) {
    static_assert(R <= 4, "8 position bits");
    wave_lds_sync();  // (the stash's previous use is over)
    uint32_t key[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = lane * R + r;
        rs[e] = v[r];
        key[r] = e < n ? ((uint32_t)(v[r] >> 32) << 8) | e : ~0u;
    }
    bitonic_sort<R>(key, lane);
    const uint32_t nxt = __shfl_down(key[0], 1);
    bool tie = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t nk = r + 1 < R ? key[r + 1] : nxt;
        tie |= (r + 1 < R || lane < 63) && lane * R + r + 1 < n && (key[r] >> 8) == (nk >> 8);
    }
    if (__any(tie)) {
        bitonic_sort<R>(v, lane);  // (v is unchanged so far)
        return;
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = key[r] == ~0u ? ~0ull : rs[key[r] & 0xffu];
}

// Row `item` of a class list: one wave.  `stash` is the wave's LDS (head
// selection, then the 32-bit sort's records).
template <int R, int MODE>
__device__ __forceinline__ void tail_item(uint32_t item, const uint32_t *__restrict__ list, int K, float conf_min,
                                          const ResolveArgs &a, float *__restrict__ head, float *__restrict__ feat,
                                          float *__restrict__ target, uint32_t *__restrict__ pix_out,
                                          uint8_t *__restrict__ mask, bool rowmajor, int64_t out_base,
                                          uint64_t *__restrict__ stash, int lane) {
    constexpr bool TRAIN = MODE == TAIL_TRAIN;
    const uint32_t p = list[item];
    uint32_t n = min(a.count[p], (uint32_t)(64 * R));
    const uint64_t first = a.off[p] - rec_base(a);
    if (first + n > a.rec_cap) n = 0;
    const uint64_t *src = a.rec + first;
    uint64_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = lane * R + r;
        v[r] = e < n ? src[e] : ~0ull;
    }
    const PixelRef pr = pixel_ref(a.tl, p);
    const ViewParams &vp = view_params(a.views, pr.view);
    const ShadeParams &sp = vp.sp;
    const VertRec *vert = a.mesh.vert + pr.view * a.mesh.V;
    const int64_t o = out_base + item;
    float H0 = 0.f, H1 = 0.f, H2 = 0.f, HA = 0.f;
    bool have_head = false;
    if constexpr (MODE == TAIL_RESOLVE) {
        uint64_t hk;
        const uint32_t m = wave_head<R, 64>(v, n, K, lane, stash, hk);
        const float4 h = head_composite(a, pr, hk, m, lane);
        if (n > (uint32_t)K && 1.f - h.w < T_EPS && h.w >= conf_min) {
            // the tail is invisible: final colour now, no row for the network
            if (lane == 0) {
                write_rgba(a, pr, sp, h.x, h.y, h.z, h.w);
                if (mask) mask[(pr.view * a.tl.H + pr.y) * (int64_t)a.tl.W + pr.x] = 0;
                reinterpret_cast<float4 *>(head)[o] = h;
                pix_out[o] = PIX_SKIP;
            }
            if (lane < NFEAT) feat[o * NFEAT + lane] = 0.f;
            return;
        }
        H0 = h.x;
        H1 = h.y;
        H2 = h.z;
        HA = h.w;
        have_head = true;
    }
    if constexpr (MODE == TAIL_RESOLVE && R <= 4)
        sort_records<R>(v, n, lane, stash);
    else
        bitonic_sort<R>(v, lane);
    if (!have_head) {
        // head: sorted element l to lane l, one exact shade per lane
        uint64_t hv = ~0ull;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const uint64_t t = __shfl(v[rr], lane / R);
            if (lane % R == rr) hv = t;
        }
        if (lane < K && (uint32_t)lane < n) {
            const Frag fr = shade(a.mesh, vert, sp, (uint32_t)(hv & 0xffffffffu), pr.x, pr.y);
            H0 = fr.r;
            H1 = fr.g;
            H2 = fr.b;
            HA = fr.a;
        }
        over_reduce(H0, H1, H2, HA, lane);
    }
    const float zs = 1.f / (vp.w1 - vp.w0);
    float T0 = 0.f, T1 = 0.f, T2 = 0.f, TA = 0.f;  // exact tail composite (TRAIN)
    float P0 = 0.f, P1 = 0.f, P2 = 0.f, PA = 0.f;  // ordered proxy composite
    float sa = 0.f, sz1 = 0.f, sz2 = 0.f, zf = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = lane * R + r;
        if (e >= n || (int)e < K) continue;
        const uint32_t tri = (uint32_t)(v[r] & 0xffffffffu);
        if (TRAIN) {
            const Frag fr = shade(a.mesh, vert, sp, tri, pr.x, pr.y);
            const float T = 1.f - TA;
            T0 += T * fr.r;
            T1 += T * fr.g;
            T2 += T * fr.b;
            TA += T * fr.a;
        }
        const float4 fp = a.mesh.face_px[tri >> 1];
        const float dx = fp.x - sp.hc[0], dy = fp.y - sp.hc[1], dz = fp.z - sp.hc[2];
        const float dist = fminf(__builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz) * sp.inv_r, 1.f);
        const float d2 = dist * dist;
        const float al = (sp.a_lo + (sp.a_hi - sp.a_lo) * fp.w) * d2 * d2;
        const float key = (float)(KMAX - (uint32_t)(v[r] >> 32));
        const float z = fminf(fmaxf((1048576.f * __builtin_amdgcn_rcpf(key) - vp.w0) * zs, 0.f), 1.f);
        sa += al;
        sz1 += al * z;
        sz2 += al * z * z;
        const float T = 1.f - PA;
        P0 += T * al * (sp.lo[0] + (sp.hi[0] - sp.lo[0]) * fp.w);
        P1 += T * al * (sp.lo[1] + (sp.hi[1] - sp.lo[1]) * fp.w);
        P2 += T * al * (sp.lo[2] + (sp.hi[2] - sp.lo[2]) * fp.w);
        PA += T * al;
        if ((int)e == K) zf = z;
    }
    if (TRAIN) over_reduce(T0, T1, T2, TA, lane);
    over_reduce(P0, P1, P2, PA, lane);
    sa = wave_sum(sa);
    sz1 = wave_sum(sz1);
    sz2 = wave_sum(sz2);
    zf = wave_sum(zf);
    if (lane == 0) {
        const float inv = sa > 0.f ? 1.f / sa : 0.f;
        float *F = feat + o * NFEAT;
        F[0] = log1pf((float)max((int)n - K, 0));
        F[1] = sa;
        F[2] = sz1 * inv;
        F[3] = sz2 * inv;
        F[4] = P0;
        F[5] = P1;
        F[6] = P2;
        F[7] = PA;
        F[8] = zf;
        reinterpret_cast<float4 *>(head)[o] = make_float4(H0, H1, H2, HA);
        if (TRAIN) reinterpret_cast<float4 *>(target)[o] = make_float4(T0, T1, T2, TA);
        pix_out[o] = rowmajor ? (uint32_t)((pr.view * a.tl.H + pr.y) * a.tl.W + pr.x) : p;
    }
}

// The rows of one length class on a resident grid: the waves drain the
// class list through its queue counters (zeroed before the launch), as the
// exact resolve's class kernels do.
template <int R, int MODE>
__global__ void __launch_bounds__(256) k_tail_features(const uint32_t *__restrict__ list, uint32_t npix,
                                                       uint32_t *__restrict__ queue, int K, float conf_min,
                                                       ResolveArgs a, float *__restrict__ head,
                                                       float *__restrict__ feat, float *__restrict__ target,
                                                       uint32_t *__restrict__ pix_out, uint8_t *__restrict__ mask,
                                                       bool rowmajor, int64_t out_base) {
    __shared__ uint64_t stash[4][MODE == TAIL_RESOLVE ? (R <= 2 ? 128 : 64 * R) : 1];
    const int lane = threadIdx.x & 63;
    if (!npix) return;
    drain<R == 1 ? 4 : R == 2 ? 2 : 1, 64>(npix, queue, lane, [&](uint32_t item) {
        wave_lds_sync();  // (the wave's stash is reused item after item)
        tail_item<R, MODE>(item, list, K, conf_min, a, head, feat, target, pix_out, mask, rowmajor, out_base,
                           stash[threadIdx.x >> 6], lane);
    });
}

// ------------------------------------------------------------------ silhouettes
// White exterior and interior screen-space silhouettes of the mesh boundary
// surface (the faces of one cell only): its depth buffer is read off the
// fragment lists (the nearest boundary fragment of each pixel), and a pixel
// that sees it is a silhouette pixel when a 4-neighbour inside the image sees
// none or sees it more than (1 + tau) farther (the depth keys are inverse
// depths, so the test is key_p > (1 + tau) key_n, in FP64).
__global__ void __launch_bounds__(256) k_boundary_depth(Tiling tl, const uint64_t *__restrict__ pass_tiles,
                                                        const ViewParams *__restrict__ views,
                                                        const uint32_t *__restrict__ count,
                                                        const uint64_t *__restrict__ off,
                                                        const uint64_t *__restrict__ rec, uint64_t rec_cap,
                                                        const uint8_t *__restrict__ face_bnd,
                                                        uint32_t *__restrict__ bdepth) {
    const int64_t TPX = (int64_t)tl.TW * tl.TH;
    const int64_t p0 = (int64_t)pass_tiles[0] * TPX, p1 = (int64_t)pass_tiles[1] * TPX;
    const int64_t p = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= p1) return;
    const int64_t view = p / ((int64_t)tl.ntiles * TPX);
    if (!(view_params(views, view).sp.sil_a > 0.f)) return;
    uint32_t n = count[p];
    const uint64_t first = off[p] - off[p0];
    if (first + n > rec_cap) n = 0;
    uint64_t best = ~0ull;
    for (uint32_t k = 0; k < n; ++k) {
        const uint64_t r = rec[first + k];
        if (r < best && face_bnd[(uint32_t)(r & 0xffffffffu) >> 1]) best = r;
    }
    bdepth[p] = best == ~0ull ? 0u : KMAX - (uint32_t)(best >> 32);
}

__global__ void __launch_bounds__(256) k_silhouette(Tiling tl, int64_t npx, const ViewParams *__restrict__ views,
                                                    const uint32_t *__restrict__ bdepth, float *__restrict__ rgba) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // row-major over views
    if (i >= npx) return;
    const int64_t WH = (int64_t)tl.W * tl.H;
    const int64_t view = i / WH;
    const ShadeParams &sp = view_params(views, view).sp;
    const float a = sp.sil_a;
    if (!(a > 0.f)) return;
    const int x = (int)((i - view * WH) % tl.W), y = (int)((i - view * WH) / tl.W);
    const int64_t vbase = view * (int64_t)tl.ntiles * tl.TW * tl.TH;
    auto tm = [&](int xx, int yy) {
        return vbase + ((int64_t)(yy / tl.TH) * tl.ntx + xx / tl.TW) * (tl.TW * tl.TH) + (yy % tl.TH) * tl.TW +
               xx % tl.TW;
    };
    const uint32_t kp = bdepth[tm(x, y)];
    if (kp == 0) return;
    const double lim = 1.0 + (double)sp.sil_tau;
    const int nx[4] = {x - 1, x + 1, x, x}, ny[4] = {y, y, y - 1, y + 1};
    bool sil = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (nx[q] < 0 || ny[q] < 0 || nx[q] >= tl.W || ny[q] >= tl.H) continue;
        const uint32_t kn = bdepth[tm(nx[q], ny[q])];
        sil |= kn == 0 || (double)kp > lim * (double)kn;
    }
    if (!sil) return;
    float4 *o = reinterpret_cast<float4 *>(rgba) + i;
    float4 c = *o;
    c.x = (1.f - a) * c.x + a;
    c.y = (1.f - a) * c.y + a;
    c.z = (1.f - a) * c.z + a;
    c.w = a + (1.f - a) * c.w;
    *o = c;
}

void launch_boundary_depth(const Tiling &tl, int nv, const uint64_t *pass_tiles, const ViewParams *views,
                           const uint32_t *count, const uint64_t *off, const uint64_t *rec, uint64_t rec_cap,
                           const uint8_t *face_bnd, uint32_t *bdepth, hipStream_t s) {
    const int64_t n = (int64_t)tl.ntiles * nv * tl.TW * tl.TH;
    if (n <= 0) return;
    k_boundary_depth<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(tl, pass_tiles, views, count, off, rec, rec_cap,
                                                                      face_bnd, bdepth);
}

void launch_silhouette(const Tiling &tl, int nv, const ViewParams *views, const uint32_t *bdepth, float *rgba,
                       hipStream_t s) {
    const int64_t n = (int64_t)nv * tl.W * tl.H;
    if (n <= 0) return;
    k_silhouette<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(tl, n, views, bdepth, rgba);
}

// ------------------------------------------------------------------ approximate resolves
// Order-independent approximations of the sorted blend on the same lists,
// one wave per pixel, every fragment shaded:
//  * multi-layer alpha blending: the list is sorted by triangle id (the
//    primitive order a rasteriser would deliver), then the wave runs the k
//    blending nodes in lockstep (every lane holds the same nodes) over the
//    fragments broadcast one at a time; a new fragment is inserted at its
//    depth (after nodes of equal depth) and the last two nodes merge when
//    there are k + 1;
//  * moment-based transparency with four power moments of the absorbance
//    over the warped depth, and per fragment the Hamburger bound of the
//    absorbance in front of it (three-point canonical distribution through
//    the fragment's depth), in FP64.
constexpr double MOM_BETA = 5e-5, MOM_ETA = 0.25;

__device__ double moment_fraction(const double (&m)[5], double x) {
    // monic cubic t^3 + p2 t^2 + p1 t + p0 with E[P] = E[X P] = 0 and P(x) = 0
    double A[3][4] = {{1.0, m[1], m[2], -m[3]}, {m[1], m[2], m[3], -m[4]}, {1.0, x, x * x, -x * x * x}};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int piv = c;
#pragma unroll
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double t = A[c][q];
            A[c][q] = piv == 1 && c == 0 ? A[1][q] : (piv == 2 ? A[2][q] : A[c][q]);
            if (piv == 1 && c == 0) A[1][q] = t;
            if (piv == 2) A[2][q] = t;
        }
        if (A[c][c] == 0.0) return MOM_ETA;
#pragma unroll
        for (int r = c + 1; r < 3; ++r) {
            const double f = A[r][c] / A[c][c];
#pragma unroll
            for (int q = 0; q < 4; ++q) A[r][q] -= q >= c ? f * A[c][q] : 0.0;
        }
    }
    const double p2 = A[2][3] / A[2][2];
    const double p1 = (A[1][3] - A[1][2] * p2) / A[1][1];
    // the quadratic factor P(t) / (t - x) = t^2 + bq t + cq
    const double bq = p2 + x, cq = p1 + x * bq;
    const double sq = sqrt(fmax(bq * bq - 4.0 * cq, 0.0));
    const double z2 = 0.5 * (-bq - sq), z3 = 0.5 * (-bq + sq);
    const double d2 = (z2 - x) * (z2 - z3), d3 = (z3 - x) * (z3 - z2);
    const double w2 = d2 != 0.0 ? (m[2] - m[1] * (x + z3) + x * z3) / d2 : 0.0;
    const double w3 = d3 != 0.0 ? (m[2] - m[1] * (x + z2) + x * z2) / d3 : 0.0;
    const double w1 = 1.0 - w2 - w3;
    const double F = (z2 < x ? w2 : 0.0) + (z3 < x ? w3 : 0.0) + MOM_ETA * w1;
    return fmin(fmax(F, 0.0), 1.0);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Loads a pixel's records (lane-blocked: lane l holds elements l*R .. l*R+R-1).
template <int R>
__device__ __forceinline__ uint32_t load_list(const ResolveArgs &a, uint32_t p, int lane, uint64_t (&v)[R]) {
    uint32_t n = min(a.count[p], (uint32_t)(64 * R));
    const uint64_t first = a.off[p] - rec_base(a);
    if (first + n > a.rec_cap) n = 0;
    const uint64_t *src = a.rec + first;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = lane * R + r;
        v[r] = e < n ? src[e] : ~0ull;
    }
    return n;
}

// Multi-layer alpha blending: one wave per workgroup; the shaded fragments
// are staged in LDS in primitive order and the wave walks them in lockstep.
// Multi-layer alpha blending in two passes.  Shade: one wave per pixel sorts
// the list by triangle id and shades every fragment, writing (colour,
// opacity) and the depth field to a scratch array laid out like the records.
// Blend: one lane per pixel runs the node insertions over its fragments in
// that order (the insertions are sequential by definition; a lane per pixel
// keeps them off the other 63 lanes).
template <int R>
__global__ void __launch_bounds__(256) k_mlab_shade(const uint32_t *__restrict__ list, uint32_t npix, ResolveArgs a,
                                                    float4 *__restrict__ mc, uint32_t *__restrict__ mz) {
    const int lane = threadIdx.x & 63;
    const uint32_t wave = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (wave >= npix) return;
    const uint32_t p = list[wave];
    uint64_t v[R];
    const uint32_t n = load_list<R>(a, p, lane, v);
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = (v[r] << 32) | (v[r] >> 32);  // triangle id first: primitive order
    bitonic_sort<R>(v, lane);
    const PixelRef pr = pixel_ref(a.tl, p);
    const ShadeParams &sp = view_params(a.views, pr.view).sp;
    const VertRec *vert = a.mesh.vert + pr.view * a.mesh.V;
    const uint64_t first = a.off[p] - rec_base(a);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = lane * R + r;
        if (e < n) {
            const Frag fr = shade(a.mesh, vert, sp, (uint32_t)(v[r] >> 32), pr.x, pr.y);
            mc[first + e] = make_float4(fr.r, fr.g, fr.b, fr.a);
            mz[first + e] = (uint32_t)(v[r] & 0xffffffffu);
        }
    }
}

// The k blending nodes of one pixel (up to k + 1 <= 9 while inserting).
struct MlabNodes {
    float c0[9], c1[9], c2[9], T[9];
    uint32_t z[9];
    int cnt = 0;
    // insert at its depth (after the nodes of equal or smaller depth); merge
    // the last two nodes when there are k + 1
    __device__ __forceinline__ void insert(const float4 x, uint32_t xz, int k) {
        int pos = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) pos += (q < cnt && z[q] <= xz) ? 1 : 0;
#pragma unroll
        for (int q = 8; q > 0; --q)
            if (q > pos && q <= cnt) {
                c0[q] = c0[q - 1];
                c1[q] = c1[q - 1];
                c2[q] = c2[q - 1];
                T[q] = T[q - 1];
                z[q] = z[q - 1];
            }
#pragma unroll
        for (int q = 0; q < 9; ++q)
            if (q == pos) {
                c0[q] = x.x;
                c1[q] = x.y;
                c2[q] = x.z;
                T[q] = 1.f - x.w;
                z[q] = xz;
            }
        ++cnt;
        if (cnt > k) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q == cnt - 2) {
                    c0[q] += T[q] * c0[q + 1];
                    c1[q] += T[q] * c1[q + 1];
                    c2[q] += T[q] * c2[q + 1];
                    T[q] *= T[q + 1];
                }
            --cnt;
        }
    }
    // blend the nodes front to back over the background
    __device__ __forceinline__ float4 finish(const ShadeParams &sp) const {
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, Tr = 1.f;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < cnt) {
                C0 += Tr * c0[q];
                C1 += Tr * c1[q];
                C2 += Tr * c2[q];
                Tr *= T[q];
            }
        return make_float4(C0 + Tr * sp.bg[0], C1 + Tr * sp.bg[1], C2 + Tr * sp.bg[2], 1.f - Tr);
    }
};

__global__ void __launch_bounds__(256) k_mlab_blend(const uint32_t *__restrict__ list, uint32_t npix, uint32_t nmax,
                                                    int k, ResolveArgs a, const float4 *__restrict__ mc,
                                                    const uint32_t *__restrict__ mz) {
    const uint32_t i = (uint32_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const uint32_t p = list[i];
    uint32_t n = min(a.count[p], nmax);
    const uint64_t first = a.off[p] - rec_base(a);
    if (first + n > a.rec_cap) n = 0;  // (as the shade pass: nothing was stored)
    MlabNodes nd;
    for (uint32_t e = 0; e < n; ++e) nd.insert(mc[first + e], mz[first + e], k);
    const PixelRef pr = pixel_ref(a.tl, p);
    reinterpret_cast<float4 *>(a.rgba)[(pr.view * a.tl.H + pr.y) * (int64_t)a.tl.W + pr.x] =
        nd.finish(view_params(a.views, pr.view).sp);
}

// Short lists (at most TS fragments): one lane per pixel sorts its list by
// triangle id in LDS, then shades and inserts the fragments in that order.
template <int TS>
__global__ void __launch_bounds__(64) k_mlab_short(const uint32_t *__restrict__ list, uint32_t npix, int k,
                                                   ResolveArgs a) {
    __shared__ uint64_t col[TS][64];
    const int lane = threadIdx.x;
    const uint32_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 64 + lane;
    if (idx >= npix) return;
    const uint32_t p = list[idx];
    uint32_t n = min(a.count[p], (uint32_t)TS);
    const uint64_t first = a.off[p] - rec_base(a);
    if (first + n > a.rec_cap) n = 0;
    const uint64_t *src = a.rec + first;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t r = (src[i] << 32) | (src[i] >> 32);  // triangle id first: primitive order
        int j = (int)i;
        while (j > 0 && col[j - 1][lane] > r) {
            col[j][lane] = col[j - 1][lane];
            --j;
        }
        col[j][lane] = r;
    }
    const PixelRef pr = pixel_ref(a.tl, p);
    const ShadeParams &sp = view_params(a.views, pr.view).sp;
    const VertRec *vert = a.mesh.vert + pr.view * a.mesh.V;
    MlabNodes nd;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t r = col[i][lane];
        const Frag fr = shade(a.mesh, vert, sp, (uint32_t)(r >> 32), pr.x, pr.y);
        nd.insert(make_float4(fr.r, fr.g, fr.b, fr.a), (uint32_t)(r & 0xffffffffu), k);
    }
    reinterpret_cast<float4 *>(a.rgba)[(pr.view * a.tl.H + pr.y) * (int64_t)a.tl.W + pr.x] = nd.finish(sp);
}

// Moment-based transparency: wave per pixel, no sort.
template <int R>
__global__ void __launch_bounds__(256) k_resolve_moments(const uint32_t *__restrict__ list, uint32_t npix,
                                                         ResolveArgs a) {
    const int lane = threadIdx.x & 63;
    const uint32_t wave = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (wave >= npix) return;
    const uint32_t p = list[wave];
    uint64_t v[R];
    const uint32_t n = load_list<R>(a, p, lane, v);
    const PixelRef pr = pixel_ref(a.tl, p);
    const ViewParams &vp = view_params(a.views, pr.view);
    const ShadeParams &sp = vp.sp;
    const VertRec *vert = a.mesh.vert + pr.view * a.mesh.V;
    const double zs = 1.0 / ((double)vp.w1 - (double)vp.w0);
    float fc0[R], fc1[R], fc2[R], fa[R];
    double xw[R], b[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = lane * R + r;
        fc0[r] = fc1[r] = fc2[r] = fa[r] = 0.f;
        const double w = 1048576.0 / (double)(KMAX - (uint32_t)(v[r] >> 32));
        xw[r] = 2.0 * fmin(fmax((w - (double)vp.w0) * zs, 0.0), 1.0) - 1.0;
        if (e < n) {
            const Frag fr = shade(a.mesh, vert, sp, (uint32_t)(v[r] & 0xffffffffu), pr.x, pr.y);
            fc0[r] = fr.r;
            fc1[r] = fr.g;
            fc2[r] = fr.b;
            fa[r] = fr.a;
            const double ab = -log1p(-fmin((double)fr.a, 1.0 - 1e-6));
            double xp = 1.0;
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                b[j] += ab * xp;
                xp *= xw[r];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) b[j] = wave_sum_d(b[j]);
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
    if (b[0] > 0.0) {
        const double ref[5] = {1.0, 0.0, 0.375, 0.0, 0.375};
        double m[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) m[j] = (1.0 - MOM_BETA) * (b[j] / b[0]) + MOM_BETA * ref[j];
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, W = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (lane * R + r < n) {
                const double T = exp(-b[0] * moment_fraction(m, xw[r]));
                c0 += T * fc0[r];
                c1 += T * fc1[r];
                c2 += T * fc2[r];
                W += T * fa[r];
            }
        c0 = wave_sum_d(c0);
        c1 = wave_sum_d(c1);
        c2 = wave_sum_d(c2);
        W = wave_sum_d(W);
        const double At = -expm1(-b[0]);
        const double sc = W > 0.0 ? At / W : 0.0;
        C0 = (float)(c0 * sc);
        C1 = (float)(c1 * sc);
        C2 = (float)(c2 * sc);
        A = (float)At;
    }
    if (lane == 0) {
        const float T = 1.f - A;
        reinterpret_cast<float4 *>(a.rgba)[(pr.view * a.tl.H + pr.y) * (int64_t)a.tl.W + pr.x] =
            make_float4(C0 + T * sp.bg[0], C1 + T * sp.bg[1], C2 + T * sp.bg[2], A);
    }
}

// Short lists (at most TS fragments; mostly empty pixels): one lane per
// pixel, the fragments shaded twice (moments, then the bound per fragment)
// instead of being held.
template <int TS>
__global__ void __launch_bounds__(256) k_moments_short(const uint32_t *__restrict__ list, uint32_t npix,
                                                       ResolveArgs a) {
    const uint32_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (idx >= npix) return;
    const uint32_t p = list[idx];
    uint32_t n = min(a.count[p], (uint32_t)TS);
    const uint64_t first = a.off[p] - rec_base(a);
    if (first + n > a.rec_cap) n = 0;
    const uint64_t *src = a.rec + first;
    const PixelRef pr = pixel_ref(a.tl, p);
    const ViewParams &vp = view_params(a.views, pr.view);
    const ShadeParams &sp = vp.sp;
    const VertRec *vert = a.mesh.vert + pr.view * a.mesh.V;
    const double zs = 1.0 / ((double)vp.w1 - (double)vp.w0);
    auto warp = [&](uint64_t r) {
        const double w = 1048576.0 / (double)(KMAX - (uint32_t)(r >> 32));
        return 2.0 * fmin(fmax((w - (double)vp.w0) * zs, 0.0), 1.0) - 1.0;
    };
    double b[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t r = src[i];
        const Frag fr = shade(a.mesh, vert, sp, (uint32_t)(r & 0xffffffffu), pr.x, pr.y);
        const double ab = -log1p(-fmin((double)fr.a, 1.0 - 1e-6)), xw = warp(r);
        double xp = 1.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            b[j] += ab * xp;
            xp *= xw;
        }
    }
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
    if (b[0] > 0.0) {
        const double ref[5] = {1.0, 0.0, 0.375, 0.0, 0.375};
        double m[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) m[j] = (1.0 - MOM_BETA) * (b[j] / b[0]) + MOM_BETA * ref[j];
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, W = 0.0;
        for (uint32_t i = 0; i < n; ++i) {
            const uint64_t r = src[i];
            const Frag fr = shade(a.mesh, vert, sp, (uint32_t)(r & 0xffffffffu), pr.x, pr.y);
            const double T = exp(-b[0] * moment_fraction(m, warp(r)));
            c0 += T * fr.r;
            c1 += T * fr.g;
            c2 += T * fr.b;
            W += T * fr.a;
        }
        const double At = -expm1(-b[0]);
        const double sc = W > 0.0 ? At / W : 0.0;
        C0 = (float)(c0 * sc);
        C1 = (float)(c1 * sc);
        C2 = (float)(c2 * sc);
        A = (float)At;
    }
    const float T = 1.f - A;
    reinterpret_cast<float4 *>(a.rgba)[(pr.view * a.tl.H + pr.y) * (int64_t)a.tl.W + pr.x] =
        make_float4(C0 + T * sp.bg[0], C1 + T * sp.bg[1], C2 + T * sp.bg[2], A);
}

void launch_resolve_approx(int cls, const uint32_t *pix_list, uint32_t npix, int method, int k, int t_sort,
                           const ResolveArgs &a, float4 *mc, uint32_t *mz, hipStream_t s) {
    if (npix == 0) return;
#define APPROX(RV)                                                                                              \
    if (method == 1) {                                                                                          \
        k_mlab_shade<RV><<<dim3((npix + 3) / 4), 256, 0, s>>>(pix_list, npix, a, mc, mz);                      \
        k_mlab_blend<<<dim3((npix + 255) / 256), 256, 0, s>>>(pix_list, npix, 64u * (RV), k, a, mc, mz);     \
    } else {                                                                                                    \
        k_resolve_moments<RV><<<dim3((npix + 3) / 4), 256, 0, s>>>(pix_list, npix, a);                          \
    }
    if (cls == 0 && method == 1) {  // short lists: a lane per pixel
        const dim3 g((npix + 63) / 64);
        if (t_sort <= 16) k_mlab_short<16><<<g, 64, 0, s>>>(pix_list, npix, k, a);
        else if (t_sort <= 32) k_mlab_short<32><<<g, 64, 0, s>>>(pix_list, npix, k, a);
        else k_mlab_short<64><<<g, 64, 0, s>>>(pix_list, npix, k, a);
        return;
    }
    if (cls == 0) {
        const dim3 g((npix + 255) / 256);
        if (t_sort <= 16) k_moments_short<16><<<g, 256, 0, s>>>(pix_list, npix, a);
        else if (t_sort <= 32) k_moments_short<32><<<g, 256, 0, s>>>(pix_list, npix, a);
        else k_moments_short<64><<<g, 256, 0, s>>>(pix_list, npix, a);
        return;
    }
    switch (cls) {
        case 0:
        case 1: APPROX(1); break;
        case 2: APPROX(2); break;
        case 3: APPROX(4); break;
        case 4: APPROX(8); break;
        case 5: APPROX(16); break;
        case 6: APPROX(32); break;
        default: break;
    }
#undef APPROX
}

void launch_tail_features(int cls, const uint32_t *pix_list, uint32_t npix, uint32_t *queue, int K,
                          const ResolveArgs &a, float *head, float *feat, float *target, uint32_t *pix_out,
                          bool rowmajor, int64_t out_base, float conf_min, uint8_t *mask, hipStream_t s) {
    if (npix == 0) return;
    // learned resolve (an output image), training rows (a target) or feature rows
    const int mode = a.rgba ? TAIL_RESOLVE : target ? TAIL_TRAIN : TAIL_FEATURES;
    int dev = 0;
    (void)hipGetDevice(&dev);
    // a resident grid (the device's workgroups of the kernel, once per kernel), at most a wave per row
    auto grid = [&](int resident_blocks) { return dim3((unsigned)std::min<uint64_t>(resident_blocks, (npix + 3) / 4)); };
#define TAIL_LAUNCH(RV, MV)                                                                                    \
    {                                                                                                          \
        static const int res = resident(dev, k_tail_features<RV, MV>, 256);                                    \
        k_tail_features<RV, MV><<<grid(res), 256, 0, s>>>(pix_list, npix, queue, K, conf_min, a, head, feat, \
                                                           target, pix_out, mask, rowmajor, out_base);         \
    }
#define TAIL(RV)                                                        \
    switch (mode) {                                                     \
        case TAIL_RESOLVE: TAIL_LAUNCH(RV, TAIL_RESOLVE) break;         \
        case TAIL_TRAIN: TAIL_LAUNCH(RV, TAIL_TRAIN) break;             \
        default: TAIL_LAUNCH(RV, TAIL_FEATURES)                         \
    }
    switch (cls) {
        case 1: TAIL(1); break;
        case 2: TAIL(2); break;
        case 3: TAIL(4); break;
        case 4: TAIL(8); break;
        case 5: TAIL(16); break;
        case 6: TAIL(32); break;
        default: break;
    }
#undef TAIL
#undef TAIL_LAUNCH
}

}  // namespace hexfc
