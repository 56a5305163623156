// Shadow-ray visibility against axis-aligned boxes: the slab test and the
// uniform-grid walk.  Compiled for the device (frame and occluder kernels)
// and for the host (the CPU check of the grid walk), so everything here is
// __host__ __device__ and free of device intrinsics.
//
// The answer of a shadow ray is defined box by box: the segment x + t d,
// t in (t_lo, 1 - t_lo), is blocked by a box when the slab intervals
// intersect with tn < tf strictly, an axis with d = 0 either excluding the
// box (origin outside the slab) or not constraining it.  The grid only
// decides which boxes a ray tests; it never changes that answer.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace rlc {

// Everything here is inlined into its callers: the small arrays it passes
// around must stay in registers.
#define RLC_WALK_INLINE __host__ __device__ __attribute__((always_inline)) inline

// Box b of the occluder set is stored as two float4: {min.xyz, max.x} and
// {max.yz, 0, 0}.  Grid cell c has a 32-bit header head[c]: RLC_OCC_ONE | b
// when box b is the only one overlapping it; RLC_OCC_LIST | s when several
// do, their count at ref[s] and their indices at ref[s + 1..]; and for a
// cell c no box overlaps, eight 3-bit radii, one per octant of directions
// o = (d_x < 0) | (d_y < 0) << 1 | (d_z < 0) << 2 at bits 3o..3o+2: the
// largest r <= RLC_OCC_SKIP_MAX for which no box overlaps the cells
// c + (i s_x, j s_y, k s_z), 0 <= i, j, k <= r (s_a = -1 where the octant's
// d_a < 0, else +1; cut by the grid's faces), so a walk heading into that
// octant can leave the cube in one step.
#define RLC_OCC_ONE 0x40000000u
#define RLC_OCC_LIST 0x80000000u
#define RLC_OCC_PAYLOAD 0x3FFFFFFFu
#define RLC_OCC_SKIP_MAX 7u
// Largest grid resolution (the walk's offsets are exact in FP32 up to it).
#define RLC_OCC_RES_MAX 256u

struct DevOcc {
    const float4* box;
    const uint32_t* head;       // res^3 cell headers
    const uint32_t* ref;        // box lists of cells holding two or more boxes
    uint32_t K;
    uint32_t res;               // 0: test every box
    float glo[3];               // grid box, slightly larger than the boxes' union
    float gcell[3];             // grid cell size
    float ginv[3];              // res / extent
    float gmax[3];
};

// Grid box and cell size for boxes whose union spans [lo, hi]: the union
// grown by 1/1000 of its largest extent, cut into res^3 cells.
RLC_WALK_INLINE void occ_grid_bounds(DevOcc& o, const float lo[3], const float hi[3], uint32_t res) {
    float ext = fmaxf(hi[0] - lo[0], fmaxf(hi[1] - lo[1], hi[2] - lo[2]));
    float margin = 1e-3f * ext + 1e-6f;
    o.res = res;
    for (int a = 0; a < 3; ++a) {
        o.glo[a] = lo[a] - margin;
        o.gmax[a] = hi[a] + margin;
        o.gcell[a] = (o.gmax[a] - o.glo[a]) / (float)res;
        o.ginv[a] = (float)res / (o.gmax[a] - o.glo[a]);
    }
}

// Box test as defined (any direction, including d_a = 0 and subnormal d_a).
RLC_WALK_INLINE bool box_blocks_def(const float4 b0, const float4 b1, const float o[3],
                                               const float d[3], const float invd[3], float t_lo) {
    const float bmin[3] = {b0.x, b0.y, b0.z};
    const float bmax[3] = {b0.w, b1.x, b1.y};
    float tn = t_lo;
    float tf = 1.0f - t_lo;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) {
            if (o[a] < bmin[a] || o[a] > bmax[a]) return false;
            continue;
        }
        float t0 = (bmin[a] - o[a]) * invd[a];
        float t1 = (bmax[a] - o[a]) * invd[a];
        float tmin = t0 < t1 ? t0 : t1;
        float tmax = t0 < t1 ? t1 : t0;
        if (tmin > tn) tn = tmin;
        if (tmax < tf) tf = tmax;
    }
    return tn < tf;
}

// The same test, branch-free, for rays whose three direction components are
// normal numbers: then 1/d is finite and non-zero, no interval bound is NaN,
// and min/max give the interval ends the definition picks (up to the sign
// of a zero, which no comparison sees).
RLC_WALK_INLINE bool box_blocks_fast(const float4 b0, const float4 b1, const float o[3],
                                                const float invd[3], float tn0, float tf0) {
    float t0x = (b0.x - o[0]) * invd[0], t1x = (b0.w - o[0]) * invd[0];
    float t0y = (b0.y - o[1]) * invd[1], t1y = (b1.x - o[1]) * invd[1];
    float t0z = (b0.z - o[2]) * invd[2], t1z = (b1.y - o[2]) * invd[2];
    float tn = fmaxf(fmaxf(tn0, fminf(t0x, t1x)), fmaxf(fminf(t0y, t1y), fminf(t0z, t1z)));
    float tf = fminf(fminf(tf0, fmaxf(t0x, t1x)), fminf(fmaxf(t0y, t1y), fmaxf(t0z, t1z)));
    return tn < tf;
}

RLC_WALK_INLINE bool normal_dir(const float d[3]) {
    const float tiny = 1.17549435e-38f;  // smallest normal float
    return fabsf(d[0]) >= tiny && fabsf(d[1]) >= tiny && fabsf(d[2]) >= tiny;
}

template <bool FAST>
RLC_WALK_INLINE bool box_blocks(const float4 b0, const float4 b1, const float o[3], const float d[3],
                                const float invd[3], float t_lo) {
    if (FAST) return box_blocks_fast(b0, b1, o, invd, t_lo, 1.0f - t_lo);
    return box_blocks_def(b0, b1, o, d, invd, t_lo);
}

template <bool FAST>
RLC_WALK_INLINE bool test_box(const DevOcc& occ, uint32_t b, const float o[3], const float d[3],
                                         const float invd[3], float t_lo) {
    return box_blocks<FAST>(occ.box[2 * b], occ.box[2 * b + 1], o, d, invd, t_lo);
}

// Grid cells overlapped by a box grown by 1/256 of a cell on every side, so
// that a walk whose cell boundaries are off by rounding still lists it.
RLC_WALK_INLINE void box_cells(const DevOcc& occ, float4 b0, float4 b1, int lo[3], int hi[3]) {
    const float bmin[3] = {b0.x, b0.y, b0.z};
    const float bmax[3] = {b0.w, b1.x, b1.y};
    const int res = (int)occ.res;
    for (int a = 0; a < 3; ++a) {
        float m = occ.gcell[a] * (1.0f / 256.0f);
        float f0 = floorf((bmin[a] - m - occ.glo[a]) * occ.ginv[a]);
        float f1 = floorf((bmax[a] + m - occ.glo[a]) * occ.ginv[a]);
        lo[a] = f0 < 0.0f ? 0 : (f0 >= (float)res ? res - 1 : (int)f0);
        hi[a] = f1 < 0.0f ? 0 : (f1 >= (float)res ? res - 1 : (int)f1);
    }
}

template <bool FAST>
RLC_WALK_INLINE bool blocked_brute(const DevOcc& occ, const float o[3], const float d[3],
                                              const float invd[3], float t_lo) {
    for (uint32_t b = 0; b < occ.K; ++b)
        if (test_box<FAST>(occ, b, o, d, invd, t_lo)) return true;
    return false;
}

// Test the boxes listed in one occupied grid cell (header h, at least
// RLC_OCC_ONE).  Two mailbox slots skip a box that was just tested in a
// previous cell.
template <bool FAST>
RLC_WALK_INLINE bool cell_blocks(const DevOcc& occ, uint32_t h, uint32_t& last0, uint32_t& last1,
                                            const float o[3], const float d[3], const float invd[3], float t_lo) {
    if (!(h & RLC_OCC_LIST)) {
        const uint32_t b = h & RLC_OCC_PAYLOAD;
        if (b == last0 || b == last1) return false;
        last1 = last0;
        last0 = b;
        return test_box<FAST>(occ, b, o, d, invd, t_lo);
    }
    // a list holds two boxes or more: its count and first two entries are
    // loaded together, and the first box's bounds with them
    const uint32_t s0 = h & RLC_OCC_PAYLOAD;
    const uint32_t n = occ.ref[s0];
    const uint32_t ba = occ.ref[s0 + 1], bb = occ.ref[s0 + 2];
    const float4 a0 = occ.box[2 * ba], a1 = occ.box[2 * ba + 1];
    if (ba != last0 && ba != last1) {
        last1 = last0;
        last0 = ba;
        if (box_blocks<FAST>(a0, a1, o, d, invd, t_lo)) return true;
    }
    if (bb != last0 && bb != last1) {
        last1 = last0;
        last0 = bb;
        if (test_box<FAST>(occ, bb, o, d, invd, t_lo)) return true;
    }
    for (uint32_t j = 3; j <= n; ++j) {
        const uint32_t b = occ.ref[s0 + j];
        if (b == last0 || b == last1) continue;
        last1 = last0;
        last0 = b;
        if (test_box<FAST>(occ, b, o, d, invd, t_lo)) return true;
    }
    return false;
}

// Walk the grid cells the segment crosses, in order (3-D DDA,
// Amanatides-Woo).  The parameter of the next boundary along each axis grows
// by the cell size over |d| per boundary; boxes are listed in cells grown by
// 1/256 of a cell, which covers the accumulated rounding of that sum (at
// most 3 res steps of half an ulp of t).  Each axis counts the cells left
// before the walk leaves the grid.
//
// In an empty cell whose radius for the segment's octant is r, the walk
// leaves the whole empty cube ahead of it at once: it exits through the
// cube's nearest far face (the r-th boundary ahead on the axis that reaches
// it first) and, on the other axes, crosses the boundaries whose parameter
// the exit point has passed, at most r.  No box overlaps the
// cells it skips, so the boxes tested, and the answer, are those of the
// cell-by-cell walk; a boundary miscounted by rounding moves the walk to a
// cell that the segment passes within an ulp or so of, which the 1/256 cell
// growth covers.  With r = 0 the step is the plain DDA step.  Every step
// takes at least one cell off the exit axis's count, so the walk ends.
//
// The walk state lives in a struct: walk_begin sets it up, each walk_step
// tests one cell's boxes and moves on.
struct WalkState {
    float t1;
    float tx, ty, tz, dtx, dty, dtz, itx, ity, itz;
    float rx, ry, rz;            // cells left before the grid's face, per axis (whole numbers)
    // byte offset of the current cell's header as a function of the counts
    // above: lin0 + rx fx + ry fy + rz fz.  Every term and partial sum is a
    // multiple of 4 below 4 res^3 <= 2^26 (res <= RLC_OCC_RES_MAX), so FP32
    // holds them exactly and the fused multiply-adds are exact.
    float lin0, fx, fy, fz;
    uint32_t osh;                // 3 x the segment's octant: shift of its radius in a header
    int it;                      // steps taken (a guard: the counts above already bound them)
    uint32_t last0, last1;
    uint32_t h;                  // header of the current cell, loaded one step ahead
};

// Byte offset of the current cell's header (see WalkState).
RLC_WALK_INLINE uint32_t walk_offset(const WalkState& w) {
    return (uint32_t)fmaf(w.rx, w.fx, fmaf(w.ry, w.fy, fmaf(w.rz, w.fz, w.lin0)));
}

// false: the segment misses the grid (nothing to test).
RLC_WALK_INLINE bool walk_begin(const DevOcc& occ, const float o[3], const float d[3],
                                           const float invd[3], float t_lo, WalkState& w) {
    float t0 = t_lo, t1 = 1.0f - t_lo;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) {
            if (o[a] < occ.glo[a] || o[a] > occ.gmax[a]) return false;
            continue;
        }
        float ta = (occ.glo[a] - o[a]) * invd[a];
        float tb = (occ.gmax[a] - o[a]) * invd[a];
        float lo = ta < tb ? ta : tb;
        float hi = ta < tb ? tb : ta;
        t0 = lo > t0 ? lo : t0;
        t1 = hi < t1 ? hi : t1;
    }
    if (!(t0 <= t1)) return false;
    const int res = (int)occ.res;
    int c[3];
    float tn[3], dt[3];
    int rem[3], st[3];
    for (int a = 0; a < 3; ++a) {
        float p = o[a] + t0 * d[a];
        float f = floorf((p - occ.glo[a]) * occ.ginv[a]);
        c[a] = f < 0.0f ? 0 : (f >= (float)res ? res - 1 : (int)f);
        if (d[a] == 0.0f) {
            tn[a] = 3.0e38f;
            dt[a] = 0.0f;
            rem[a] = 0;
            st[a] = 0;
        } else {
            const bool up = d[a] > 0.0f;
            const float bound = occ.glo[a] + (float)(c[a] + (up ? 1 : 0)) * occ.gcell[a];
            tn[a] = (bound - o[a]) * invd[a];
            dt[a] = occ.gcell[a] * fabsf(invd[a]);
            rem[a] = up ? res - 1 - c[a] : c[a];
            st[a] = up ? 1 : -1;
        }
    }
    w.t1 = t1;
    // cell coordinate c = (res - 1) - rem on an axis walked upwards, rem
    // otherwise (a zero direction leaves rem at 0)
    const int stride[3] = {4, 4 * res, 4 * res * res};
    int lin0 = 0;
    for (int a = 0; a < 3; ++a) lin0 += stride[a] * (c[a] + st[a] * rem[a]);
    w.lin0 = (float)lin0;
    w.fx = (float)(-st[0] * stride[0]);
    w.fy = (float)(-st[1] * stride[1]);
    w.fz = (float)(-st[2] * stride[2]);
    w.tx = tn[0];
    w.ty = tn[1];
    w.tz = tn[2];
    w.dtx = dt[0];
    w.dty = dt[1];
    w.dtz = dt[2];
    w.itx = dt[0] > 0.0f ? 1.0f / dt[0] : 0.0f;
    w.ity = dt[1] > 0.0f ? 1.0f / dt[1] : 0.0f;
    w.itz = dt[2] > 0.0f ? 1.0f / dt[2] : 0.0f;
    w.rx = (float)rem[0];
    w.ry = (float)rem[1];
    w.rz = (float)rem[2];
    w.osh = 3u * ((d[0] < 0.0f ? 1u : 0u) | (d[1] < 0.0f ? 2u : 0u) | (d[2] < 0.0f ? 4u : 0u));
    w.it = 0;
    w.last0 = 0xFFFFFFFFu;
    w.last1 = 0xFFFFFFFFu;
    w.h = *(const uint32_t*)((const char*)occ.head + walk_offset(w));
    return true;
}

// Boundaries of one axis that the exit parameter tm has reached: those at
// t, t + dt, ..., at most ra of them (ra as a float, fra).  With FAST every
// parameter is finite and idt > 0, so a tm short of t gives a count below
// zero, which the clamp removes; otherwise dt may be infinite (idt = 0) and
// tm is compared with t first.
template <bool FAST>
RLC_WALK_INLINE float walk_crossed(float tm, float t, float idt, float fra) {
    if (FAST) {
        const float q = floorf(fmaf(tm - t, idt, 1.0f));
#if defined(__HIP_DEVICE_COMPILE__)
        return __builtin_amdgcn_fmed3f(q, 0.0f, fra);
#else
        return fminf(fmaxf(q, 0.0f), fra);
#endif
    }
    const float q = tm >= t ? floorf((tm - t) * idt) + 1.0f : 0.0f;
    return fminf(fmaxf(q, 0.0f), fra);
}

// t + k dt; with FAST dt is finite, so k = 0 leaves t as it is.
template <bool FAST>
RLC_WALK_INLINE float walk_advance(float t, float fk, float dt) {
    if (FAST) return fmaf(fk, dt, t);
    return fk != 0.0f ? t + fk * dt : t;
}

// min(a, b) of two non-NaN floats: the median of a, b and a value below
// both (one v_med3_f32 on the device)
RLC_WALK_INLINE float walk_min(float a, float b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fmed3f(a, b, -3.0e38f);
#else
    return a < b ? a : b;
#endif
}

// Test the current cell, then move on.  Returns 1 when a box blocks the
// segment, 2 when the walk has ended unblocked, 0 otherwise.  The step out
// of a cell depends on its header alone (an occupied cell is left through
// one boundary), so it is taken first and the next cell's header is loaded
// before the current cell's boxes are tested: the two loads overlap.  The
// header is loaded only when the walk goes on, so it stays in the grid.
// Outside the box tests everything is computed for every lane and
// selected, without branches, so a wave runs it once.
template <bool FAST>
RLC_WALK_INLINE int walk_step(const DevOcc& occ, WalkState& w, const float o[3], const float d[3],
                                         const float invd[3], float t_lo) {
    const uint32_t h = w.h;
    // an empty cell's header holds only its radii, in the low 24 bits
    const bool occupied = h >= RLC_OCC_ONE;
    const float r = occupied ? 0.0f : (float)((h >> w.osh) & RLC_OCC_SKIP_MAX);
    // exit parameter of the empty cube on each axis (cut by the grid); the
    // axis that reaches its face first moves on (ties: x, then y).  Value
    // selects and integer masks, not selects between fields, keep the state
    // in registers.
    const float frx = walk_min(r, w.rx);
    const float fry = walk_min(r, w.ry);
    const float frz = walk_min(r, w.rz);
    const float ex = walk_advance<FAST>(w.tx, frx, w.dtx);
    const float ey = walk_advance<FAST>(w.ty, fry, w.dty);
    const float ez = walk_advance<FAST>(w.tz, frz, w.dtz);
    const bool ax = ex <= ey && ex <= ez;
    const bool ay = !ax && ey <= ez;
    const float tm = fminf(ex, fminf(ey, ez));
    const float rm = ax ? w.rx : (ay ? w.ry : w.rz);
    const float cx = walk_crossed<FAST>(tm, w.tx, w.itx, frx);
    const float cy = walk_crossed<FAST>(tm, w.ty, w.ity, fry);
    const float cz = walk_crossed<FAST>(tm, w.tz, w.itz, frz);
    const float fr1 = r + 1.0f;
    const float fkx = ax ? fr1 : cx;
    const float fky = ay ? fr1 : cy;
    const float fkz = (ax || ay) ? cz : fr1;
    ++w.it;
    const bool ends = (tm > w.t1) | (rm <= r) | (w.it >= 3 * (int)occ.res + 3);
    if (!ends) {
        w.tx = walk_advance<FAST>(w.tx, fkx, w.dtx);
        w.ty = walk_advance<FAST>(w.ty, fky, w.dty);
        w.tz = walk_advance<FAST>(w.tz, fkz, w.dtz);
        w.rx -= fkx;
        w.ry -= fky;
        w.rz -= fkz;
        w.h = *(const uint32_t*)((const char*)occ.head + walk_offset(w));
    }
    if (occupied && cell_blocks<FAST>(occ, h, w.last0, w.last1, o, d, invd, t_lo)) return 1;
    return ends ? 2 : 0;
}

template <bool FAST>
RLC_WALK_INLINE bool blocked_grid(const DevOcc& occ, const float o[3], const float d[3],
                                             const float invd[3], float t_lo) {
    WalkState w;
    if (!walk_begin(occ, o, d, invd, t_lo, w)) return false;
    for (;;) {
        const int r = walk_step<FAST>(occ, w, o, d, invd, t_lo);
        if (r) return r == 1;
    }
}

// Is the segment o -> o + d blocked over t in (t_lo, 1 - t_lo)?
RLC_WALK_INLINE bool segment_blocked(const DevOcc& occ, const float o[3], const float d[3], float t_lo) {
    if (occ.K == 0) return false;
    const float invd[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
    if (normal_dir(d))
        return occ.res ? blocked_grid<true>(occ, o, d, invd, t_lo) : blocked_brute<true>(occ, o, d, invd, t_lo);
    return occ.res ? blocked_grid<false>(occ, o, d, invd, t_lo) : blocked_brute<false>(occ, o, d, invd, t_lo);
}

}  // namespace rlc
