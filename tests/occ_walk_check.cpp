// Runs the library's shadow-ray walk (occ_trace.h, compiled for the host) on
// segments read from stdin, over a grid laid out as occ.hip lays it out (box
// lists as there; the empty-cube radii from their definition, not from the
// device's separable passes), so the CPU suite can compare it with the
// oracle's brute-force visibility.
// stdin:  K res n, then K lines of 6 floats (box min, max), then n lines of
//         6 floats (x, y); floats are given as hex bit patterns.
// stdout: n characters, '1' = visible, '0' = blocked.
#include <cstdio>
#include <cstring>
#include <vector>

#include "occ_trace.h"

static float rd() {
    unsigned u;
    if (std::scanf("%x", &u) != 1) return 0.0f;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

int main() {
    unsigned K, res, n;
    if (std::scanf("%u %u %u", &K, &res, &n) != 3) return 1;
    std::vector<float4> box(2 * (size_t)K);
    float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
    for (unsigned i = 0; i < K; ++i) {
        float a[6];
        for (float& v : a) v = rd();
        box[2 * i] = make_float4(a[0], a[1], a[2], a[3]);
        box[2 * i + 1] = make_float4(a[4], a[5], 0.0f, 0.0f);
        for (int k = 0; k < 3; ++k) {
            lo[k] = a[k] < lo[k] ? a[k] : lo[k];
            hi[k] = a[3 + k] > hi[k] ? a[3 + k] : hi[k];
        }
    }
    rlc::DevOcc occ{};
    occ.box = box.data();
    occ.K = K;
    std::vector<uint32_t> head, ref;
    if (res) {
        // same layout as the device build: header per cell, lists for cells
        // with two or more boxes
        rlc::occ_grid_bounds(occ, lo, hi, res);
        size_t nc = (size_t)res * res * res;
        std::vector<uint32_t> cnt(nc, 0), start(nc + 1, 0), cur(nc, 0);
        for (unsigned i = 0; i < K; ++i) {
            int l[3], h[3];
            rlc::box_cells(occ, box[2 * i], box[2 * i + 1], l, h);
            for (int z = l[2]; z <= h[2]; ++z)
                for (int y = l[1]; y <= h[1]; ++y)
                    for (int x = l[0]; x <= h[0]; ++x) cnt[x + res * (y + res * (size_t)z)]++;
        }
        uint32_t run = 0;
        for (size_t c = 0; c < nc; ++c) {
            start[c] = run;
            run += cnt[c] >= 2 ? cnt[c] + 1 : 0;
        }
        head.assign(nc, 0);
        ref.assign(run ? run : 1, 0);
        for (size_t c = 0; c < nc; ++c)
            if (cnt[c] >= 2) {
                head[c] = RLC_OCC_LIST | start[c];
                ref[start[c]] = cnt[c];
            }
        for (unsigned i = 0; i < K; ++i) {
            int l[3], h[3];
            rlc::box_cells(occ, box[2 * i], box[2 * i + 1], l, h);
            for (int z = l[2]; z <= h[2]; ++z)
                for (int y = l[1]; y <= h[1]; ++y)
                    for (int x = l[0]; x <= h[0]; ++x) {
                        size_t c = x + res * (y + res * (size_t)z);
                        if (cnt[c] == 1)
                            head[c] = RLC_OCC_ONE | i;
                        else
                            ref[start[c] + 1 + cur[c]++] = i;
                    }
        }
        // octant radii of every empty cell, from their definition: for each
        // octant, the largest r <= RLC_OCC_SKIP_MAX for which the cube of
        // cells c + (i s_x, j s_y, k s_z), 0 <= i, j, k <= r (cut by the
        // grid) holds no occupied cell, counted with a 3-D prefix sum of
        // occupancy
        const size_t R1 = (size_t)res + 1;
        std::vector<uint32_t> sat(R1 * R1 * R1, 0);
        auto S = [&](int x, int y, int z) -> uint32_t& { return sat[x + R1 * (y + R1 * (size_t)z)]; };
        for (int z = 0; z < (int)res; ++z)
            for (int y = 0; y < (int)res; ++y)
                for (int x = 0; x < (int)res; ++x)
                    S(x + 1, y + 1, z + 1) = (head[x + res * (y + res * (size_t)z)] != 0) + S(x, y + 1, z + 1) +
                                             S(x + 1, y, z + 1) + S(x + 1, y + 1, z) - S(x, y, z + 1) -
                                             S(x, y + 1, z) - S(x + 1, y, z) + S(x, y, z);
        // cells [a0, a1) along each axis, cut by the grid
        auto clip = [&](int v) { return v < 0 ? 0 : (v > (int)res ? (int)res : v); };
        auto occupied_in = [&](int x0, int x1, int y0, int y1, int z0, int z1) {
            x0 = clip(x0), x1 = clip(x1), y0 = clip(y0), y1 = clip(y1), z0 = clip(z0), z1 = clip(z1);
            return S(x1, y1, z1) - S(x0, y1, z1) - S(x1, y0, z1) - S(x1, y1, z0) + S(x0, y0, z1) + S(x0, y1, z0) +
                   S(x1, y0, z0) - S(x0, y0, z0);
        };
        for (int z = 0; z < (int)res; ++z)
            for (int y = 0; y < (int)res; ++y)
                for (int x = 0; x < (int)res; ++x) {
                    uint32_t& h = head[x + res * (y + res * (size_t)z)];
                    if (h) continue;
                    uint32_t word = 0;
                    for (int o = 0; o < 8; ++o) {
                        const bool nx = o & 1, ny = o & 2, nz = o & 4;
                        uint32_t r = 0;
                        while (r < RLC_OCC_SKIP_MAX) {
                            const int q = (int)r + 1;
                            const int x0 = nx ? x - q : x, x1 = nx ? x + 1 : x + q + 1;
                            const int y0 = ny ? y - q : y, y1 = ny ? y + 1 : y + q + 1;
                            const int z0 = nz ? z - q : z, z1 = nz ? z + 1 : z + q + 1;
                            if (occupied_in(x0, x1, y0, y1, z0, z1)) break;
                            r = (uint32_t)q;
                        }
                        word |= r << (3 * o);
                    }
                    h = word;
                }
        occ.head = head.data();
        occ.ref = ref.data();
    }
    std::vector<char> out(n + 1, 0);
    for (unsigned i = 0; i < n; ++i) {
        float x[3], y[3], d[3];
        for (float& v : x) v = rd();
        for (float& v : y) v = rd();
        for (int a = 0; a < 3; ++a) d[a] = y[a] - x[a];
        out[i] = rlc::segment_blocked(occ, x, d, 1e-4f) ? '0' : '1';
    }
    std::fwrite(out.data(), 1, n, stdout);
    return 0;
}
