// Runs the library's shadow-ray code (the grid build of occ.hip and the walk
// of occ_trace.h, compiled for the host) on segments read from stdin, so the
// CPU suite can compare it with the oracle's brute-force visibility.
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
