// Vertex-face contact generation for boxes in a bin, shared by the
// stand-alone generation kernel and the fused step: every vertex of every
// box against the floor (z = 0), the four walls (|x| = wx, |y| = wy) and every
// other box of the world.  A contact (Sec. 3: point, normal from body b to
// body a, signed gap, friction) is kept when its gap is below the margin; of
// those, the deepest ones up to the world's contact capacity, ties broken by
// key = (target * 64 + box) * 8 + vertex with targets 0-4 the floor and the
// walls -x, +x, -y, +y and 5 + k the k-th box.  One workgroup per world,
// candidates in LDS, bitonic sort of (orderable gap << 32 | key).
#pragma once

#include "kamx_internal.h"

namespace kamx {

constexpr int kBoxCandidates = 4096;  // 20 boxes x 8 vertices x 24 targets fit
constexpr int kBoxPlanes = 5;         // floor, wall -x, wall +x, wall -y, wall +y

struct BoxLds {
    float c[3 * kMaxBodies];   // centres
    float R[9 * kMaxBodies];   // rotations (row-major, body to world)
    float h[3 * kMaxBodies];   // half extents
    float mu[kMaxBodies];
    int box[kMaxBodies];       // local body index of the k-th box
    unsigned long long cand[kBoxCandidates];  // (orderable gap << 32) | key
    int n_box, n_cand;
};

__host__ __device__ inline int box_bin_max_boxes_of() {
    int n = 1;
    while ((n + 1) * 8 * (kBoxPlanes + n) <= kBoxCandidates) ++n;
    return n;
}

__device__ inline uint32_t box_orderable(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline float box_from_orderable(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// vertex v (bits x, y, z: sign +) of box k in world coordinates
__device__ inline void box_vertex(const BoxLds &S, int k, int v, float out[3]) {
    float l[3];
    for (int e = 0; e < 3; ++e) l[e] = ((v >> e) & 1 ? 1.f : -1.f) * S.h[3 * k + e];
    for (int e = 0; e < 3; ++e)
        out[e] = S.c[3 * k + e] + S.R[9 * k + 3 * e] * l[0] + S.R[9 * k + 3 * e + 1] * l[1] + S.R[9 * k + 3 * e + 2] * l[2];
}

// Gap and normal of point p against target t (planes 0-4, box t - 5);
// false when the point is not over a face of a box target.
__device__ inline bool box_test_point(const BoxLds &S, float wx, float wy, int t, const float p[3], float &gap,
                                      float n[3]) {
    if (t < kBoxPlanes) {
        n[0] = n[1] = n[2] = 0.f;
        switch (t) {
        case 0: gap = p[2]; n[2] = 1.f; break;
        case 1: gap = p[0] + wx; n[0] = 1.f; break;
        case 2: gap = wx - p[0]; n[0] = -1.f; break;
        case 3: gap = p[1] + wy; n[1] = 1.f; break;
        default: gap = wy - p[1]; n[1] = -1.f; break;
        }
        return true;
    }
    const int k = t - kBoxPlanes;
    float d[3], q[3];
    for (int e = 0; e < 3; ++e) d[e] = p[e] - S.c[3 * k + e];
    for (int e = 0; e < 3; ++e) q[e] = S.R[9 * k + e] * d[0] + S.R[9 * k + 3 + e] * d[1] + S.R[9 * k + 6 + e] * d[2];
    float dist[3];
    for (int e = 0; e < 3; ++e) dist[e] = fabsf(q[e]) - S.h[3 * k + e];
    int f = 0;
    if (dist[1] > dist[f]) f = 1;
    if (dist[2] > dist[f]) f = 2;
    // the point must lie within the lateral extent of face f
    for (int e = 0; e < 3; ++e)
        if (e != f && dist[e] > 0.f) return false;
    gap = dist[f];
    const float s = q[f] >= 0.f ? 1.f : -1.f;
    for (int e = 0; e < 3; ++e) n[e] = s * S.R[9 * k + 3 * e + f];
    return true;
}

// Contacts of one world.  Called by every thread of the workgroup (NT
// threads; it synchronizes).  pose(b, c[3], quat[4]) gives the centre and
// orientation (x, y, z, w) of local body b; geom points at the world's
// per-body box records (half extents, friction; half extents 0: not a box).
// emit(c, key, gap, point, normal, mu, local body a, local body b or -1) is
// called once for each kept contact c < n, by some thread; returns n.
template <int NT, class Pose, class Emit>
__device__ inline int box_bin_generate(BoxLds &S, int nb, const float *geom, float wx, float wy, float margin, int cap,
                                       Pose &&pose, Emit &&emit) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        int nbx = 0;
        for (int b = 0; b < nb; ++b)
            if (geom[4 * b] > 0.f) S.box[nbx++] = b;
        S.n_box = nbx;
        S.n_cand = 0;
    }
    __syncthreads();
    const int nbx = S.n_box;
    for (int k = tid; k < nbx; k += NT) {
        const int b = S.box[k];
        float cc[3], qq[4];
        pose(b, cc, qq);
        const float x = qq[0], y = qq[1], z = qq[2], s = qq[3];
        float *R = S.R + 9 * k;
        R[0] = 1.f - 2.f * (y * y + z * z);
        R[1] = 2.f * (x * y - z * s);
        R[2] = 2.f * (x * z + y * s);
        R[3] = 2.f * (x * y + z * s);
        R[4] = 1.f - 2.f * (x * x + z * z);
        R[5] = 2.f * (y * z - x * s);
        R[6] = 2.f * (x * z - y * s);
        R[7] = 2.f * (y * z + x * s);
        R[8] = 1.f - 2.f * (x * x + y * y);
        for (int e = 0; e < 3; ++e) {
            S.c[3 * k + e] = cc[e];
            S.h[3 * k + e] = geom[4 * b + e];
        }
        S.mu[k] = geom[4 * b + 3];
    }
    __syncthreads();
    // candidates: box k vertex v against target t (planes, then other boxes)
    const int nt = kBoxPlanes + nbx;
    const int tasks = nbx * 8 * nt;
    for (int i = tid; i < tasks; i += NT) {
        const int k = i / (8 * nt), r = i - k * 8 * nt, v = r / nt, t = r - (r / nt) * nt;
        if (t >= kBoxPlanes && t - kBoxPlanes == k) continue;
        float p[3], n[3], gap;
        box_vertex(S, k, v, p);
        if (!box_test_point(S, wx, wy, t, p, gap, n) || !(gap < margin)) continue;
        const int key = (t * kMaxBodies + k) * 8 + v;
        const int slot = atomicAdd(&S.n_cand, 1);
        if (slot < kBoxCandidates) S.cand[slot] = ((unsigned long long)box_orderable(gap) << 32) | (uint32_t)key;
    }
    __syncthreads();
    const int nc = S.n_cand < kBoxCandidates ? S.n_cand : kBoxCandidates;
    // bitonic sort of the candidates, padded with +inf to a power of two
    int np2 = 1;
    while (np2 < nc) np2 <<= 1;
    for (int i = nc + tid; i < np2; i += NT) S.cand[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= np2; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < np2; i += NT) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    unsigned long long x = S.cand[i], y = S.cand[j];
                    if ((x > y) == up) {
                        S.cand[i] = y;
                        S.cand[j] = x;
                    }
                }
            }
            __syncthreads();
        }
    const int keep = nc < cap ? nc : cap;
    for (int c = tid; c < keep; c += NT) {
        const unsigned long long e = S.cand[c];
        const int key = (int)(uint32_t)(e & 0xffffffffu);
        const int v = key & 7, k = (key >> 3) % kMaxBodies, t = (key >> 3) / kMaxBodies;
        float p[3], n[3], gap;
        box_vertex(S, k, v, p);
        box_test_point(S, wx, wy, t, p, gap, n);
        const float mu = t < kBoxPlanes ? S.mu[k] : fminf(S.mu[k], S.mu[t - kBoxPlanes]);
        emit(c, key, box_from_orderable((uint32_t)(e >> 32)), p, n, mu, S.box[k],
             t < kBoxPlanes ? -1 : S.box[t - kBoxPlanes]);
    }
    return keep;
}

}  // namespace kamx
