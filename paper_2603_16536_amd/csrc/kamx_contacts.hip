// Contact generation for boxes in a bin: vertex-face tests of every box
// vertex against the floor (z = 0), the four walls (|x| = wx, |y| = wy) and
// every other box of the world.  A contact (Sec. 3: point, normal from body
// b to body a, signed gap, friction) is kept when its gap is below the
// margin; of those, the deepest ones up to the world's contact capacity,
// ties broken by key.  One workgroup per world, candidates in LDS.
#include "kamx_internal.h"

namespace kamx {

namespace {

constexpr int kNarrowThreads = 256;
constexpr int kMaxCandidates = 4096;  // 20 boxes x 8 vertices x 24 targets fit
constexpr int kPlanes = 5;            // floor, wall -x, wall +x, wall -y, wall +y

struct BoxLds {
    float c[3 * kMaxBodies];   // centres
    float R[9 * kMaxBodies];   // rotations (row-major, body to world)
    float h[3 * kMaxBodies];   // half extents (0: not a box)
    float mu[kMaxBodies];
    int box[kMaxBodies];       // local body index of the k-th box
    unsigned long long cand[kMaxCandidates];  // (orderable gap << 32) | key
    int n_box, n_cand;
};

__device__ inline uint32_t orderable(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline float from_orderable(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// vertex v (bits x, y, z: sign +) of box k in world coordinates
__device__ inline void vertex(const BoxLds &S, int k, int v, float out[3]) {
    float l[3];
    for (int e = 0; e < 3; ++e) l[e] = ((v >> e) & 1 ? 1.f : -1.f) * S.h[3 * k + e];
    for (int e = 0; e < 3; ++e)
        out[e] = S.c[3 * k + e] + S.R[9 * k + 3 * e] * l[0] + S.R[9 * k + 3 * e + 1] * l[1] + S.R[9 * k + 3 * e + 2] * l[2];
}

// Gap and normal of point p against target t (planes 0-4, box t - 5);
// returns false when the point is not over a face of a box target.
__device__ inline bool test_point(const BoxLds &S, float wx, float wy, int t, const float p[3], float &gap,
                                  float n[3]) {
    if (t < kPlanes) {
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
    const int k = t - kPlanes;
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

__global__ __launch_bounds__(kNarrowThreads) void box_bin_kernel(const WorldInfo *worlds, const float *q,
                                                                 const float *box_geom, float wx, float wy,
                                                                 float margin, kamx_contact *out, int32_t *count) {
    __shared__ BoxLds S;
    const int w = blockIdx.x, tid = threadIdx.x;
    const WorldInfo W = worlds[w];
    if (tid == 0) {
        int nbx = 0;
        for (int b = 0; b < W.nb; ++b)
            if (box_geom[4 * (W.b0 + b)] > 0.f) S.box[nbx++] = b;
        S.n_box = nbx;
        S.n_cand = 0;
    }
    __syncthreads();
    const int nbx = S.n_box;
    for (int k = tid; k < nbx; k += kNarrowThreads) {
        const int gb = W.b0 + S.box[k];
        const float *qq = q + 7 * gb;
        const float x = qq[3], y = qq[4], z = qq[5], s = qq[6];
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
            S.c[3 * k + e] = qq[e];
            S.h[3 * k + e] = box_geom[4 * gb + e];
        }
        S.mu[k] = box_geom[4 * gb + 3];
    }
    __syncthreads();
    // candidates: box k vertex v against target t (planes, then other boxes)
    const int nt = kPlanes + nbx;
    const int tasks = nbx * 8 * nt;
    for (int i = tid; i < tasks; i += kNarrowThreads) {
        const int k = i / (8 * nt), r = i - k * 8 * nt, v = r / nt, t = r - (r / nt) * nt;
        if (t >= kPlanes && t - kPlanes == k) continue;
        float p[3], n[3], gap;
        vertex(S, k, v, p);
        if (!test_point(S, wx, wy, t, p, gap, n) || !(gap < margin)) continue;
        const int key = (t * kMaxBodies + k) * 8 + v;
        const int slot = atomicAdd(&S.n_cand, 1);
        if (slot < kMaxCandidates) S.cand[slot] = ((unsigned long long)orderable(gap) << 32) | (uint32_t)key;
    }
    __syncthreads();
    int nc = S.n_cand < kMaxCandidates ? S.n_cand : kMaxCandidates;
    // bitonic sort of the candidates, padded with +inf to a power of two
    int np2 = 1;
    while (np2 < nc) np2 <<= 1;
    for (int i = nc + tid; i < np2; i += kNarrowThreads) S.cand[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= np2; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < np2; i += kNarrowThreads) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    unsigned long long a = S.cand[i], b = S.cand[j];
                    if ((a > b) == up) {
                        S.cand[i] = b;
                        S.cand[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    const int keep = nc < W.contact_cap ? nc : W.contact_cap;
    for (int c = tid; c < keep; c += kNarrowThreads) {
        const unsigned long long e = S.cand[c];
        const int key = (int)(uint32_t)(e & 0xffffffffu);
        const int v = key & 7, k = (key >> 3) % kMaxBodies, t = (key >> 3) / kMaxBodies;
        float p[3], n[3], gap;
        vertex(S, k, v, p);
        test_point(S, wx, wy, t, p, gap, n);
        kamx_contact ct;
        ct.body_a = W.b0 + S.box[k];
        ct.body_b = t < kPlanes ? -1 : W.b0 + S.box[t - kPlanes];
        for (int d = 0; d < 3; ++d) {
            ct.point[d] = p[d];
            ct.normal[d] = n[d];
        }
        ct.gap = from_orderable((uint32_t)(e >> 32));
        ct.mu = t < kPlanes ? S.mu[k] : fminf(S.mu[k], S.mu[t - kPlanes]);
        ct.key = key;
        out[(long)w * kMaxContacts + c] = ct;
    }
    if (tid == 0) count[w] = keep;
}

}  // namespace

hipError_t launch_box_bin(const WorldInfo *worlds, int n_worlds, const float *q, const float *box_geom, float wx,
                          float wy, float margin, kamx_contact *out, int32_t *count, hipStream_t stream) {
    if (n_worlds <= 0) return hipSuccess;
    hipLaunchKernelGGL(box_bin_kernel, dim3(n_worlds), dim3(kNarrowThreads), 0, stream, worlds, q, box_geom, wx, wy,
                       margin, out, count);
    return hipGetLastError();
}

int box_bin_max_boxes() {
    int n = 1;
    while ((n + 1) * 8 * (kPlanes + n) <= kMaxCandidates) ++n;
    return n;
}

}  // namespace kamx
