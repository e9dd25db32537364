// Contact generation for boxes in a bin: vertex-face tests of every box
// vertex against the floor (z = 0), the four walls (|x| = wx, |y| = wy) and
// every other box of the world.  A contact (Sec. 3: point, normal from body
// b to body a, signed gap, friction) is kept when its gap is below the
// margin; of those, the deepest ones up to the world's contact capacity,
// ties broken by key.  One workgroup per world, candidates in LDS.
#include "kamx_boxbin.h"

namespace kamx {

namespace {

constexpr int kNarrowThreads = 256;

// half_dt > 0: the boxes at their Moreau-Jean half-step poses (q advanced
// by half_dt with the twists u), the configuration the step builds its rows at
__global__ __launch_bounds__(kNarrowThreads) void box_bin_kernel(const WorldInfo *worlds, const float *q,
                                                                 const float *u, float half_dt,
                                                                 const float *box_geom, float wx, float wy,
                                                                 float margin, kamx_contact *out, int32_t *count) {
    __shared__ BoxLds S;
    const int w = blockIdx.x;
    const WorldInfo W = worlds[w];
    const float *qw = q + 7 * (long)W.b0;
    const float *uw = u + 6 * (long)W.b0;
    const int keep = box_bin_generate<kNarrowThreads>(
        S, W.nb, box_geom + 4 * (long)W.b0, wx, wy, margin, W.contact_cap,
        [&](int b, float c[3], float qt[4]) {
            float pose[7];
            for (int e = 0; e < 7; ++e) pose[e] = qw[7 * b + e];
            if (half_dt > 0.f) {
                double q7[7], u6[6], qm[7];
                for (int e = 0; e < 7; ++e) q7[e] = pose[e];
                for (int e = 0; e < 6; ++e) u6[e] = uw[6 * b + e];
                advance_pose(q7, u6, (double)half_dt, qm);
                for (int e = 0; e < 7; ++e) pose[e] = (float)qm[e];
            }
            for (int e = 0; e < 3; ++e) c[e] = pose[e];
            for (int e = 0; e < 4; ++e) qt[e] = pose[3 + e];
        },
        [&](int c, int key, float gap, const float p[3], const float n[3], float mu, int la, int lb) {
            kamx_contact ct;
            ct.body_a = W.b0 + la;
            ct.body_b = lb < 0 ? -1 : W.b0 + lb;
            for (int d = 0; d < 3; ++d) {
                ct.point[d] = p[d];
                ct.normal[d] = n[d];
            }
            ct.gap = gap;
            ct.mu = mu;
            ct.key = key;
            out[(long)w * kMaxContacts + c] = ct;
        });
    if (threadIdx.x == 0) count[w] = keep;
}

}  // namespace

hipError_t launch_box_bin(const WorldInfo *worlds, int n_worlds, const float *q, const float *u, float half_dt,
                          const float *box_geom, float wx, float wy, float margin, kamx_contact *out, int32_t *count,
                          hipStream_t stream) {
    if (n_worlds <= 0) return hipSuccess;
    hipLaunchKernelGGL(box_bin_kernel, dim3(n_worlds), dim3(kNarrowThreads), 0, stream, worlds, q, u, half_dt,
                       box_geom, wx, wy, margin, out, count);
    return hipGetLastError();
}

int box_bin_max_boxes() { return box_bin_max_boxes_of(); }

}  // namespace kamx
