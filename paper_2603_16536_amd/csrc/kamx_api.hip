// Host runtime of libkamx: model construction, device buffers, size
// buckets, and the C entry points declared in include/kamx.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "kamx_internal.h"

namespace kamx {
hipError_t launch_step(const StepArgs &args, int mc, int nt, int n, hipStream_t stream);
int step_threads_variants(int mc, int out[4]);
int bucket_capacity(int rows);
int sparse_row_class(int thread_rows);
size_t step_smem_bytes(int mc);
hipError_t launch_lpt_order(const int32_t *worlds, int n, const int32_t *iters, int32_t *order, hipStream_t stream);
hipError_t launch_advance_step(uint32_t *ctr, uint32_t inc, hipStream_t stream);
hipError_t launch_fk(const WorldInfo *worlds, int n_worlds, const int32_t *jint, const float *jf, const float *mass,
                     const float *inertia, float *q, float *u, const float *targets, int max_iters, float tol,
                     int32_t *iters, float *resid, hipStream_t stream);
hipError_t launch_box_bin(const WorldInfo *worlds, int n_worlds, const float *q, const float *u, float half_dt,
                          const float *box_geom, float wx, float wy, float margin, kamx_contact *out, int32_t *count,
                          hipStream_t stream);
int box_bin_max_boxes();
bool step_generates_box_contacts(int mc);
hipError_t launch_impulse_slots(const WorldInfo *worlds, int n_worlds, int n_contact_slots, int n_slots,
                                const float *lambda, const int32_t *keys, const int32_t *ncontacts, float *out,
                                hipStream_t stream);
MlpView mlp_view(kamx_mlp n);
int mlp_n_in(kamx_mlp n);
int mlp_n_out(kamx_mlp n);
int mlp_capacity(kamx_mlp n);
}  // namespace kamx

using namespace kamx;

static thread_local std::string g_error;

static kamx_status fail(kamx_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

namespace kamx {
kamx_status mlp_fail(kamx_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}
}  // namespace kamx

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(KAMX_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Bucket {
    int mc;
    int nt;             // workgroup size of the bucket's step kernel
    int n;
    int32_t *d_worlds;  // the bucket's worlds in index order
    int32_t *d_order;   // dispatch order of the next step (a permutation of d_worlds)
};

struct kamx_model_s {
    int device = 0;
    int n_worlds = 0, nb = 0, nj = 0, np = 0;
    int rows_cap = 0;
    int max_contacts = 0;
    kamx_params params{};
    uint32_t step_index = 0;
    int32_t schedule = KAMX_SCHED_CHAIN;
    int32_t *iter_log = nullptr;  // caller-owned [iter_log_rows * n_worlds] iterations per step
    int32_t *row_log = nullptr;   // caller-owned, same shape: active rows per step
    int32_t *status_log = nullptr;  // caller-owned, same shape: status bits per step
    int32_t iter_log_rows = 0;
    float *iterate_log = nullptr;  // caller-owned [rows_cap * 4] final iterate of the last step
    std::vector<int32_t> row_offsets;
    std::vector<Bucket> buckets;
    std::vector<void *> allocations;
    // device buffers
    WorldInfo *d_worlds = nullptr;
    float *d_mass = nullptr, *d_inertia = nullptr, *d_q = nullptr, *d_u = nullptr, *d_q0 = nullptr, *d_u0 = nullptr;
    int32_t *d_jint = nullptr;
    float *d_jf = nullptr;
    int32_t *d_pbody = nullptr;
    float *d_pf = nullptr;
    int32_t *d_coff = nullptr;
    const kamx_contact *d_contacts = nullptr;  // caller-owned
    const float *d_ext = nullptr;              // caller-owned
    float *d_lambda = nullptr, *d_lambda_ext = nullptr;
    int32_t *d_keys = nullptr, *d_iters = nullptr, *d_status = nullptr, *d_rows = nullptr;
    float *d_resid = nullptr;
    uint8_t *d_rlog = nullptr;
    int rlog_stride = 0;
    float *d_tau = nullptr;
    kamx_contact *d_contacts_out = nullptr;
    int32_t *d_ncontacts = nullptr, *d_reset_count = nullptr;
    uint64_t *d_phase_clk = nullptr;  // debug phase stamps (enabled by KAMX_PHASE_CLOCK)
    uint32_t *d_step = nullptr;       // step counter read by the step kernels
    // worlds solved matrix-free (Conjugate Residual), and the largest world
    bool has_sparse = false;
    int max_nb = 0, max_nj = 0;
    // learned warm start (worlds of identical structure only)
    bool uniform = false;
    int n_feat = 0, n_slots = 0, n_contact_slots = 0;
    int contact_cap0 = 0, n_slots_joint = 0, n_feat_body = 0, n_feat_joint = 0;  // parts of the layout
    kamx_mlp mlp = nullptr;
    float *d_ws = nullptr;  // network prediction by slot [n_worlds * n_slots]
    // generated contacts (boxes in a bin)
    bool box_bin = false;
    bool box_fused = false;  // every bucket's step kernel generates the contacts itself
    float bin_wx = 0.f, bin_wy = 0.f, bin_margin = 0.f;
    float *d_box_geom = nullptr;
    kamx_contact *d_gen = nullptr;
    int32_t *d_gen_count = nullptr;
    // captured multi-step rollouts: graph executables by step count; kernel
    // arguments are baked in, so every setter that changes one clears them
    std::vector<std::pair<int, hipGraphExec_t>> graphs;
    hipStream_t capture_stream = nullptr;
    // concurrent size buckets: one stream per bucket (default priority)
    std::vector<hipStream_t> bucket_streams;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
};

static constexpr int kGraphSteps = 32;  // steps per captured graph
static constexpr int kChainSteps = 64;  // steps per launch when worlds keep their workgroup

static void drop_graphs(kamx_model m) {
    for (auto &g : m->graphs) (void)hipGraphExecDestroy(g.second);
    m->graphs.clear();
}

template <typename T>
static kamx_status dalloc(kamx_model m, T **p, size_t count) {
    void *ptr = nullptr;
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) return fail(KAMX_ENOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    e = hipMemset(ptr, 0, bytes);
    if (e != hipSuccess) return fail(KAMX_EDEVICE, "hipMemset: %s", hipGetErrorString(e));
    m->allocations.push_back(ptr);
    *p = reinterpret_cast<T *>(ptr);
    return KAMX_OK;
}

#define K_TRY(expr)                       \
    do {                                  \
        kamx_status s_ = (expr);          \
        if (s_ != KAMX_OK) return s_;     \
    } while (0)

static kamx_status check_device() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(KAMX_EDEVICE, "pending device error: %s", hipGetErrorString(e));
    return KAMX_OK;
}

static kamx_status validate_params(const kamx_params *p) {
    if (p && p->integrator != KAMX_EULER && p->integrator != KAMX_MOREAU_JEAN)
        return fail(KAMX_EINVAL, "integrator must be KAMX_EULER or KAMX_MOREAU_JEAN");
    if (!p) return fail(KAMX_EINVAL, "params is NULL");
    if (!(p->dt > 0.f)) return fail(KAMX_EINVAL, "dt must be positive");
    if (!(p->eta >= 0.f) || !(p->rho_bilateral > 0.f) || !(p->rho_contact > 0.f))
        return fail(KAMX_EINVAL, "eta must be >= 0 and both rho > 0");
    if (p->max_iters < 1 || p->max_iters > 1000000) return fail(KAMX_EINVAL, "max_iters out of range");
    if (p->fixed_iters < 0 || p->fixed_iters > 1000000) return fail(KAMX_EINVAL, "fixed_iters out of range");
    if (!(p->restart_factor > 0.f)) return fail(KAMX_EINVAL, "restart_factor must be positive");
    if (p->warmstart < KAMX_WARM_COLD || p->warmstart > KAMX_WARM_LEARNED) return fail(KAMX_EINVAL, "bad warmstart");
    if (p->linear_solver < KAMX_SOLVER_AUTO || p->linear_solver > KAMX_SOLVER_SPARSE)
        return fail(KAMX_EINVAL, "linear_solver must be KAMX_SOLVER_AUTO, _DENSE or _SPARSE");
    if (p->cr_iters < 1 || p->cr_iters > 1000) return fail(KAMX_EINVAL, "cr_iters must be in [1, 1000]");
    if (!(p->adapt_ratio >= 0.f) || (p->adapt_ratio > 0.f && (!(p->adapt_factor > 1.f) || p->adapt_first < 1)))
        return fail(KAMX_EINVAL, "adapt_ratio must be >= 0; when on, adapt_factor > 1 and adapt_first >= 1");
    return KAMX_OK;
}

static SolverParams to_solver(const kamx_params &p) {
    SolverParams s;
    s.dt = p.dt;
    s.gx = p.gravity[0];
    s.gy = p.gravity[1];
    s.gz = p.gravity[2];
    s.eta = p.eta;
    s.rho_bil = p.rho_bilateral;
    s.rho_c = p.rho_contact;
    s.eps = p.eps;
    s.max_iters = p.max_iters;
    s.fixed_iters = p.fixed_iters;
    s.accel = p.accel;
    s.restart_factor = p.restart_factor;
    s.precond = p.precond;
    s.baumgarte = p.baumgarte;
    s.warmstart = p.warmstart;
    s.contact_margin = p.contact_margin;
    s.torque_sigma = p.torque_sigma;
    s.seed_lo = (uint32_t)(p.seed & 0xFFFFFFFFull);
    s.seed_hi = (uint32_t)(p.seed >> 32);
    s.reset_height = p.reset_height;
    s.log_restarts = p.log_restarts;
    s.integrator = p.integrator;
    s.cr_iters = p.cr_iters;
    s.adapt_ratio = p.adapt_ratio;
    s.adapt_factor = p.adapt_factor;
    s.adapt_first = p.adapt_first;
    return s;
}

extern "C" {

void kamx_default_params(kamx_params *p) {
    if (!p) return;
    memset(p, 0, sizeof *p);
    p->dt = 2e-3f;
    p->gravity[2] = -9.81f;
    p->eta = 1e-4f;
    p->rho_bilateral = 1e-4f;
    p->rho_contact = 0.3f;
    p->eps = 1e-6f;
    p->max_iters = 2000;
    p->fixed_iters = 0;
    p->accel = 1;
    p->restart_factor = 0.999f;
    p->precond = 1;
    p->baumgarte = 0.2f;
    p->warmstart = KAMX_WARM_COLD;
    p->contact_margin = 0.02f;
    p->torque_sigma = 0.f;
    p->seed = 0;
    p->reset_height = -INFINITY;
    p->log_restarts = 0;
    p->integrator = KAMX_EULER;
    p->linear_solver = KAMX_SOLVER_AUTO;
    p->cr_iters = 9;
    p->adapt_ratio = 10.f;
    p->adapt_factor = 5.f;
    p->adapt_first = 100;
}

const char *kamx_last_error(void) { return g_error.c_str(); }

static kamx_status ensure_rlog(kamx_model m) {
    if (!m->params.log_restarts) return KAMX_OK;
    if (m->d_rlog && m->rlog_stride == m->params.max_iters) return KAMX_OK;
    drop_graphs(m);
    if (m->d_rlog) {
        HIP_TRY(hipDeviceSynchronize());
        auto it = std::find(m->allocations.begin(), m->allocations.end(), (void *)m->d_rlog);
        if (it != m->allocations.end()) m->allocations.erase(it);
        HIP_TRY(hipFree(m->d_rlog));
        m->d_rlog = nullptr;
    }
    K_TRY(dalloc(m, &m->d_rlog, (size_t)m->n_worlds * m->params.max_iters));
    m->rlog_stride = m->params.max_iters;
    return KAMX_OK;
}

kamx_status kamx_model_create(const kamx_body_desc *bodies, int32_t nb, const kamx_joint_desc *joints, int32_t nj,
                              const kamx_probe_desc *probes, int32_t np, const int32_t *reset_body, int32_t n_worlds,
                              int32_t max_contacts_per_world, const kamx_params *params, kamx_model *out) {
    if (!out) return fail(KAMX_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_worlds <= 0 || nb <= 0 || nj < 0 || np < 0) return fail(KAMX_EINVAL, "bad sizes");
    if (!bodies || (nj > 0 && !joints) || (np > 0 && !probes)) return fail(KAMX_EINVAL, "NULL descriptor array");
    if (max_contacts_per_world < 0 || max_contacts_per_world > kMaxContacts)
        return fail(KAMX_EINVAL, "max_contacts_per_world must be in [0, %d]", kMaxContacts);
    K_TRY(validate_params(params));
    K_TRY(check_device());

    // per-world ranges (inputs sorted by world)
    std::vector<WorldInfo> wi(n_worlds);
    memset(wi.data(), 0, sizeof(WorldInfo) * n_worlds);
    for (int w = 0; w < n_worlds; ++w) wi[w].reset_body = -1;
    auto ranges = [&](auto get_world, int n, const char *what, auto set) -> kamx_status {
        int prev = -1;
        for (int k = 0; k < n; ++k) {
            int w = get_world(k);
            if (w < 0 || w >= n_worlds) return fail(KAMX_EINVAL, "%s %d: world %d out of range", what, k, w);
            if (w < prev) return fail(KAMX_EINVAL, "%s must be sorted by world (%s %d)", what, what, k);
            if (w != prev) set(w, k);
            prev = w;
        }
        return KAMX_OK;
    };
    std::vector<int> bstart(n_worlds, -1), jstart(n_worlds, -1), pstart(n_worlds, -1);
    K_TRY(ranges([&](int k) { return bodies[k].world; }, nb, "body", [&](int w, int k) { bstart[w] = k; }));
    K_TRY(ranges([&](int k) { return joints[k].world; }, nj, "joint", [&](int w, int k) { jstart[w] = k; }));
    K_TRY(ranges([&](int k) { return probes[k].world; }, np, "probe", [&](int w, int k) { pstart[w] = k; }));
    for (int k = 0; k < nb; ++k) wi[bodies[k].world].nb++;
    for (int k = 0; k < nj; ++k) wi[joints[k].world].nj++;
    for (int k = 0; k < np; ++k) wi[probes[k].world].np++;
    for (int k = 0; k < nb; ++k) {
        const kamx_body_desc &b = bodies[k];
        if (!(b.mass > 0.f) || !(b.inertia[0] > 0.f) || !(b.inertia[1] > 0.f) || !(b.inertia[2] > 0.f))
            return fail(KAMX_EINVAL, "body %d: mass and inertia must be positive", k);
    }
    std::vector<int32_t> row_off(n_worlds + 1, 0);
    int cursor_b = 0, cursor_j = 0, cursor_p = 0;
    for (int w = 0; w < n_worlds; ++w) {
        WorldInfo &W = wi[w];
        W.b0 = cursor_b;
        W.j0 = cursor_j;
        W.p0 = cursor_p;
        cursor_b += W.nb;
        cursor_j += W.nj;
        cursor_p += W.np;
        if (W.nb < 1 || W.nb > KAMX_MAX_BODIES_SPARSE)
            return fail(KAMX_EINVAL, "world %d: %d bodies (1..%d)", w, W.nb, KAMX_MAX_BODIES_SPARSE);
        if (W.nj > KAMX_MAX_JOINTS_SPARSE)
            return fail(KAMX_EINVAL, "world %d: %d joints (max %d)", w, W.nj, KAMX_MAX_JOINTS_SPARSE);
        if (W.np > kMaxContacts) return fail(KAMX_EINVAL, "world %d: %d probes (max %d)", w, W.np, kMaxContacts);
        W.nlim = 0;
        W.ndrv = 0;
        for (int j = W.j0; j < W.j0 + W.nj; ++j) {
            const kamx_joint_desc &J = joints[j];
            if (J.type != KAMX_REVOLUTE && J.type != KAMX_PRISMATIC)
                return fail(KAMX_EINVAL, "joint %d: unknown type %d", j, J.type);
            if (J.body_a < W.b0 || J.body_a >= W.b0 + W.nb)
                return fail(KAMX_EINVAL, "joint %d: body_a %d not in world %d", j, J.body_a, w);
            if (J.body_b != -1 && (J.body_b < W.b0 || J.body_b >= W.b0 + W.nb || J.body_b == J.body_a))
                return fail(KAMX_EINVAL, "joint %d: body_b %d invalid", j, J.body_b);
            if (!isnan(J.limit_lo) || !isnan(J.limit_hi)) W.nlim++;
            if (!(J.damping >= 0.f) || !(J.armature >= 0.f) || !isfinite(J.damping) || !isfinite(J.armature))
                return fail(KAMX_EINVAL, "joint %d: damping and armature must be finite and >= 0", j);
            if (J.implicit_drive) {
                if (!(J.kp >= 0.f) || !(J.kd >= 0.f) || !isfinite(J.kp) || !isfinite(J.kd) || !isfinite(J.ref))
                    return fail(KAMX_EINVAL, "joint %d: implicit drive needs finite kp, kd >= 0 and ref", j);
                if (!(J.kp > 0.f || J.kd > 0.f || J.damping > 0.f || J.armature > 0.f))
                    return fail(KAMX_EINVAL, "joint %d: implicit drive with all gains zero", j);
                W.ndrv++;
            } else if (J.damping != 0.f || J.armature != 0.f) {
                return fail(KAMX_EINVAL, "joint %d: damping and armature need implicit_drive", j);
            }
        }
        for (int k = W.p0; k < W.p0 + W.np; ++k)
            if (probes[k].body < W.b0 || probes[k].body >= W.b0 + W.nb)
                return fail(KAMX_EINVAL, "probe %d: body %d not in world %d", k, probes[k].body, w);
        W.contact_cap = std::max(W.np, (int)max_contacts_per_world);
        W.row_cap = 5 * W.nj + W.nlim + W.ndrv + 3 * W.contact_cap;
        // dense (assembled and factored Delassus matrix) where the world fits
        // the dense limits, matrix-free otherwise (Sec. 5.1), unless the
        // parameters force one of them
        {
            const bool dense_ok = W.nb <= kMaxBodies && W.nj <= kMaxJoints && W.row_cap <= kMaxRows;
            const int thread_rows = ((5 * W.nj + W.nlim + W.ndrv + 3) & ~3) + 4 * W.contact_cap;
            const bool sparse_ok = thread_rows <= KAMX_MAX_THREAD_ROWS_SPARSE;
            const int solver = params->linear_solver;
            if (solver == KAMX_SOLVER_DENSE && !dense_ok)
                return fail(KAMX_EINVAL, "world %d: %d bodies, %d joints, %d rows exceed the dense limits (%d, %d, %d)", w,
                            W.nb, W.nj, W.row_cap, kMaxBodies, kMaxJoints, kMaxRows);
            if ((solver == KAMX_SOLVER_SPARSE || !dense_ok) && !sparse_ok)
                return fail(KAMX_EINVAL, "world %d: %d thread rows exceed the matrix-free limit %d", w, thread_rows,
                            KAMX_MAX_THREAD_ROWS_SPARSE);
            W.sparse = solver == KAMX_SOLVER_SPARSE || (solver == KAMX_SOLVER_AUTO && !dense_ok);
        }
        W.row_base = row_off[w];
        row_off[w + 1] = row_off[w] + W.row_cap;
        if (reset_body && reset_body[w] >= 0) {
            if (reset_body[w] < W.b0 || reset_body[w] >= W.b0 + W.nb)
                return fail(KAMX_EINVAL, "reset_body of world %d not in the world", w);
            W.reset_body = reset_body[w] - W.b0;
        }
    }

    kamx_model m = new kamx_model_s();
    HIP_TRY(hipGetDevice(&m->device));
    m->n_worlds = n_worlds;
    m->nb = nb;
    m->nj = nj;
    m->np = np;
    m->rows_cap = row_off[n_worlds];
    m->max_contacts = max_contacts_per_world;
    m->params = *params;
    m->row_offsets = row_off;
    m->uniform = true;
    for (int w = 0; w < n_worlds; ++w) {
        m->has_sparse = m->has_sparse || wi[w].sparse;
        m->max_nb = std::max(m->max_nb, (int)wi[w].nb);
        m->max_nj = std::max(m->max_nj, (int)wi[w].nj);
    }
    for (int w = 1; w < n_worlds; ++w)
        if (wi[w].nb != wi[0].nb || wi[w].nj != wi[0].nj || wi[w].nlim != wi[0].nlim ||
            wi[w].ndrv != wi[0].ndrv || wi[w].contact_cap != wi[0].contact_cap)
            m->uniform = false;
    m->n_contact_slots = m->contact_cap0 = wi[0].contact_cap;
    m->n_slots_joint = 5 * wi[0].nj + wi[0].nlim + wi[0].ndrv;
    m->n_feat_body = 13 * wi[0].nb;
    m->n_feat_joint = wi[0].nj;
    m->n_slots = m->n_slots_joint + 3 * m->n_contact_slots;
    m->n_feat = m->n_feat_body + m->n_slots + m->n_feat_joint;

    auto cleanup_fail = [&](kamx_status st) {
        kamx_model_destroy(m);
        return st;
    };
#define M_TRY(expr)                               \
    do {                                          \
        kamx_status s_ = (expr);                  \
        if (s_ != KAMX_OK) return cleanup_fail(s_); \
    } while (0)

    // host staging
    std::vector<float> mass(nb), inertia(3 * (size_t)nb);
    for (int k = 0; k < nb; ++k) {
        mass[k] = bodies[k].mass;
        for (int e = 0; e < 3; ++e) inertia[3 * k + e] = bodies[k].inertia[e];
    }
    std::vector<int32_t> jint(4 * (size_t)std::max(nj, 1), 0);
    std::vector<float> jf(kJointFloats * (size_t)std::max(nj, 1), 0.f);
    for (int j = 0; j < nj; ++j) {
        const kamx_joint_desc &J = joints[j];
        const WorldInfo &W = wi[J.world];
        jint[4 * j] = J.type;
        jint[4 * j + 1] = J.body_a - W.b0;
        jint[4 * j + 2] = J.body_b < 0 ? -1 : J.body_b - W.b0;
        int fl = 0;
        if (J.actuated) fl |= kJointActuated;
        if (!isnan(J.limit_lo) || !isnan(J.limit_hi)) fl |= kJointLimited;
        if (J.implicit_drive) fl |= kJointDriven;
        jint[4 * j + 3] = fl;
        float *f = &jf[kJointFloats * (size_t)j];
        for (int e = 0; e < 7; ++e) {
            f[e] = J.frame_a[e];
            f[7 + e] = J.frame_b[e];
        }
        f[14] = J.limit_lo;
        f[15] = J.limit_hi;
        f[16] = J.kp;
        f[17] = J.kd;
        f[18] = J.ref;
        f[19] = J.damping;
        f[20] = J.armature;
    }
    std::vector<int32_t> pbody(std::max(np, 1), 0);
    std::vector<float> pf(4 * (size_t)std::max(np, 1), 0.f);
    for (int k = 0; k < np; ++k) {
        const WorldInfo &W = wi[probes[k].world];
        pbody[k] = probes[k].body - W.b0;
        for (int e = 0; e < 3; ++e) pf[4 * k + e] = probes[k].point[e];
        pf[4 * k + 3] = probes[k].mu;
    }

    M_TRY(dalloc(m, &m->d_worlds, n_worlds));
    M_TRY(dalloc(m, &m->d_mass, nb));
    M_TRY(dalloc(m, &m->d_inertia, 3 * (size_t)nb));
    M_TRY(dalloc(m, &m->d_q, 7 * (size_t)nb));
    M_TRY(dalloc(m, &m->d_u, 6 * (size_t)nb));
    M_TRY(dalloc(m, &m->d_q0, 7 * (size_t)nb));
    M_TRY(dalloc(m, &m->d_u0, 6 * (size_t)nb));
    M_TRY(dalloc(m, &m->d_jint, jint.size()));
    M_TRY(dalloc(m, &m->d_jf, jf.size()));
    M_TRY(dalloc(m, &m->d_pbody, pbody.size()));
    M_TRY(dalloc(m, &m->d_pf, pf.size()));
    M_TRY(dalloc(m, &m->d_coff, n_worlds + 1));
    M_TRY(dalloc(m, &m->d_step, 1));
    M_TRY(dalloc(m, &m->d_lambda, m->rows_cap));
    M_TRY(dalloc(m, &m->d_lambda_ext, m->rows_cap));
    M_TRY(dalloc(m, &m->d_keys, (size_t)n_worlds * kMaxContacts));
    M_TRY(dalloc(m, &m->d_iters, n_worlds));
    M_TRY(dalloc(m, &m->d_status, n_worlds));
    M_TRY(dalloc(m, &m->d_rows, n_worlds));
    M_TRY(dalloc(m, &m->d_resid, 4 * (size_t)n_worlds));
    M_TRY(dalloc(m, &m->d_tau, std::max(nj, 1)));
    M_TRY(dalloc(m, &m->d_contacts_out, (size_t)n_worlds * kMaxContacts));
    M_TRY(dalloc(m, &m->d_ncontacts, n_worlds));
    M_TRY(dalloc(m, &m->d_reset_count, n_worlds));
    M_TRY(ensure_rlog(m));
    if (getenv("KAMX_PHASE_CLOCK")) M_TRY(dalloc(m, &m->d_phase_clk, 16 * (size_t)n_worlds));

    auto up = [&](void *dst, const void *src, size_t bytes) -> kamx_status {
        hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(KAMX_EDEVICE, "upload: %s", hipGetErrorString(e));
        return KAMX_OK;
    };
    M_TRY(up(m->d_worlds, wi.data(), sizeof(WorldInfo) * n_worlds));
    M_TRY(up(m->d_mass, mass.data(), sizeof(float) * nb));
    M_TRY(up(m->d_inertia, inertia.data(), sizeof(float) * 3 * nb));
    M_TRY(up(m->d_jint, jint.data(), sizeof(int32_t) * jint.size()));
    M_TRY(up(m->d_jf, jf.data(), sizeof(float) * jf.size()));
    M_TRY(up(m->d_pbody, pbody.data(), sizeof(int32_t) * pbody.size()));
    M_TRY(up(m->d_pf, pf.data(), sizeof(float) * pf.size()));

    // size buckets: worlds grouped by the smallest row capacity class
    // (slots 0-6: dense buckets of 32, ..., 224 rows; 7-9: matrix-free
    // buckets of 256, 512 and 1024 thread rows)
    std::vector<std::vector<int32_t>> groups(10);
    for (int w = 0; w < n_worlds; ++w) {
        int slot;
        if (wi[w].sparse) {
            const int tr = ((5 * wi[w].nj + wi[w].nlim + wi[w].ndrv + 3) & ~3) + 4 * wi[w].contact_cap;
            const int nt = sparse_row_class(std::max(tr, 1));
            if (nt < 0) return cleanup_fail(fail(KAMX_EINVAL, "world %d: no matrix-free class for %d rows", w, tr));
            slot = nt == 256 ? 7 : (nt == 512 ? 8 : 9);
        } else {
            int mc = bucket_capacity(std::max(wi[w].row_cap, 1));
            if (mc < 0) return cleanup_fail(fail(KAMX_EINVAL, "world %d: no bucket for %d rows", w, wi[w].row_cap));
            slot = mc / 32 - 1;
        }
        groups[slot].push_back(w);
    }
    for (int s = 9; s >= 0; --s) {  // largest worlds first
        if (groups[s].empty()) continue;
        Bucket b;
        b.mc = s < 7 ? 32 * (s + 1) : (s == 7 ? 256 : (s == 8 ? 512 : 1024));
        int nts[4];
        if (step_threads_variants(b.mc, nts) < 1) return cleanup_fail(fail(KAMX_EINVAL, "no kernel for %d rows", b.mc));
        b.nt = nts[0];
        b.n = (int)groups[s].size();
        b.d_worlds = nullptr;
        M_TRY(dalloc(m, &b.d_worlds, groups[s].size()));
        M_TRY(up(b.d_worlds, groups[s].data(), sizeof(int32_t) * groups[s].size()));
        b.d_order = nullptr;
        M_TRY(dalloc(m, &b.d_order, groups[s].size()));
        M_TRY(up(b.d_order, groups[s].data(), sizeof(int32_t) * groups[s].size()));
        m->buckets.push_back(b);
    }
    *out = m;
    return KAMX_OK;
#undef M_TRY
}

kamx_status kamx_model_destroy(kamx_model m) {
    if (!m) return KAMX_OK;
    (void)hipDeviceSynchronize();
    drop_graphs(m);
    if (m->capture_stream) (void)hipStreamDestroy(m->capture_stream);
    for (hipStream_t st : m->bucket_streams) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : m->ev_join) (void)hipEventDestroy(ev);
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    for (void *p : m->allocations) (void)hipFree(p);
    delete m;
    return KAMX_OK;
}

kamx_status kamx_set_params(kamx_model m, const kamx_params *params) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    K_TRY(validate_params(params));
    if (params->linear_solver != m->params.linear_solver)
        return fail(KAMX_EINVAL, "linear_solver is fixed at model creation");
    m->params = *params;
    drop_graphs(m);
    K_TRY(ensure_rlog(m));
    return KAMX_OK;
}

kamx_status kamx_model_info(kamx_model m, int32_t *n_bodies, int32_t *n_joints, int32_t *rows_capacity,
                            int32_t *n_buckets, int32_t *row_offsets) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (n_bodies) *n_bodies = m->nb;
    if (n_joints) *n_joints = m->nj;
    if (rows_capacity) *rows_capacity = m->rows_cap;
    if (n_buckets) *n_buckets = (int32_t)m->buckets.size();
    if (row_offsets) memcpy(row_offsets, m->row_offsets.data(), sizeof(int32_t) * (m->n_worlds + 1));
    return KAMX_OK;
}

kamx_status kamx_state_upload(kamx_model m, const float *q_dev, const float *u_dev, int32_t as_reset_state,
                              kamx_stream stream) {
    if (!m || !q_dev || !u_dev) return fail(KAMX_EINVAL, "NULL argument");
    K_TRY(check_device());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(m->d_q, q_dev, sizeof(float) * 7 * m->nb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(m->d_u, u_dev, sizeof(float) * 6 * m->nb, hipMemcpyDeviceToDevice, s));
    if (as_reset_state) {
        HIP_TRY(hipMemcpyAsync(m->d_q0, q_dev, sizeof(float) * 7 * m->nb, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(m->d_u0, u_dev, sizeof(float) * 6 * m->nb, hipMemcpyDeviceToDevice, s));
    }
    return KAMX_OK;
}

kamx_status kamx_state_download(kamx_model m, float *q_dev, float *u_dev, kamx_stream stream) {
    if (!m || !q_dev || !u_dev) return fail(KAMX_EINVAL, "NULL argument");
    K_TRY(check_device());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(q_dev, m->d_q, sizeof(float) * 7 * m->nb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(u_dev, m->d_u, sizeof(float) * 6 * m->nb, hipMemcpyDeviceToDevice, s));
    return KAMX_OK;
}

kamx_status kamx_contacts_upload(kamx_model m, const kamx_contact *contacts_dev, const int32_t *world_offsets,
                                 kamx_stream stream) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (!contacts_dev) {
        if (m->d_contacts) drop_graphs(m);
        m->d_contacts = nullptr;
        return KAMX_OK;
    }
    if (!world_offsets) return fail(KAMX_EINVAL, "world_offsets is NULL");
    if (world_offsets[0] != 0) return fail(KAMX_EINVAL, "world_offsets[0] must be 0");
    for (int w = 0; w < m->n_worlds; ++w) {
        int n = world_offsets[w + 1] - world_offsets[w];
        if (n < 0 || n > m->max_contacts)
            return fail(KAMX_EINVAL, "world %d: %d contacts (max %d for this model)", w, n, m->max_contacts);
    }
    K_TRY(check_device());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(m->d_coff, world_offsets, sizeof(int32_t) * (m->n_worlds + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // world_offsets is a host array of the caller
    if (m->d_contacts != contacts_dev || m->box_bin) drop_graphs(m);
    m->d_contacts = contacts_dev;
    m->box_bin = false;
    return KAMX_OK;
}

kamx_status kamx_set_external(kamx_model m, const float *joint_torque_dev, kamx_stream stream) {
    (void)stream;
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (m->d_ext != joint_torque_dev) drop_graphs(m);
    m->d_ext = joint_torque_dev;
    return KAMX_OK;
}

kamx_status kamx_set_warmstart(kamx_model m, const float *lambda_dev, kamx_stream stream) {
    if (!m || !lambda_dev) return fail(KAMX_EINVAL, "NULL argument");
    K_TRY(check_device());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(m->d_lambda_ext, lambda_dev, sizeof(float) * m->rows_cap, hipMemcpyDeviceToDevice, s));
    return KAMX_OK;
}

static StepArgs step_args(kamx_model m) {
    StepArgs a;
    memset(&a, 0, sizeof a);
    a.worlds = m->d_worlds;
    a.mass = m->d_mass;
    a.inertia = m->d_inertia;
    a.q = m->d_q;
    a.u = m->d_u;
    a.q0 = m->d_q0;
    a.u0 = m->d_u0;
    a.jint = m->d_jint;
    a.jf = m->d_jf;
    a.ext_tau = m->d_ext;
    a.pbody = m->d_pbody;
    a.pf = m->d_pf;
    if (m->box_bin && m->box_fused) {
        a.box_geom = m->d_box_geom;
        a.bin_wx = m->bin_wx;
        a.bin_wy = m->bin_wy;
        a.bin_margin = m->bin_margin;
    }
    a.contacts = m->box_bin ? m->d_gen : m->d_contacts;
    a.coff = m->d_coff;
    a.ccount = m->box_bin ? m->d_gen_count : nullptr;
    a.lambda = m->d_lambda;
    a.lambda_ext = m->d_lambda_ext;
    a.keys = m->d_keys;
    a.iters = m->d_iters;
    a.resid = m->d_resid;
    a.status = m->d_status;
    a.rows = m->d_rows;
    a.rlog = m->params.log_restarts ? m->d_rlog : nullptr;
    a.iterate_out = m->iterate_log;
    a.tau_out = m->d_tau;
    a.contacts_out = m->d_contacts_out;
    a.ncontacts_out = m->d_ncontacts;
    a.reset_count = m->d_reset_count;
    a.phase_clk = m->d_phase_clk;
    a.p = to_solver(m->params);
    a.step_ctr = m->d_step;
    a.nsteps = 1;
    a.n_worlds = m->n_worlds;
    a.stage = 0;
    a.n_feat = m->n_feat;
    a.ws_slots = m->d_ws;
    if (m->mlp) a.mlp = mlp_view(m->mlp);
    a.n_contact_slots = m->n_contact_slots;
    return a;
}

// time by which the stand-alone contact generation advances the poses: the
// step builds its rows at the half-step configuration for Moreau-Jean
static float gen_half_dt(kamx_model m) {
    return m->params.integrator == KAMX_MOREAU_JEAN ? 0.5f * m->params.dt : 0.f;
}

static kamx_status ensure_bucket_streams(kamx_model m) {
    if (!m->bucket_streams.empty()) return KAMX_OK;
    HIP_TRY(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
    for (size_t i = 0; i < m->buckets.size(); ++i) {
        hipStream_t st = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        m->bucket_streams.push_back(st);
        hipEvent_t ev = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        m->ev_join.push_back(ev);
    }
    return KAMX_OK;
}

// Feature pass of every bucket (the step kernels stopped after actuation).
static kamx_status enqueue_features(kamx_model m, float *x, hipStream_t s) {
    StepArgs a = step_args(m);
    a.stage = 1;
    a.features = x;
    a.phase_clk = nullptr;
    for (const Bucket &b : m->buckets) {
        a.bucket_worlds = b.d_worlds;
        a.n_bucket_worlds = b.n;
        hipError_t e = launch_step(a, b.mc, b.nt, b.n, s);
        if (e != hipSuccess) return fail(KAMX_EDEVICE, "feature launch (bucket %d rows): %s", b.mc, hipGetErrorString(e));
    }
    return KAMX_OK;
}

// One launch per bucket advancing every world by n steps (n > 1 only when
// every step's inputs are already on the device: no per-step contact
// generation or network), starting at position pos of the current call.
// Single steps also run the contact generation, the feature pass and the
// network when those are on, and reorder the bucket for the next step.
static kamx_status enqueue_launch(kamx_model m, int n, int pos, hipStream_t s) {
    StepArgs base = step_args(m);
    base.nsteps = n;
    base.n_worlds = m->n_worlds;
    if (m->iter_log && pos < m->iter_log_rows) {
        base.iter_log = m->iter_log + (long)pos * m->n_worlds;
        base.row_log = m->row_log ? m->row_log + (long)pos * m->n_worlds : nullptr;
        base.status_log = m->status_log ? m->status_log + (long)pos * m->n_worlds : nullptr;
        base.iter_log_rows = m->iter_log_rows - pos;
    }
    const bool lpt = n == 1 && m->schedule != KAMX_SCHED_INDEX;
    if (m->box_bin && !m->box_fused) {
        hipError_t e = launch_box_bin(m->d_worlds, m->n_worlds, m->d_q, m->d_u, gen_half_dt(m), m->d_box_geom,
                                      m->bin_wx, m->bin_wy, m->bin_margin, m->d_gen, m->d_gen_count, s);
        if (e != hipSuccess) return fail(KAMX_EDEVICE, "contact generation launch: %s", hipGetErrorString(e));
    }
    // several buckets run concurrently on the model's bucket streams (fork
    // from s, join back), so the tail of one bucket overlaps the others; a
    // single bucket runs on s itself
    const int nbk = (int)m->buckets.size();
    const bool fork = nbk > 1;
    if (fork) {
        K_TRY(ensure_bucket_streams(m));
        HIP_TRY(hipEventRecord(m->ev_fork, s));
    }
    for (int bi = 0; bi < nbk; ++bi) {
        const Bucket &b = m->buckets[bi];
        hipStream_t bs = fork ? m->bucket_streams[bi] : s;
        if (fork) HIP_TRY(hipStreamWaitEvent(bs, m->ev_fork, 0));
        StepArgs a = base;
        a.bucket_worlds = lpt ? b.d_order : b.d_worlds;
        a.n_bucket_worlds = b.n;
        hipError_t e = launch_step(a, b.mc, b.nt, b.n, bs);
        if (e != hipSuccess) return fail(KAMX_EDEVICE, "step launch (bucket %d rows): %s", b.mc, hipGetErrorString(e));
        if (lpt && b.n > 1) {
            e = launch_lpt_order(b.d_worlds, b.n, m->d_iters, b.d_order, bs);
            if (e != hipSuccess) return fail(KAMX_EDEVICE, "schedule launch (bucket %d rows): %s", b.mc, hipGetErrorString(e));
        }
        if (fork) {
            HIP_TRY(hipEventRecord(m->ev_join[bi], bs));
            HIP_TRY(hipStreamWaitEvent(s, m->ev_join[bi], 0));
        }
    }
    hipError_t e = launch_advance_step(m->d_step, (uint32_t)n, s);
    if (e != hipSuccess) return fail(KAMX_EDEVICE, "counter launch: %s", hipGetErrorString(e));
    return KAMX_OK;
}

static bool chained(kamx_model m) { return m->schedule == KAMX_SCHED_CHAIN && (!m->box_bin || m->box_fused); }

// Enqueue nsteps steps from position pos of the current call.
static kamx_status enqueue_steps(kamx_model m, int nsteps, hipStream_t s, int pos = 0) {
    const bool chain = chained(m);
    for (int k = 0; k < nsteps;) {
        const int n = chain ? std::min(nsteps - k, kChainSteps) : 1;
        K_TRY(enqueue_launch(m, n, pos + k, s));
        k += n;
    }
    return KAMX_OK;
}

// Graph executable of n steps (captured on the model's own stream on first
// use; replayed on any stream).
static kamx_status rollout_graph(kamx_model m, int n, hipGraphExec_t *out) {
    for (auto &g : m->graphs)
        if (g.first == n) {
            *out = g.second;
            return KAMX_OK;
        }
    if (!m->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&m->capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(m->capture_stream, hipStreamCaptureModeRelaxed));
    kamx_status st = enqueue_steps(m, n, m->capture_stream, 0);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(m->capture_stream, &graph);
    if (st != KAMX_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(KAMX_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(KAMX_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
    m->graphs.push_back({n, exec});
    *out = exec;
    return KAMX_OK;
}

kamx_status kamx_step(kamx_model m, int32_t nsteps, kamx_stream stream) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (nsteps < 0) return fail(KAMX_EINVAL, "nsteps < 0");
    if (m->params.warmstart == KAMX_WARM_LEARNED && !m->mlp)
        return fail(KAMX_ESTATE, "warm start LEARNED needs a network (kamx_model_attach_mlp)");
    K_TRY(check_device());
    if (m->params.log_restarts) K_TRY(ensure_rlog(m));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (nsteps == 1 || chained(m)) {
        K_TRY(enqueue_steps(m, nsteps, s, 0));
    } else if (nsteps > 1) {
        // per-step launches replayed from captured graphs; the iteration
        // log positions are part of the captured arguments, so a call is
        // cut into graph-sized pieces at fixed positions
        const int chunk = std::min<int>(nsteps, kGraphSteps);
        int pos = 0;
        hipGraphExec_t g = nullptr;
        if (!m->iter_log) {
            K_TRY(rollout_graph(m, chunk, &g));
            for (int k = 0; k < nsteps / chunk; ++k) HIP_TRY(hipGraphLaunch(g, s));
            pos = (nsteps / chunk) * chunk;
            if (nsteps % chunk) {
                K_TRY(rollout_graph(m, nsteps % chunk, &g));
                HIP_TRY(hipGraphLaunch(g, s));
            }
        } else {
            K_TRY(enqueue_steps(m, nsteps, s, 0));
        }
        (void)pos;
    }
    m->step_index += (uint32_t)nsteps;
    return KAMX_OK;
}

kamx_status kamx_bucket_count(kamx_model m, int32_t *n_buckets) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (n_buckets) *n_buckets = (int32_t)m->buckets.size();
    return KAMX_OK;
}

kamx_status kamx_bucket_info(kamx_model m, int32_t bucket, int32_t *rows_cap, int32_t *n_worlds, int32_t *threads,
                             int32_t *n_variants, int32_t *variants) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (bucket < 0 || bucket >= (int32_t)m->buckets.size()) return fail(KAMX_EINVAL, "bucket %d out of range", bucket);
    const Bucket &b = m->buckets[bucket];
    int nts[4] = {0, 0, 0, 0};
    const int nv = step_threads_variants(b.mc, nts);
    if (rows_cap) *rows_cap = b.mc;
    if (n_worlds) *n_worlds = b.n;
    if (threads) *threads = b.nt;
    if (n_variants) *n_variants = nv;
    if (variants)
        for (int k = 0; k < 4; ++k) variants[k] = k < nv ? nts[k] : 0;
    return KAMX_OK;
}

kamx_status kamx_set_bucket_threads(kamx_model m, int32_t bucket, int32_t threads) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (bucket < 0 || bucket >= (int32_t)m->buckets.size()) return fail(KAMX_EINVAL, "bucket %d out of range", bucket);
    Bucket &b = m->buckets[bucket];
    int nts[4];
    const int nv = step_threads_variants(b.mc, nts);
    for (int k = 0; k < nv; ++k)
        if (nts[k] == threads) {
            drop_graphs(m);
            b.nt = threads;
            return KAMX_OK;
        }
    return fail(KAMX_EINVAL, "bucket of %d rows has no kernel for %d threads", b.mc, threads);
}

namespace {
struct StateSpan {
    void *p;
    size_t bytes;
};
}  // namespace

// Every device buffer a step writes (the state the autotuner restores).
static std::vector<StateSpan> step_state(kamx_model m) {
    std::vector<StateSpan> v;
    auto add = [&](void *p, size_t bytes) {
        if (p && bytes) v.push_back({p, bytes});
    };
    const size_t nw = (size_t)m->n_worlds;
    add(m->d_q, sizeof(float) * 7 * (size_t)m->nb);
    add(m->d_u, sizeof(float) * 6 * (size_t)m->nb);
    add(m->d_lambda, sizeof(float) * (size_t)m->rows_cap);
    add(m->d_keys, sizeof(int32_t) * nw * kMaxContacts);
    add(m->d_iters, sizeof(int32_t) * nw);
    add(m->d_status, sizeof(int32_t) * nw);
    add(m->d_rows, sizeof(int32_t) * nw);
    add(m->d_resid, sizeof(float) * 4 * nw);
    add(m->d_tau, sizeof(float) * (size_t)std::max(m->nj, 1));
    add(m->d_contacts_out, sizeof(kamx_contact) * nw * kMaxContacts);
    add(m->d_ncontacts, sizeof(int32_t) * nw);
    add(m->d_reset_count, sizeof(int32_t) * nw);
    add(m->d_step, sizeof(uint32_t));
    add(m->d_ws, sizeof(float) * nw * (size_t)m->n_slots);
    add(m->d_gen, sizeof(kamx_contact) * nw * kMaxContacts);
    add(m->d_gen_count, sizeof(int32_t) * nw);
    add(m->d_rlog, nw * (size_t)m->rlog_stride);
    add(m->d_phase_clk, sizeof(uint64_t) * 16 * nw);
    for (const Bucket &b : m->buckets) add(b.d_order, sizeof(int32_t) * (size_t)b.n);
    return v;
}

static kamx_status copy_state(const std::vector<StateSpan> &spans, char *snap, bool save, hipStream_t s) {
    size_t off = 0;
    for (const StateSpan &sp : spans) {
        void *dst = save ? (void *)(snap + off) : sp.p;
        const void *src = save ? (const void *)sp.p : (const void *)(snap + off);
        HIP_TRY(hipMemcpyAsync(dst, src, sp.bytes, hipMemcpyDeviceToDevice, s));
        off += (sp.bytes + 255) & ~(size_t)255;
    }
    return KAMX_OK;
}

// trial_steps steps of bucket bi alone, in the model's dispatch (one chained
// launch, or single steps with contact generation when contacts are
// generated); the step counter advances as in kamx_step.
static kamx_status enqueue_bucket_trial(kamx_model m, int bi, int steps, hipStream_t s) {
    const Bucket &b = m->buckets[bi];
    StepArgs a = step_args(m);
    a.bucket_worlds = b.d_worlds;
    a.n_bucket_worlds = b.n;
    a.iterate_out = nullptr;  // trials leave the caller's iterate log alone
    const bool chain = chained(m);
    for (int k = 0; k < steps;) {
        const int n = chain ? steps - k : 1;
        if (m->box_bin && !m->box_fused) {
            hipError_t e = launch_box_bin(m->d_worlds, m->n_worlds, m->d_q, m->d_u, gen_half_dt(m), m->d_box_geom,
                                          m->bin_wx, m->bin_wy, m->bin_margin, m->d_gen, m->d_gen_count, s);
            if (e != hipSuccess) return fail(KAMX_EDEVICE, "contact generation launch: %s", hipGetErrorString(e));
        }
        a.nsteps = n;
        hipError_t e = launch_step(a, b.mc, b.nt, b.n, s);
        if (e != hipSuccess) return fail(KAMX_EDEVICE, "step launch (bucket %d rows): %s", b.mc, hipGetErrorString(e));
        e = launch_advance_step(m->d_step, (uint32_t)n, s);
        if (e != hipSuccess) return fail(KAMX_EDEVICE, "counter launch: %s", hipGetErrorString(e));
        k += n;
    }
    return KAMX_OK;
}

kamx_status kamx_autotune(kamx_model m, int32_t trial_steps, float *ms_out) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (trial_steps < 1 || trial_steps > kChainSteps) return fail(KAMX_EINVAL, "trial_steps must be 1..%d", kChainSteps);
    if (m->params.warmstart == KAMX_WARM_LEARNED && !m->mlp)
        return fail(KAMX_ESTATE, "warm start LEARNED needs a network (kamx_model_attach_mlp)");
    K_TRY(check_device());
    if (m->params.log_restarts) K_TRY(ensure_rlog(m));
    const int nbk = (int)m->buckets.size();
    if (ms_out)
        for (int k = 0; k < 4 * nbk; ++k) ms_out[k] = 0.f;
    if (!m->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&m->capture_stream, hipStreamNonBlocking));
    hipStream_t s = m->capture_stream;
    HIP_TRY(hipDeviceSynchronize());
    const std::vector<StateSpan> spans = step_state(m);
    size_t total = 0;
    for (const StateSpan &sp : spans) total += (sp.bytes + 255) & ~(size_t)255;
    char *snap = nullptr;
    {
        hipError_t e = hipMalloc((void **)&snap, std::max<size_t>(total, 1));
        if (e != hipSuccess) return fail(KAMX_ENOMEM, "autotune snapshot (%zu bytes): %s", total, hipGetErrorString(e));
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    kamx_status st = KAMX_OK;
    auto run = [&]() -> kamx_status {
        HIP_TRY(hipEventCreate(&t0));
        HIP_TRY(hipEventCreate(&t1));
        K_TRY(copy_state(spans, snap, true, s));
        for (int bi = 0; bi < nbk; ++bi) {
            Bucket &b = m->buckets[bi];
            int nts[4];
            const int nv = step_threads_variants(b.mc, nts);
            if (nv < 2) continue;
            const int keep = b.nt;
            int best = keep;
            float best_ms = INFINITY;
            for (int v = 0; v < nv; ++v) {
                b.nt = nts[v];
                float ms = 0.f;
                for (int rep = 0; rep < 2; ++rep) {
                    K_TRY(copy_state(spans, snap, false, s));
                    HIP_TRY(hipEventRecord(t0, s));
                    kamx_status e = enqueue_bucket_trial(m, bi, trial_steps, s);
                    if (e != KAMX_OK) {
                        b.nt = keep;
                        return e;
                    }
                    HIP_TRY(hipEventRecord(t1, s));
                    HIP_TRY(hipEventSynchronize(t1));
                    HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
                }
                if (ms_out) ms_out[4 * bi + v] = ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = nts[v];
                }
            }
            b.nt = best;
        }
        return KAMX_OK;
    };
    st = run();
    // the state as it was before the call, whatever happened above
    kamx_status rs = copy_state(spans, snap, false, s);
    hipError_t se = hipStreamSynchronize(s);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipFree(snap);
    drop_graphs(m);
    if (st != KAMX_OK) return st;
    if (rs != KAMX_OK) return rs;
    if (se != hipSuccess) return fail(KAMX_EDEVICE, "autotune: %s", hipGetErrorString(se));
    return KAMX_OK;
}

kamx_status kamx_set_iteration_log(kamx_model m, int32_t *iters_dev, int32_t *rows_dev, int32_t *status_dev,
                                   int32_t steps) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (iters_dev && steps < 1) return fail(KAMX_EINVAL, "steps must be positive");
    drop_graphs(m);
    m->iter_log = iters_dev;
    m->row_log = iters_dev ? rows_dev : nullptr;
    m->status_log = iters_dev ? status_dev : nullptr;
    m->iter_log_rows = iters_dev ? steps : 0;
    return KAMX_OK;
}

kamx_status kamx_forward_kinematics(kamx_model m, const float *targets_dev, int32_t max_iters, float tol,
                                    int32_t *iters_dev, float *resid_dev, kamx_stream stream) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (!targets_dev) return fail(KAMX_EINVAL, "targets_dev is NULL");
    if (max_iters < 0 || max_iters > 10000) return fail(KAMX_EINVAL, "max_iters must be in [0, 10000]");
    if (!(tol >= 0.f)) return fail(KAMX_EINVAL, "tol must be >= 0");
    if (m->max_nb > kMaxBodies || m->max_nj > kMaxJoints)
        return fail(KAMX_EUNSUPPORTED, "forward kinematics supports worlds of at most %d bodies and %d joints",
                    kMaxBodies, kMaxJoints);
    K_TRY(check_device());
    hipError_t e = launch_fk(m->d_worlds, m->n_worlds, m->d_jint, m->d_jf, m->d_mass, m->d_inertia, m->d_q, m->d_u,
                             targets_dev, max_iters, tol, iters_dev, resid_dev, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(KAMX_EDEVICE, "forward kinematics launch: %s", hipGetErrorString(e));
    return KAMX_OK;
}

kamx_status kamx_set_iterate_log(kamx_model m, float *iterate_dev) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (iterate_dev && (reinterpret_cast<uintptr_t>(iterate_dev) & 15))
        return fail(KAMX_EINVAL, "iterate_dev must be 16-byte aligned");
    drop_graphs(m);
    m->iterate_log = iterate_dev;
    return KAMX_OK;
}

kamx_status kamx_model_feature_dims(kamx_model m, int32_t *n_features, int32_t *n_slots) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (m->has_sparse) return fail(KAMX_EUNSUPPORTED, "matrix-free worlds have no learned warm start");
    if (!m->uniform) return fail(KAMX_EUNSUPPORTED, "worlds differ in structure: no common feature layout");
    if (n_features) *n_features = m->n_feat;
    if (n_slots) *n_slots = m->n_slots;
    return KAMX_OK;
}

kamx_status kamx_model_features(kamx_model m, float *x_dev, kamx_stream stream) {
    if (!m || !x_dev) return fail(KAMX_EINVAL, "NULL argument");
    if (m->has_sparse) return fail(KAMX_EUNSUPPORTED, "matrix-free worlds have no learned warm start");
    if (!m->uniform) return fail(KAMX_EUNSUPPORTED, "worlds differ in structure: no common feature layout");
    K_TRY(check_device());
    return enqueue_features(m, x_dev, reinterpret_cast<hipStream_t>(stream));
}

kamx_status kamx_read_impulse_slots(kamx_model m, float *y_dev, kamx_stream stream) {
    if (!m || !y_dev) return fail(KAMX_EINVAL, "NULL argument");
    if (m->has_sparse) return fail(KAMX_EUNSUPPORTED, "matrix-free worlds have no learned warm start");
    if (!m->uniform) return fail(KAMX_EUNSUPPORTED, "worlds differ in structure: no common slot layout");
    K_TRY(check_device());
    hipError_t e = launch_impulse_slots(m->d_worlds, m->n_worlds, m->n_contact_slots, m->n_slots, m->d_lambda,
                                        m->d_keys, m->d_ncontacts, y_dev, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(KAMX_EDEVICE, "slot launch: %s", hipGetErrorString(e));
    return KAMX_OK;
}

kamx_status kamx_model_attach_mlp(kamx_model m, kamx_mlp net) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    drop_graphs(m);
    if (!net) {
        m->mlp = nullptr;
        return KAMX_OK;
    }
    if (m->has_sparse) return fail(KAMX_EUNSUPPORTED, "matrix-free worlds have no learned warm start");
    if (!m->uniform) return fail(KAMX_EUNSUPPORTED, "worlds differ in structure: no common feature layout");
    if (mlp_n_in(net) != m->n_feat || mlp_n_out(net) != m->n_slots)
        return fail(KAMX_EINVAL, "network is %d -> %d, the model needs %d -> %d", mlp_n_in(net), mlp_n_out(net),
                    m->n_feat, m->n_slots);
    if (mlp_capacity(net) < m->n_worlds)
        return fail(KAMX_EINVAL, "network batch capacity %d below %d worlds", mlp_capacity(net), m->n_worlds);
    {
        // the step kernel evaluates the network with its activations (BF16:
        // input, two hidden layers) in the LDS region of the Delassus triangle
        const MlpView v = mlp_view(net);
        for (const Bucket &b : m->buckets)
            if (2 * (size_t)(v.fp + 2 * v.H) > sizeof(float) * (size_t)tri_row_offset(b.mc))
                return fail(KAMX_EUNSUPPORTED, "network activations (%d + 2 x %d) exceed the %d-row bucket's LDS", v.fp,
                            v.H, b.mc);
    }
    if (!m->d_ws) K_TRY(dalloc(m, &m->d_ws, (size_t)m->n_worlds * m->n_slots));
    m->mlp = net;
    return KAMX_OK;
}

kamx_status kamx_contacts_box_bin(kamx_model m, const kamx_box_desc *boxes, float half_x, float half_y,
                                  float margin) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (m->mlp) return fail(KAMX_ESTATE, "set up box contacts before attaching a network (the slot layout changes)");
    drop_graphs(m);
    if (!boxes) {
        m->box_bin = false;
        m->n_contact_slots = m->contact_cap0;
        m->n_slots = m->n_slots_joint + 3 * m->n_contact_slots;
        m->n_feat = m->n_feat_body + m->n_slots + m->n_feat_joint;
        return KAMX_OK;
    }
    if (!(half_x > 0.f) || !(half_y > 0.f) || !(margin >= 0.f))
        return fail(KAMX_EINVAL, "bin half widths must be positive and margin >= 0");
    if (m->max_contacts < 1) return fail(KAMX_EINVAL, "the model has no contact capacity (max_contacts_per_world)");
    std::vector<float> geom(4 * (size_t)m->nb);
    std::vector<int> per_world(m->n_worlds, 0);
    std::vector<WorldInfo> wi(m->n_worlds);
    HIP_TRY(hipMemcpy(wi.data(), m->d_worlds, sizeof(WorldInfo) * m->n_worlds, hipMemcpyDeviceToHost));
    for (int w = 0; w < m->n_worlds; ++w)
        for (int b = wi[w].b0; b < wi[w].b0 + wi[w].nb; ++b) {
            const kamx_box_desc &d = boxes[b];
            bool is_box = d.half[0] > 0.f || d.half[1] > 0.f || d.half[2] > 0.f;
            if (is_box && !(d.half[0] > 0.f && d.half[1] > 0.f && d.half[2] > 0.f && d.mu >= 0.f))
                return fail(KAMX_EINVAL, "body %d: box half extents must all be positive and mu >= 0", b);
            for (int e = 0; e < 3; ++e) geom[4 * b + e] = is_box ? d.half[e] : 0.f;
            geom[4 * b + 3] = is_box ? d.mu : 0.f;
            per_world[w] += is_box;
        }
    const int cap = box_bin_max_boxes();
    for (int w = 0; w < m->n_worlds; ++w)
        if (per_world[w] > cap) return fail(KAMX_EINVAL, "world %d: %d boxes (at most %d)", w, per_world[w], cap);
    if (!m->d_box_geom) {
        K_TRY(dalloc(m, &m->d_box_geom, 4 * (size_t)m->nb));
        K_TRY(dalloc(m, &m->d_gen, (size_t)m->n_worlds * kMaxContacts));
        K_TRY(dalloc(m, &m->d_gen_count, (size_t)m->n_worlds));
    }
    HIP_TRY(hipMemcpy(m->d_box_geom, geom.data(), sizeof(float) * geom.size(), hipMemcpyHostToDevice));
    int most = 0;
    for (int w = 0; w < m->n_worlds; ++w) most = std::max(most, per_world[w]);
    // learned warm start: a slot per box vertex (contact_slot of a box key)
    m->n_contact_slots = 8 * most;
    m->n_slots = m->n_slots_joint + 3 * m->n_contact_slots;
    m->n_feat = m->n_feat_body + m->n_slots + m->n_feat_joint;
    m->bin_wx = half_x;
    m->bin_wy = half_y;
    m->bin_margin = margin;
    m->box_bin = true;
    m->box_fused = true;
    for (const Bucket &b : m->buckets) m->box_fused = m->box_fused && step_generates_box_contacts(b.mc);
    return KAMX_OK;
}

kamx_status kamx_set_schedule(kamx_model m, int32_t mode) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    if (mode != KAMX_SCHED_INDEX && mode != KAMX_SCHED_LPT && mode != KAMX_SCHED_CHAIN)
        return fail(KAMX_EINVAL, "unknown schedule mode %d", mode);
    if (m->schedule != mode) drop_graphs(m);
    m->schedule = mode;
    return KAMX_OK;
}

kamx_status kamx_read_impulses(kamx_model m, float *lambda_dev, kamx_stream stream) {
    if (!m || !lambda_dev) return fail(KAMX_EINVAL, "NULL argument");
    K_TRY(check_device());
    HIP_TRY(hipMemcpyAsync(lambda_dev, m->d_lambda, sizeof(float) * m->rows_cap, hipMemcpyDeviceToDevice,
                           reinterpret_cast<hipStream_t>(stream)));
    return KAMX_OK;
}

kamx_status kamx_read_stats(kamx_model m, int32_t *iters_dev, float *resid_dev, int32_t *status_dev, int32_t *rows_dev,
                            kamx_stream stream) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    K_TRY(check_device());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int n = m->n_worlds;
    if (iters_dev) HIP_TRY(hipMemcpyAsync(iters_dev, m->d_iters, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    if (resid_dev) HIP_TRY(hipMemcpyAsync(resid_dev, m->d_resid, sizeof(float) * 4 * n, hipMemcpyDeviceToDevice, s));
    if (status_dev) HIP_TRY(hipMemcpyAsync(status_dev, m->d_status, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    if (rows_dev) HIP_TRY(hipMemcpyAsync(rows_dev, m->d_rows, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    return KAMX_OK;
}

kamx_status kamx_read_restart_log(kamx_model m, uint8_t *log_dev, kamx_stream stream) {
    if (!m || !log_dev) return fail(KAMX_EINVAL, "NULL argument");
    if (!m->d_rlog) return fail(KAMX_ESTATE, "restart logging was not enabled (params.log_restarts)");
    K_TRY(check_device());
    HIP_TRY(hipMemcpyAsync(log_dev, m->d_rlog, (size_t)m->n_worlds * m->rlog_stride, hipMemcpyDeviceToDevice,
                           reinterpret_cast<hipStream_t>(stream)));
    return KAMX_OK;
}

kamx_status kamx_read_torques(kamx_model m, float *torque_dev, kamx_stream stream) {
    if (!m || !torque_dev) return fail(KAMX_EINVAL, "NULL argument");
    K_TRY(check_device());
    if (m->nj > 0)
        HIP_TRY(hipMemcpyAsync(torque_dev, m->d_tau, sizeof(float) * m->nj, hipMemcpyDeviceToDevice,
                               reinterpret_cast<hipStream_t>(stream)));
    return KAMX_OK;
}

kamx_status kamx_read_contacts(kamx_model m, kamx_contact *contacts_dev, int32_t *counts_dev, kamx_stream stream) {
    if (!m) return fail(KAMX_EINVAL, "model is NULL");
    K_TRY(check_device());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (contacts_dev)
        HIP_TRY(hipMemcpyAsync(contacts_dev, m->d_contacts_out, sizeof(kamx_contact) * m->n_worlds * kMaxContacts,
                               hipMemcpyDeviceToDevice, s));
    if (counts_dev)
        HIP_TRY(hipMemcpyAsync(counts_dev, m->d_ncontacts, sizeof(int32_t) * m->n_worlds, hipMemcpyDeviceToDevice, s));
    return KAMX_OK;
}

kamx_status kamx_read_phase_clock(kamx_model m, uint64_t *clk_dev, kamx_stream stream) {
    if (!m || !clk_dev) return fail(KAMX_EINVAL, "NULL argument");
    if (!m->d_phase_clk) return fail(KAMX_ESTATE, "phase clock not enabled (set KAMX_PHASE_CLOCK before model create)");
    HIP_TRY(hipMemcpyAsync(clk_dev, m->d_phase_clk, sizeof(uint64_t) * 16 * m->n_worlds, hipMemcpyDeviceToDevice,
                           reinterpret_cast<hipStream_t>(stream)));
    return KAMX_OK;
}

kamx_status kamx_reset_count(kamx_model m, int64_t *count, kamx_stream stream) {
    if (!m || !count) return fail(KAMX_EINVAL, "NULL argument");
    K_TRY(check_device());
    std::vector<int32_t> h(m->n_worlds);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(h.data(), m->d_reset_count, sizeof(int32_t) * m->n_worlds, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t c = 0;
    for (int32_t v : h) c += v;
    *count = c;
    return KAMX_OK;
}

}  // extern "C"
