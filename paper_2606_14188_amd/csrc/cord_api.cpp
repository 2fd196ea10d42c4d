// Host side of the libcord C ABI: validation, size classes, offsets,
// workspaces, launch modes (grouped / per instance / persistent / hipGraph)
// and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/cord.h"
#include "cord_internal.h"
#include "cord_host.h"
#include "cord_kernels.h"

using namespace cord;

namespace cord {
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
}

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define CORD_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(CORD_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

namespace cord {
// size classes: upper node counts per topology
const int kRopeBuckets[] = {32, 64, 128, 256};
const int kClothBuckets[] = {64, 128, 256, 512, 1024, 2304};

// Dense A_t/B_t of rope classes go to the banded direct kernel; JVPs, cloth,
// B_t alone, penalty grasps, friction and classes it does not cover use the class's
// iterative kernel.
// Setting CORD_LINEARIZE_ITERATIVE=1 in the environment forces the iterative
// kernel everywhere (for comparisons).
namespace {
bool use_iterative_only() {
    static const bool it = [] {
        const char* e = std::getenv("CORD_LINEARIZE_ITERATIVE");
        return e && e[0] == '1';
    }();
    return it;
}
}  // namespace

hipError_t launch_linearize(int cfg_index, int topo, int nmax, bool penalty, bool fric, const KArgs& a, int nblk,
                            int tmax, hipStream_t st, const KeptSource& ks) {
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    const auto lin = fric ? cfg[cfg_index].linearize_f : cfg[cfg_index].linearize;
    int wg = 0;
    const size_t kf = (a.A && topo == kRope && !penalty && !fric && !use_iterative_only())
                          ? linearize_rope_direct_scratch(nmax, &wg) : 0;
    if (wg > 0) {
        KArgs ad = a;
        ad.jvp_k = 0; ad.jvp_ds = nullptr; ad.jvp_du = nullptr; ad.jvp_out = nullptr;
        // null: vectors kept inside A (also forced by CORD_LINEARIZE_NO_SCRATCH=1)
        const char* ns = std::getenv("CORD_LINEARIZE_NO_SCRATCH");
        ad.kept = (ns && ns[0] == '1') ? nullptr : ks.get(ks.ctx, kf);
        ad.kept_tg = wg;
        hipError_t e = linearize_rope_direct(nmax, ad, nblk, tmax, st);
        if (e != hipSuccess) return e;
        if (a.redo) {
            // steps whose band factors met a non-positive pivot (an
            // indefinite dF/dq*, e.g. a compressed rope) are done again by
            // the iterative kernel, whose solves fall back to MINRES; the
            // other workgroups of this launch return at once
            KArgs ar = a;
            ar.jvp_k = 0; ar.jvp_ds = nullptr; ar.jvp_du = nullptr; ar.jvp_out = nullptr;
            e = lin(ar, nblk, tmax, st);
            if (e != hipSuccess) return e;
        }
        if (!a.jvp_out) return hipSuccess;
        KArgs aj = a;
        aj.A = nullptr; aj.Bm = nullptr; aj.redo = nullptr;
        return lin(aj, nblk, tmax, st);
    }
    KArgs ai = a;
    ai.redo = nullptr;
    return lin(ai, nblk, tmax, st);
}

int bucket_of(int topo, int n) {
    const int* b = topo == kRope ? kRopeBuckets : kClothBuckets;
    const int nb = topo == kRope ? 4 : 6;
    for (int i = 0; i < nb; ++i)
        if (n <= b[i]) return b[i];
    return -1;
}
}  // namespace cord

namespace {

struct Group {
    int topo = 0;
    int nmax = 0;              // bucket upper bound
    int cfg = -1;
    std::vector<int32_t> ids;  // longest (n T) first
    int32_t* d_ids = nullptr;
    int tmax = 0;
    int cap[2] = {1, 1};       // persistent grid: resident workgroups (rollout, backward)
    bool penalty = false;      // some instance uses the penalty grasp
    bool fric = false;         // some instance has friction (mu > 0): the friction kernels
};

enum Op { kOpRollout = 0, kOpBackward = 1 };

}  // namespace

struct cord_sim {
    int device = 0;
    int n_cu = 1;
    int launch = CORD_LAUNCH_GROUPED;
    std::vector<cord_instance_desc> desc;
    std::vector<InstDev> h;
    InstDev* d_inst = nullptr;
    int32_t* d_ident = nullptr;      // 0..B-1 (per-instance launches)
    std::vector<Group> groups;
    std::vector<int> group_of;       // instance -> group
    cord_sim_info_t info{};
    std::map<int, std::vector<int64_t>> ckpt_host;   // K -> offsets (n_inst + 1)
    std::map<int, int64_t*> ckpt_dev;
    float* seg = nullptr;            // backward segment workspace
    size_t seg_floats = 0;
    int seg_K = 0;
    int64_t* seg_off = nullptr;
    int32_t* d_queues = nullptr;     // one work-queue counter per group
    int32_t* d_redo = nullptr;       // per (instance, step) flags of the direct linearization
    float* cp_pred = nullptr;        // one-step predictions of cord_cp_scores (s_floats)
    uint32_t* lin_stats = nullptr;   // direct linearization counters (scratch-slot overlaps, steps redone)
    void* noalloc = nullptr;         // this device's static scratch (cord_rollout_backward_noalloc)
    hipError_t noalloc_err = hipSuccess;
    int64_t n_steps = 0;             // sum T
    std::vector<hipStream_t> streams;
    hipStream_t cap_stream = nullptr;   // graph capture (the caller's stream may be the null stream)
    hipEvent_t fork_ev = nullptr;
    std::vector<hipEvent_t> join_ev;
    std::map<std::vector<uintptr_t>, hipGraphExec_t> graphs;
    std::vector<std::vector<uintptr_t>> graph_order;
    float* aux = nullptr;               // step internals (cord_sim_set_aux), caller-owned
    float* kept = nullptr;              // direct rope linearization scratch
    size_t kept_floats = 0;
};

namespace cord {

int validate(const cord_instance_desc& d, int i) {
    const cord_params& p = d.params;
    if (d.kind != CORD_ROPE && d.kind != CORD_CLOTH) return fail(CORD_EINVAL, "instance %d: bad kind %d", i, d.kind);
    if (d.kind == CORD_ROPE && (d.ny != 1 || d.nx < 1)) return fail(CORD_EINVAL, "instance %d: rope needs nx >= 1, ny == 1", i);
    if (d.kind == CORD_CLOTH && (d.nx < 2 || d.ny < 2)) return fail(CORD_EINVAL, "instance %d: cloth needs nx, ny >= 2", i);
    if (d.T < 1) return fail(CORD_EINVAL, "instance %d: T must be >= 1", i);
    if (!(p.dt > 0.f) || !std::isfinite(p.dt)) return fail(CORD_EINVAL, "instance %d: dt must be > 0", i);
    if (!(p.gamma >= 0.f && p.gamma <= 1.f)) return fail(CORD_EINVAL, "instance %d: gamma must be in [0,1]", i);
    if (!(p.kappa_fwd >= 0.f) || !(p.kappa_bwd > 0.f)) return fail(CORD_EINVAL, "instance %d: need kappa_fwd >= 0, kappa_bwd > 0", i);
    if (!(d.mass > 0.f) || !(d.h > 0.f)) return fail(CORD_EINVAL, "instance %d: mass and h must be > 0", i);
    if (!(d.k_struct >= 0.f) || !(d.k_shear >= 0.f) || !(d.k_bend >= 0.f)) return fail(CORD_EINVAL, "instance %d: negative stiffness", i);
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(p.gravity[c])) return fail(CORD_EINVAL, "instance %d: gravity not finite", i);
    if (!(p.mu >= 0.f) || !std::isfinite(p.mu)) return fail(CORD_EINVAL, "instance %d: friction mu must be >= 0", i);
    if (p.mu > 0.f && !(p.kappa_fwd > 0.f))
        return fail(CORD_EUNSUPPORTED, "instance %d: friction (mu > 0) needs smoothed forward contact (kappa_fwd > 0)", i);
    const int n = d.nx * d.ny;
    if (d.n_grip < 0 || d.n_grip > CORD_MAX_GRIP) return fail(CORD_EINVAL, "instance %d: n_grip out of range", i);
    for (int g = 0; g < d.n_grip; ++g) {
        if (d.grip_node[g] < 0 || d.grip_node[g] >= n) return fail(CORD_EINVAL, "instance %d: grip node out of range", i);
        for (int g2 = 0; g2 < g; ++g2)
            if (d.grip_node[g2] == d.grip_node[g]) return fail(CORD_EINVAL, "instance %d: duplicate grip node", i);
    }
    if (d.n_sphere < 0 || d.n_sphere > CORD_MAX_SPHERE || d.n_box < 0 || d.n_box > CORD_MAX_BOX)
        return fail(CORD_EINVAL, "instance %d: obstacle count out of range", i);
    for (int s = 0; s < d.n_sphere; ++s)
        if (!(d.sphere[s][3] > 0.f)) return fail(CORD_EINVAL, "instance %d: sphere radius must be > 0", i);
    for (int b = 0; b < d.n_box; ++b) {
        const float* bx = d.box[b];
        const float mh = fminf(bx[3], fminf(bx[4], bx[5]));
        if (!(bx[6] >= 0.f) || !(bx[6] < mh)) return fail(CORD_EINVAL, "instance %d: box rounding must be in [0, min half extent)", i);
    }
    const int nobs = (d.ground ? 1 : 0) + d.n_sphere + d.n_box;
    if (nobs > CORD_MAX_OBST) return fail(CORD_EUNSUPPORTED, "instance %d: %d obstacles > %d", i, nobs, CORD_MAX_OBST);
    if (d.grip_mode != CORD_GRIP_DIRICHLET && d.grip_mode != CORD_GRIP_PENALTY)
        return fail(CORD_EINVAL, "instance %d: unknown grip_mode %d", i, d.grip_mode);
    if (d.grip_mode == CORD_GRIP_PENALTY) {
        if (!(d.D_max > 0.f) || !std::isfinite(d.D_max)) return fail(CORD_EINVAL, "instance %d: penalty grasp needs D_max > 0", i);
        if (!(d.kappa_h >= 0.f) || !std::isfinite(d.kappa_h)) return fail(CORD_EINVAL, "instance %d: kappa_h must be >= 0", i);
        if (d.kappa_h == 0.f && !(d.r_g > 0.f)) return fail(CORD_EINVAL, "instance %d: hard activation needs r_g > 0", i);
    }
    if (bucket_of(d.kind == CORD_ROPE ? kRope : kCloth, n) < 0)
        return fail(CORD_EUNSUPPORTED, "instance %d: %d nodes exceed every kernel configuration", i, n);
    return CORD_OK;
}

// Device descriptor of one instance (offsets are set by the caller).
void fill_instdev(const cord_instance_desc& d, InstDev& I) {
    std::memset(&I, 0, sizeof(I));
    I.kind = d.kind == CORD_ROPE ? kRope : kCloth;
    I.nx = d.nx; I.ny = d.ny; I.n = d.nx * d.ny;
    I.T = d.T; I.n_grip = d.n_grip;
    I.grip_mode = d.grip_mode == CORD_GRIP_PENALTY ? 1 : 0;
    I.n_s = 6 * I.n + (I.grip_mode ? 3 * d.n_grip : 0); I.n_u = 3 * d.n_grip;
    I.D_max = d.D_max; I.kappa_h = d.kappa_h; I.r_g = d.r_g;
    I.mu = d.params.mu;
    for (int g = 0; g < d.n_grip; ++g) I.grip_node[g] = d.grip_node[g];
    int o = 0;
    if (d.ground) { I.obs_type[o] = kObsGround; ++o; }
    for (int k = 0; k < d.n_sphere; ++k, ++o) {
        I.obs_type[o] = kObsSphere;
        for (int c = 0; c < 4; ++c) I.obs[o][c] = d.sphere[k][c];
    }
    for (int k = 0; k < d.n_box; ++k, ++o) {
        I.obs_type[o] = kObsBox;
        for (int c = 0; c < 7; ++c) I.obs[o][c] = d.box[k][c];
    }
    I.n_obs = o;
    I.h = d.h; I.mass = d.mass; I.k_struct = d.k_struct; I.k_shear = d.k_shear; I.k_bend = d.k_bend;
    I.dt = d.params.dt; I.gamma = d.params.gamma;
    I.kappa_fwd = d.params.kappa_fwd; I.kappa_bwd = d.params.kappa_bwd;
    I.g0 = d.params.gravity[0]; I.g1 = d.params.gravity[1]; I.g2 = d.params.gravity[2];
}

// first table entry of this topology covering nmax nodes
int default_config(int topo, int nmax) {
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    for (int c = 0; c < count; ++c)
        if (cfg[c].topo == topo && cfg[c].nt * cfg[c].ppt >= nmax) return c;
    return -1;
}

int find_config(int topo, int nt, int ppt) {
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    for (int c = 0; c < count; ++c)
        if (cfg[c].topo == topo && cfg[c].nt == nt && cfg[c].ppt == ppt) return c;
    return -1;
}

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

}  // namespace cord

namespace {

void drop_graphs(cord_sim* s) {
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    s->graphs.clear();
    s->graph_order.clear();
}

int upload_group(cord_sim* s, Group& g) {
    if (g.d_ids) { (void)hipFree(g.d_ids); g.d_ids = nullptr; }
    CORD_HIP(hipMalloc(&g.d_ids, sizeof(int32_t) * g.ids.size()));
    CORD_HIP(hipMemcpy(g.d_ids, g.ids.data(), sizeof(int32_t) * g.ids.size(), hipMemcpyHostToDevice));
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    for (int w = 0; w < 2; ++w) {
        const int c = cfg[g.cfg].blocks_per_cu(w) * s->n_cu;
        g.cap[w] = std::max(1, std::min((int)g.ids.size(), c));
    }
    return CORD_OK;
}

int ensure_ckpt(cord_sim* s, int K) {
    if (s->ckpt_dev.count(K)) return CORD_OK;
    const int B = (int)s->h.size();
    std::vector<int64_t> off(B + 1, 0);
    for (int b = 0; b < B; ++b) {
        const InstDev& I = s->h[b];
        off[b + 1] = off[b] + (int64_t)((I.T + K - 1) / K + 1) * I.n_s;
    }
    int64_t* d = nullptr;
    CORD_HIP(hipMalloc(&d, sizeof(int64_t) * B));
    CORD_HIP(hipMemcpy(d, off.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice));
    s->ckpt_host[K] = off;
    s->ckpt_dev[K] = d;
    return CORD_OK;
}

int ensure_seg(cord_sim* s, int K) {
    if (s->seg && s->seg_K == K) return CORD_OK;
    const int B = (int)s->h.size();
    std::vector<int64_t> off(B + 1, 0);
    for (int b = 0; b < B; ++b) off[b + 1] = off[b] + (int64_t)K * s->h[b].n_s;
    drop_graphs(s);
    if (s->seg) { (void)hipFree(s->seg); s->seg = nullptr; }
    if (s->seg_off) { (void)hipFree(s->seg_off); s->seg_off = nullptr; }
    if (hipMalloc(&s->seg, sizeof(float) * (size_t)off[B]) != hipSuccess)
        return fail(CORD_ENOMEM, "backward workspace of %lld floats", (long long)off[B]);
    CORD_HIP(hipMalloc(&s->seg_off, sizeof(int64_t) * B));
    CORD_HIP(hipMemcpy(s->seg_off, off.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice));
    s->seg_floats = (size_t)off[B];
    s->seg_K = K;
    return CORD_OK;
}

// Scratch table of the direct rope linearization, grown on demand (hipFree
// waits for work still using the old buffer); null if it cannot be had.
float* sim_kept(void* ctx, size_t floats) {
    cord_sim* s = static_cast<cord_sim*>(ctx);
    if (floats > s->kept_floats) {
        if (s->kept) { (void)hipFree(s->kept); s->kept = nullptr; s->kept_floats = 0; }
        if (hipMalloc(&s->kept, sizeof(float) * floats) != hipSuccess) {
            (void)hipGetLastError();   // run without the scratch
            s->kept = nullptr;
            return nullptr;
        }
        // the guard words after the slots start at zero (every use of a
        // slot returns its busy count to zero; the start counts only grow)
        if (hipMemset(s->kept, 0, sizeof(float) * floats) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(s->kept);
            s->kept = nullptr;
            return nullptr;
        }
        s->kept_floats = floats;
    }
    return s->kept;
}

int ensure_streams(cord_sim* s) {
    const size_t ng = s->groups.size();
    if (!s->fork_ev) CORD_HIP(hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming));
    if (!s->cap_stream) CORD_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    while (s->streams.size() < ng) {
        hipStream_t st;
        CORD_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));   // default priority
        s->streams.push_back(st);
        hipEvent_t ev;
        CORD_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        s->join_ev.push_back(ev);
    }
    if (!s->d_queues) CORD_HIP(hipMalloc(&s->d_queues, sizeof(int32_t) * std::max<size_t>(ng, 1) + 64));
    return CORD_OK;
}

KArgs base_args(const cord_sim* s) {
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.inst = s->d_inst;
    return a;
}

hipError_t launch_op(const KernelCfg& c, int op, const KArgs& a, int nblk, hipStream_t st, bool fric) {
    if (fric) return op == kOpRollout ? c.rollout_f(a, nblk, st) : c.backward_f(a, nblk, st);
    return op == kOpRollout ? c.rollout(a, nblk, st) : c.backward(a, nblk, st);
}

// Enqueue the persistent multi-stream sequence on `st` (capturable: the
// queue counters are cleared by a kernel, not a memset).
int enqueue_persistent(cord_sim* s, int op, KArgs a, hipStream_t st) {
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    const int ng = (int)s->groups.size();
    CORD_HIP(launch_fill_i32(s->d_queues, ng, 0, st));
    CORD_HIP(hipEventRecord(s->fork_ev, st));
    for (int g = 0; g < ng; ++g) {
        Group& G = s->groups[g];
        hipStream_t sg = s->streams[g];
        CORD_HIP(hipStreamWaitEvent(sg, s->fork_ev, 0));
        a.ids = G.d_ids;
        a.n_ids = (int)G.ids.size();
        a.queue = s->d_queues + g;
        CORD_HIP(launch_op(cfg[G.cfg], op, a, G.cap[op], sg, G.fric));
        CORD_HIP(hipEventRecord(s->join_ev[g], sg));
        CORD_HIP(hipStreamWaitEvent(st, s->join_ev[g], 0));
    }
    return CORD_OK;
}

std::vector<uintptr_t> graph_key(int op, const KArgs& a) {
    return {(uintptr_t)op, (uintptr_t)a.s0, (uintptr_t)a.u, (uintptr_t)a.traj, (uintptr_t)a.final_out,
            (uintptr_t)a.traj_in, (uintptr_t)a.traj_bar, (uintptr_t)a.sT_bar, (uintptr_t)a.s0_bar,
            (uintptr_t)a.u_bar, (uintptr_t)a.status, (uintptr_t)a.counters, (uintptr_t)a.store,
            (uintptr_t)a.ckpt_every, (uintptr_t)a.use_kappa_bwd, (uintptr_t)a.seg, (uintptr_t)a.aux,
            (uintptr_t)a.aux_mode};
}

int launch_all(cord_sim* s, int op, KArgs a, hipStream_t st) {
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    switch (s->launch) {
        case CORD_LAUNCH_PER_INSTANCE: {
            for (int i = 0; i < (int)s->h.size(); ++i) {
                a.ids = s->d_ident + i;
                a.n_ids = 1;
                a.queue = nullptr;
                const Group& Gi = s->groups[s->group_of[i]];
                CORD_HIP(launch_op(cfg[Gi.cfg], op, a, 1, st, Gi.fric));
            }
            return CORD_OK;
        }
        case CORD_LAUNCH_PERSISTENT: {
            int rc = ensure_streams(s);
            if (rc) return rc;
            return enqueue_persistent(s, op, a, st);
        }
        case CORD_LAUNCH_GRAPH: {
            int rc = ensure_streams(s);
            if (rc) return rc;
            auto key = graph_key(op, a);
            auto it = s->graphs.find(key);
            if (it == s->graphs.end()) {
                hipGraph_t graph = nullptr;
                hipStream_t cs = s->cap_stream;
                CORD_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                rc = enqueue_persistent(s, op, a, cs);
                hipError_t e = hipStreamEndCapture(cs, &graph);
                if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
                if (e != hipSuccess) return fail(CORD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
                hipGraphExec_t ex = nullptr;
                e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) return fail(CORD_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
                if (s->graph_order.size() >= 16) {
                    auto old = s->graph_order.front();
                    s->graph_order.erase(s->graph_order.begin());
                    (void)hipGraphExecDestroy(s->graphs[old]);
                    s->graphs.erase(old);
                }
                it = s->graphs.emplace(key, ex).first;
                s->graph_order.push_back(key);
            }
            CORD_HIP(hipGraphLaunch(it->second, st));
            return CORD_OK;
        }
        default: {
            for (const Group& G : s->groups) {
                a.ids = G.d_ids;
                a.n_ids = (int)G.ids.size();
                a.queue = nullptr;
                CORD_HIP(launch_op(cfg[G.cfg], op, a, a.n_ids, st, G.fric));
            }
            return CORD_OK;
        }
    }
}

// ---- tiny JSON cache: {"entries": [[topo, nmax, nt, ppt], ...]}
std::vector<std::vector<int>> read_cache(const char* path) {
    std::vector<std::vector<int>> out;
    if (!path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    std::string t = ss.str();
    size_t p = t.find("\"entries\"");
    if (p == std::string::npos) return out;
    p = t.find('[', p);
    if (p == std::string::npos) return out;
    ++p;
    while (true) {
        size_t a = t.find('[', p), e = t.find(']', p);
        if (a == std::string::npos || e == std::string::npos || e < a) break;
        size_t b = t.find(']', a);
        std::string inner = t.substr(a + 1, b - a - 1);
        std::vector<int> v;
        std::stringstream is(inner);
        std::string tok;
        while (std::getline(is, tok, ',')) v.push_back(std::atoi(tok.c_str()));
        if (v.size() == 4) out.push_back(v);
        p = b + 1;
    }
    return out;
}

bool write_cache(const char* path, const std::vector<std::vector<int>>& e) {
    if (!path) return true;
    std::ofstream f(path);
    if (!f) return false;
    f << "{\"format\": \"topo, nmax, threads, particles_per_thread\", \"entries\": [";
    for (size_t i = 0; i < e.size(); ++i)
        f << (i ? ", " : "") << "[" << e[i][0] << ", " << e[i][1] << ", " << e[i][2] << ", " << e[i][3] << "]";
    f << "]}\n";
    return (bool)f;
}

}  // namespace

extern "C" {

const char* cord_last_error(void) { return g_err.c_str(); }

int cord_abi_sizes(int64_t* out, int32_t n) {
    if (!out) return fail(CORD_EINVAL, "cord_abi_sizes: NULL out");
    const int64_t sz[6] = {(int64_t)sizeof(cord_params), (int64_t)sizeof(cord_instance_desc),
                           (int64_t)sizeof(cord_sim_info_t), (int64_t)sizeof(cord_rollout_opts),
                           (int64_t)sizeof(cord_backward_opts), (int64_t)sizeof(cord_jvp)};
    for (int i = 0; i < n && i < 6; ++i) out[i] = sz[i];
    return CORD_OK;
}

int cord_sim_create(const cord_instance_desc* inst, int32_t n_inst, cord_sim** out) {
    g_err.clear();
    if (!inst || !out || n_inst < 1) return fail(CORD_EINVAL, "cord_sim_create: need inst, out and n_inst >= 1");
    for (int i = 0; i < n_inst; ++i) {
        int rc = validate(inst[i], i);
        if (rc) return rc;
    }
    cord_sim* s = new (std::nothrow) cord_sim();
    if (!s) return fail(CORD_ENOMEM, "host allocation");
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return fail(CORD_EHIP, "hipGetDevice failed"); }
    if (hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess) s->n_cu = 1;
    // the address of this device's copy of the no-alloc scratch, looked up
    // here with the device current (an error is reported by the entry point)
    s->noalloc_err = noalloc_scratch(s->device, &s->noalloc);
    if (s->noalloc_err != hipSuccess) (void)hipGetLastError();
    s->desc.assign(inst, inst + n_inst);
    s->h.resize(n_inst);
    s->group_of.assign(n_inst, -1);
    int64_t so = 0, uo = 0, to = 0, tns = 0, ao = 0, bo = 0, xo = 0, steps = 0;
    int max_n = 0, max_T = 0;
    std::map<std::pair<int, int>, int> class_group;
    for (int i = 0; i < n_inst; ++i) {
        const cord_instance_desc& d = inst[i];
        InstDev& I = s->h[i];
        fill_instdev(d, I);
        I.s_off = so; I.u_off = uo; I.traj_off = to; I.tns_off = tns; I.A_off = ao; I.B_off = bo;
        I.aux_off = xo;
        I.t_off = (int32_t)steps;
        steps += I.T;
        if (steps > INT32_MAX) {
            delete s;
            return fail(CORD_EUNSUPPORTED, "more than 2^31 - 1 steps in one batch");
        }
        xo += (int64_t)kAuxFields * I.T * I.n;
        so += I.n_s;
        uo += (int64_t)I.T * I.n_u;
        to += (int64_t)(I.T + 1) * I.n_s;
        tns += (int64_t)I.T * I.n_s;
        ao += (int64_t)I.T * I.n_s * I.n_s;
        bo += (int64_t)I.T * I.n_s * I.n_u;
        max_n = I.n > max_n ? I.n : max_n;
        max_T = I.T > max_T ? I.T : max_T;
        const int bkt = bucket_of(I.kind, I.n);
        auto key = std::make_pair((int)I.kind, bkt);
        if (!class_group.count(key)) {
            class_group[key] = (int)s->groups.size();
            Group G;
            G.topo = I.kind;
            G.nmax = bkt;
            G.cfg = default_config(I.kind, bkt);
            s->groups.push_back(G);
        }
        const int gi = class_group[key];
        s->groups[gi].ids.push_back(i);
        if (I.grip_mode) s->groups[gi].penalty = true;
        if (I.mu > 0.f) s->groups[gi].fric = true;
        s->groups[gi].tmax = std::max(s->groups[gi].tmax, I.T);
        s->group_of[i] = gi;
    }
    s->info.n_inst = n_inst;
    s->info.s_floats = so; s->info.u_floats = uo; s->info.traj_floats = to;
    s->info.A_floats = ao; s->info.B_floats = bo; s->info.aux_floats = xo;
    s->info.max_n = max_n; s->info.max_T = max_T;
    s->n_steps = steps;
    auto cleanup = [&](int code, const std::string& what) {
        cord_sim_destroy(s);
        return fail(code, "%s", what.c_str());
    };
    for (Group& G : s->groups)   // longest work first
        std::stable_sort(G.ids.begin(), G.ids.end(), [&](int a, int b) {
            return (int64_t)s->h[a].n * s->h[a].T > (int64_t)s->h[b].n * s->h[b].T;
        });
    if (hipMalloc(&s->d_inst, sizeof(InstDev) * n_inst) != hipSuccess) return cleanup(CORD_ENOMEM, "device instance table");
    if (hipMemcpy(s->d_inst, s->h.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(CORD_EHIP, "upload of instance table failed");
    std::vector<int32_t> ident(n_inst);
    for (int i = 0; i < n_inst; ++i) ident[i] = i;
    if (hipMalloc(&s->d_ident, sizeof(int32_t) * n_inst) != hipSuccess) return cleanup(CORD_ENOMEM, "device id table");
    if (hipMemcpy(s->d_ident, ident.data(), sizeof(int32_t) * n_inst, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(CORD_EHIP, "upload of id table failed");
    for (Group& G : s->groups)
        if (upload_group(s, G)) return cleanup(CORD_EHIP, g_err);
    *out = s;
    return CORD_OK;
}

int cord_sim_destroy(cord_sim* s) {
    if (!s) return CORD_OK;
    drop_graphs(s);
    if (s->d_inst) (void)hipFree(s->d_inst);
    if (s->d_ident) (void)hipFree(s->d_ident);
    for (Group& g : s->groups)
        if (g.d_ids) (void)hipFree(g.d_ids);
    for (auto& kv : s->ckpt_dev) (void)hipFree(kv.second);
    if (s->seg) (void)hipFree(s->seg);
    if (s->seg_off) (void)hipFree(s->seg_off);
    if (s->kept) (void)hipFree(s->kept);
    if (s->d_queues) (void)hipFree(s->d_queues);
    if (s->d_redo) (void)hipFree(s->d_redo);
    if (s->cp_pred) (void)hipFree(s->cp_pred);
    if (s->lin_stats) (void)hipFree(s->lin_stats);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    for (hipEvent_t ev : s->join_ev) (void)hipEventDestroy(ev);
    if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
    delete s;
    return CORD_OK;
}

int cord_sim_info(const cord_sim* s, cord_sim_info_t* out) {
    if (!s || !out) return fail(CORD_EINVAL, "cord_sim_info: NULL argument");
    *out = s->info;
    return CORD_OK;
}

int cord_sim_offsets(const cord_sim* s, int32_t K, int64_t* s_off, int64_t* u_off, int64_t* traj_off,
                     int64_t* ckpt_off, int64_t* A_off, int64_t* B_off) {
    if (!s) return fail(CORD_EINVAL, "cord_sim_offsets: NULL sim");
    if (ckpt_off && K < 1) return fail(CORD_EINVAL, "cord_sim_offsets: ckpt_every must be >= 1");
    const int B = (int)s->h.size();
    int64_t ck = 0;
    for (int b = 0; b <= B; ++b) {
        const bool last = b == B;
        const InstDev* I = last ? nullptr : &s->h[b];
        if (s_off) s_off[b] = last ? s->info.s_floats : I->s_off;
        if (u_off) u_off[b] = last ? s->info.u_floats : I->u_off;
        if (traj_off) traj_off[b] = last ? s->info.traj_floats : I->traj_off;
        if (A_off) A_off[b] = last ? s->info.A_floats : I->A_off;
        if (B_off) B_off[b] = last ? s->info.B_floats : I->B_off;
        if (ckpt_off) {
            ckpt_off[b] = ck;
            if (!last) ck += (int64_t)((I->T + K - 1) / K + 1) * I->n_s;
        }
    }
    return CORD_OK;
}

int cord_sim_set_launch(cord_sim* s, int32_t mode) {
    if (!s) return fail(CORD_EINVAL, "cord_sim_set_launch: NULL sim");
    if (mode < CORD_LAUNCH_GROUPED || mode > CORD_LAUNCH_GRAPH) return fail(CORD_EINVAL, "unknown launch mode %d", mode);
    if (mode != s->launch) drop_graphs(s);
    s->launch = mode;
    return CORD_OK;
}

int cord_sim_classes(const cord_sim* s, int32_t* topo, int32_t* nmax, int32_t* nt, int32_t* ppt, int32_t* n_inst,
                     int32_t cap, int32_t* count) {
    if (!s || !count) return fail(CORD_EINVAL, "cord_sim_classes: NULL argument");
    int c = 0;
    const KernelCfg* cfg = kernel_configs(&c);
    *count = (int32_t)s->groups.size();
    for (int g = 0; g < (int)s->groups.size() && g < cap; ++g) {
        const Group& G = s->groups[g];
        if (topo) topo[g] = G.topo == kRope ? CORD_ROPE : CORD_CLOTH;
        if (nmax) nmax[g] = G.nmax;
        if (nt) nt[g] = cfg[G.cfg].nt;
        if (ppt) ppt[g] = cfg[G.cfg].ppt;
        if (n_inst) n_inst[g] = (int32_t)G.ids.size();
    }
    return CORD_OK;
}

int cord_rollout(cord_sim* s, const float* s0, const float* u, float* traj, int32_t* inst_status,
                 const cord_rollout_opts* opts, void* stream) {
    g_err.clear();
    if (!s || !s0 || !traj) return fail(CORD_EINVAL, "cord_rollout: NULL sim, s0 or traj");
    if (!u && s->info.u_floats > 0) return fail(CORD_EINVAL, "cord_rollout: NULL u");
    cord_rollout_opts o{};
    o.store = CORD_STORE_FULL;
    if (opts) o = *opts;
    if (o.store != CORD_STORE_FULL && o.store != CORD_STORE_CKPT && o.store != CORD_STORE_FINAL)
        return fail(CORD_EINVAL, "cord_rollout: bad store mode %d", o.store);
    if (o.store == CORD_STORE_CKPT && o.ckpt_every < 1) return fail(CORD_EINVAL, "cord_rollout: ckpt_every must be >= 1");
    KArgs a = base_args(s);
    a.store = o.store;
    a.ckpt_every = o.store == CORD_STORE_CKPT ? o.ckpt_every : 1;
    a.use_kappa_bwd = o.use_kappa_bwd;
    if (o.store == CORD_STORE_CKPT) {
        int rc = ensure_ckpt(s, o.ckpt_every);
        if (rc) return rc;
        a.ckpt_off = s->ckpt_dev[o.ckpt_every];
    }
    a.s0 = s0; a.u = u; a.traj = traj; a.status = inst_status; a.counters = o.counters;
    a.final_out = o.final_state;
    if (s->aux && o.store == CORD_STORE_FULL) { a.aux = s->aux; a.aux_mode = 1; }
    return launch_all(s, kOpRollout, a, (hipStream_t)stream);
}

int cord_sim_set_aux(cord_sim* s, float* aux) {
    g_err.clear();
    if (!s) return fail(CORD_EINVAL, "cord_sim_set_aux: NULL sim");
    s->aux = aux;
    return CORD_OK;
}

int cord_rollout_backward(cord_sim* s, const float* u, const float* traj, const float* traj_bar, float* s0_bar,
                          float* u_bar, int32_t* inst_status, const cord_backward_opts* opts, void* stream) {
    g_err.clear();
    if (!s || !traj || !s0_bar) return fail(CORD_EINVAL, "cord_rollout_backward: NULL sim, traj or s0_bar");
    if ((!u || !u_bar) && s->info.u_floats > 0) return fail(CORD_EINVAL, "cord_rollout_backward: NULL u or u_bar");
    cord_backward_opts o{};
    o.store = CORD_STORE_FULL;
    if (opts) o = *opts;
    if (o.store != CORD_STORE_FULL && o.store != CORD_STORE_CKPT)
        return fail(CORD_EINVAL, "cord_rollout_backward: store must be FULL or CKPT");
    if (o.store == CORD_STORE_CKPT && o.ckpt_every < 1) return fail(CORD_EINVAL, "cord_rollout_backward: ckpt_every must be >= 1");
    KArgs a = base_args(s);
    a.store = o.store;
    a.ckpt_every = o.store == CORD_STORE_CKPT ? o.ckpt_every : 1;
    a.use_kappa_bwd = o.use_kappa_bwd;
    if (o.store == CORD_STORE_CKPT) {
        int rc = ensure_ckpt(s, o.ckpt_every);
        if (rc) return rc;
        rc = ensure_seg(s, o.ckpt_every);
        if (rc) return rc;
        a.ckpt_off = s->ckpt_dev[o.ckpt_every];
        a.seg = s->seg;
        a.seg_off = s->seg_off;
    }
    a.u = u; a.traj_in = traj; a.traj_bar = traj_bar; a.sT_bar = o.sT_bar;
    a.s0_bar = s0_bar; a.u_bar = u_bar; a.status = inst_status; a.counters = o.counters;
    if (s->aux && o.store == CORD_STORE_FULL) { a.aux = s->aux; a.aux_mode = 2; }
    return launch_all(s, kOpBackward, a, (hipStream_t)stream);
}

int cord_rollout_backward_noalloc(cord_sim* s, const float* u, const float* traj, const float* traj_bar,
                                  float* s0_bar, float* u_bar, int32_t* inst_status, const cord_backward_opts* opts,
                                  void* stream) {
    g_err.clear();
    if (!s || !traj || !s0_bar) return fail(CORD_EINVAL, "cord_rollout_backward_noalloc: NULL sim, traj or s0_bar");
    if ((!u || !u_bar) && s->info.u_floats > 0)
        return fail(CORD_EINVAL, "cord_rollout_backward_noalloc: NULL u or u_bar");
    cord_backward_opts o{};
    o.store = CORD_STORE_FULL;
    if (opts) o = *opts;
    if (o.store != CORD_STORE_FULL && o.store != CORD_STORE_CKPT)
        return fail(CORD_EINVAL, "cord_rollout_backward_noalloc: store must be FULL or CKPT");
    if (o.store == CORD_STORE_CKPT && o.ckpt_every < 1)
        return fail(CORD_EINVAL, "cord_rollout_backward_noalloc: ckpt_every must be >= 1");
    if (!s->noalloc)
        return fail(CORD_EHIP, "cord_rollout_backward_noalloc: no device scratch (%s)", hipGetErrorString(s->noalloc_err));
    hipStream_t st = (hipStream_t)stream;
    KArgs a = base_args(s);
    a.store = o.store;
    a.ckpt_every = o.store == CORD_STORE_CKPT ? o.ckpt_every : 1;
    a.use_kappa_bwd = o.use_kappa_bwd;
    if (o.store == CORD_STORE_CKPT) {
        const int B = (int)s->h.size();
        const int64_t K = o.ckpt_every;
        const size_t table = ((size_t)8 * B + 255) / 256 * 256;
        const int64_t seg = K * s->info.s_floats;
        if (seg > (int64_t)((kNoAllocScratchBytes - std::min(table, kNoAllocScratchBytes)) / sizeof(float)))
            return fail(CORD_ETOOBIG, "cord_rollout_backward_noalloc: needs %zu + %lld bytes of scratch, the maximum is %zu",
                        table, (long long)(4 * seg), kNoAllocScratchBytes);
        int64_t* off = static_cast<int64_t*>(s->noalloc);
        CORD_HIP(launch_ckpt_offsets(s->d_inst, B, o.ckpt_every, off, st));
        a.ckpt_off = off;
        a.seg = reinterpret_cast<float*>(static_cast<char*>(s->noalloc) + table);
        a.seg_off = nullptr;   // K n_s floats per instance in instance order
    }
    a.u = u; a.traj_in = traj; a.traj_bar = traj_bar; a.sT_bar = o.sT_bar;
    a.s0_bar = s0_bar; a.u_bar = u_bar; a.status = inst_status; a.counters = o.counters;
    if (s->aux && o.store == CORD_STORE_FULL) { a.aux = s->aux; a.aux_mode = 2; }
    // one launch per size class, whatever the simulator's launch mode (the
    // persistent and graph modes create streams, queues and graphs)
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    for (const Group& G : s->groups) {
        a.ids = G.d_ids;
        a.n_ids = (int)G.ids.size();
        a.queue = nullptr;
        CORD_HIP(launch_op(cfg[G.cfg], kOpBackward, a, a.n_ids, st, G.fric));
    }
    return CORD_OK;
}

int cord_linearize(cord_sim* s, const float* traj, const float* u, float* A, float* Bm, const cord_jvp* jvp,
                   int32_t* inst_status, void* stream) {
    g_err.clear();
    if (!s || !traj) return fail(CORD_EINVAL, "cord_linearize: NULL sim or traj");
    if (!A && !Bm && !jvp) return fail(CORD_EINVAL, "cord_linearize: nothing requested (A, Bm and jvp are NULL)");
    if (!u && s->info.u_floats > 0) return fail(CORD_EINVAL, "cord_linearize: NULL u");
    if (jvp && (jvp->k < 1 || !jvp->out)) return fail(CORD_EINVAL, "cord_linearize: jvp needs k >= 1 and out");
    KArgs a = base_args(s);
    a.traj_in = traj; a.u = u; a.A = A; a.Bm = Bm; a.status = inst_status;
    if (s->aux) { a.aux = s->aux; a.aux_mode = 2; }
    if (jvp) { a.jvp_k = jvp->k; a.jvp_ds = jvp->ds; a.jvp_du = jvp->du; a.jvp_out = jvp->out; }
    hipStream_t st = (hipStream_t)stream;
    if (inst_status) CORD_HIP(launch_fill_i32(inst_status, s->info.n_inst, 0, st));
    if (A || Bm) {
        // per-step flags of the direct rope linearization (allocated once;
        // without them a failed band factorization is reported as NOT_PD)
        if (!s->d_redo && hipMalloc(&s->d_redo, sizeof(int32_t) * (size_t)s->n_steps) != hipSuccess) {
            s->d_redo = nullptr;
            (void)hipGetLastError();
        }
        if (s->d_redo) {
            CORD_HIP(launch_fill_i32(s->d_redo, s->n_steps, 0, st));
            a.redo = s->d_redo;
        }
        if (!s->lin_stats) {
            if (hipMalloc(&s->lin_stats, 4 * sizeof(uint32_t)) != hipSuccess ||
                hipMemset(s->lin_stats, 0, 4 * sizeof(uint32_t)) != hipSuccess) {
                (void)hipGetLastError();
                if (s->lin_stats) (void)hipFree(s->lin_stats);
                s->lin_stats = nullptr;
            }
        }
        a.lin_stats = s->lin_stats;
    }
    for (const Group& g : s->groups) {
        a.ids = g.d_ids;
        a.n_ids = (int)g.ids.size();
        CORD_HIP(launch_linearize(g.cfg, g.topo, g.nmax, g.penalty, g.fric, a, a.n_ids, g.tmax, st,
                                  KeptSource{&sim_kept, s}));
    }
    return CORD_OK;
}

int cord_sim_lin_stats(cord_sim* s, int64_t* out2) {
    g_err.clear();
    if (!s || !out2) return fail(CORD_EINVAL, "cord_sim_lin_stats: NULL argument");
    uint32_t h[2] = {0, 0};
    if (s->lin_stats) CORD_HIP(hipMemcpy(h, s->lin_stats, sizeof(h), hipMemcpyDeviceToHost));
    out2[0] = h[0];
    out2[1] = h[1];
    return CORD_OK;
}

int cord_cp_scores(cord_sim* s, const float* s_bar, const float* u, const float* s_next, float* scores,
                   int32_t* inst_status, void* stream) {
    g_err.clear();
    if (!s || !s_bar || !s_next || !scores) return fail(CORD_EINVAL, "cord_cp_scores: NULL argument");
    if (!u && s->info.u_floats > 0) return fail(CORD_EINVAL, "cord_cp_scores: NULL u");
    if (s->info.max_T != 1) return fail(CORD_EINVAL, "cord_cp_scores: every calibration instance needs T = 1");
    if (!s->cp_pred && hipMalloc(&s->cp_pred, sizeof(float) * (size_t)s->info.s_floats) != hipSuccess) {
        s->cp_pred = nullptr;
        (void)hipGetLastError();
        return fail(CORD_ENOMEM, "cord_cp_scores: prediction buffer");
    }
    hipStream_t st = (hipStream_t)stream;
    KArgs a = base_args(s);
    a.store = CORD_STORE_FINAL;
    a.ckpt_every = 1;
    a.s0 = s_bar; a.u = u; a.traj = s->cp_pred; a.status = inst_status;
    int rc = launch_all(s, kOpRollout, a, st);
    if (rc) return rc;
    CORD_HIP(launch_cp_scores(s->d_inst, (int)s->h.size(), s->cp_pred, s_next, scores, st));
    return CORD_OK;
}

int cord_cp_radius(const float* scores, int32_t n, double delta, int32_t horizon, float* radius, int32_t* index,
                   void* stream) {
    g_err.clear();
    if (!scores || !radius || n < 1 || horizon < 1) return fail(CORD_EINVAL, "cord_cp_radius: bad arguments");
    if (n > (1 << 16)) return fail(CORD_EUNSUPPORTED, "cord_cp_radius: at most 65536 scores");
    const double lvl = delta / horizon;
    if (!(lvl > 0.0 && lvl < 1.0)) return fail(CORD_EINVAL, "cord_cp_radius: delta / horizon must lie in (0, 1)");
    const double kk = std::ceil((n + 1.0) * (1.0 - lvl) - 1e-9);
    const int k = kk > n ? n + 1 : (int)kk;
    CORD_HIP(launch_cp_radius(scores, n, k, radius, index, (hipStream_t)stream));
    return CORD_OK;
}

int cord_autotune(cord_sim* s, const float* s0, const float* u, int32_t sample, const char* cache_path, void* stream) {
    g_err.clear();
    if (!s || !s0 || (!u && s->info.u_floats > 0) || sample < 1) return fail(CORD_EINVAL, "cord_autotune: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    auto cache = read_cache(cache_path);
    float* out = nullptr;
    if (hipMalloc(&out, sizeof(float) * (size_t)s->info.s_floats) != hipSuccess) return fail(CORD_ENOMEM, "autotune buffer");
    int32_t* ids = nullptr;
    if (hipMalloc(&ids, sizeof(int32_t) * (size_t)sample) != hipSuccess) {
        (void)hipFree(out);
        return fail(CORD_ENOMEM, "autotune ids");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int rc = CORD_OK;
    for (Group& G : s->groups) {
        const int ctopo = G.topo == kRope ? CORD_ROPE : CORD_CLOTH;
        int chosen = -1;
        for (const auto& e : cache)
            if (e[0] == ctopo && e[1] == G.nmax) chosen = find_config(G.topo, e[2], e[3]);
        if (chosen < 0) {
            // sample: the first `sample` ids (longest first) of the class
            const int ns = std::min<int>(sample, (int)G.ids.size());
            if (hipMemcpy(ids, G.ids.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice) != hipSuccess) {
                rc = fail(CORD_EHIP, "autotune upload");
                break;
            }
            float best = 1e30f;
            for (int c = 0; c < count && !rc; ++c) {
                if (cfg[c].topo != G.topo || cfg[c].nt * cfg[c].ppt < G.nmax) continue;
                KArgs a = base_args(s);
                a.store = CORD_STORE_FINAL;
                a.ckpt_every = 1;
                a.s0 = s0; a.u = u; a.traj = out;
                a.ids = ids; a.n_ids = ns;
                std::vector<float> t;
                for (int r = 0; r < 4; ++r) {
                    (void)hipEventRecord(e0, st);
                    if ((G.fric ? cfg[c].rollout_f : cfg[c].rollout)(a, ns, st) != hipSuccess) {
                        rc = fail(CORD_EHIP, "autotune launch");
                        break;
                    }
                    (void)hipEventRecord(e1, st);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (r) t.push_back(ms);
                }
                if (rc) break;
                std::sort(t.begin(), t.end());
                if (t[t.size() / 2] < best) { best = t[t.size() / 2]; chosen = c; }
            }
            if (rc) break;
            cache.push_back({ctopo, G.nmax, cfg[chosen].nt, cfg[chosen].ppt});
        }
        if (chosen >= 0 && chosen != G.cfg) {
            G.cfg = chosen;
            if ((rc = upload_group(s, G))) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(ids);
    drop_graphs(s);
    if (rc) return rc;
    if (!write_cache(cache_path, cache)) return fail(CORD_EINVAL, "cannot write autotune cache %s", cache_path);
    return CORD_OK;
}

}  // extern "C"
