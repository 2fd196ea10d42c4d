// Host side of the libcord C ABI: validation, size classes, offsets,
// workspaces and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/cord.h"
#include "cord_internal.h"
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

#define CORD_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) return fail(CORD_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

struct Group {
    int cfg = -1;
    std::vector<int32_t> ids;
    int32_t* d_ids = nullptr;
    int tmax = 0;
};

}  // namespace

struct cord_sim {
    int device = 0;
    std::vector<cord_instance_desc> desc;
    std::vector<InstDev> h;
    InstDev* d_inst = nullptr;
    std::vector<Group> groups;
    cord_sim_info_t info{};
    std::map<int, std::vector<int64_t>> ckpt_host;   // K -> offsets (n_inst + 1)
    std::map<int, int64_t*> ckpt_dev;
    float* seg = nullptr;          // backward segment workspace
    size_t seg_floats = 0;
    int seg_K = 0;
    int64_t* seg_off = nullptr;
    std::vector<int64_t> seg_off_host;
    int32_t* scratch_status = nullptr;
};

namespace {

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
    if (p.mu != 0.f) return fail(CORD_EUNSUPPORTED, "instance %d: friction mu != 0 is not supported", i);
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
    return CORD_OK;
}

int pick_config(const cord_instance_desc& d) {
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    const int n = d.nx * d.ny;
    const int topo = d.kind == CORD_ROPE ? kRope : kCloth;
    for (int c = 0; c < count; ++c)
        if (cfg[c].topo == topo && cfg[c].nt * cfg[c].ppt >= n) return c;
    return -1;
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
    if (s->seg) { (void)hipFree(s->seg); s->seg = nullptr; }
    if (s->seg_off) { (void)hipFree(s->seg_off); s->seg_off = nullptr; }
    if (hipMalloc(&s->seg, sizeof(float) * (size_t)off[B]) != hipSuccess)
        return fail(CORD_ENOMEM, "backward workspace of %lld floats", (long long)off[B]);
    CORD_HIP(hipMalloc(&s->seg_off, sizeof(int64_t) * B));
    CORD_HIP(hipMemcpy(s->seg_off, off.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice));
    s->seg_off_host = off;
    s->seg_floats = (size_t)off[B];
    s->seg_K = K;
    return CORD_OK;
}

KArgs base_args(const cord_sim* s) {
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.inst = s->d_inst;
    return a;
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
    s->desc.assign(inst, inst + n_inst);
    s->h.resize(n_inst);
    int64_t so = 0, uo = 0, to = 0, tns = 0, ao = 0, bo = 0;
    int max_n = 0, max_T = 0;
    std::map<int, int> cfg_group;
    for (int i = 0; i < n_inst; ++i) {
        const cord_instance_desc& d = inst[i];
        InstDev& I = s->h[i];
        std::memset(&I, 0, sizeof(I));
        I.kind = d.kind == CORD_ROPE ? kRope : kCloth;
        I.nx = d.nx; I.ny = d.ny; I.n = d.nx * d.ny;
        I.T = d.T; I.n_grip = d.n_grip;
        I.n_s = 6 * I.n; I.n_u = 3 * d.n_grip;
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
        I.s_off = so; I.u_off = uo; I.traj_off = to; I.tns_off = tns; I.A_off = ao; I.B_off = bo;
        so += I.n_s;
        uo += (int64_t)I.T * I.n_u;
        to += (int64_t)(I.T + 1) * I.n_s;
        tns += (int64_t)I.T * I.n_s;
        ao += (int64_t)I.T * I.n_s * I.n_s;
        bo += (int64_t)I.T * I.n_s * I.n_u;
        max_n = I.n > max_n ? I.n : max_n;
        max_T = I.T > max_T ? I.T : max_T;
        const int c = pick_config(d);
        if (c < 0) { delete s; return fail(CORD_EUNSUPPORTED, "instance %d: %d nodes exceed every kernel configuration", i, I.n); }
        if (!cfg_group.count(c)) { cfg_group[c] = (int)s->groups.size(); s->groups.push_back(Group{}); s->groups.back().cfg = c; }
        Group& g = s->groups[cfg_group[c]];
        g.ids.push_back(i);
        g.tmax = I.T > g.tmax ? I.T : g.tmax;
    }
    s->info.n_inst = n_inst;
    s->info.s_floats = so; s->info.u_floats = uo; s->info.traj_floats = to;
    s->info.A_floats = ao; s->info.B_floats = bo;
    s->info.max_n = max_n; s->info.max_T = max_T;
    auto cleanup = [&](int code, const char* what) {
        cord_sim_destroy(s);
        return fail(code, "%s", what);
    };
    if (hipMalloc(&s->d_inst, sizeof(InstDev) * n_inst) != hipSuccess) return cleanup(CORD_ENOMEM, "device instance table");
    if (hipMemcpy(s->d_inst, s->h.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(CORD_EHIP, "upload of instance table failed");
    for (Group& g : s->groups) {
        if (hipMalloc(&g.d_ids, sizeof(int32_t) * g.ids.size()) != hipSuccess) return cleanup(CORD_ENOMEM, "device id table");
        if (hipMemcpy(g.d_ids, g.ids.data(), sizeof(int32_t) * g.ids.size(), hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(CORD_EHIP, "upload of id table failed");
    }
    *out = s;
    return CORD_OK;
}

int cord_sim_destroy(cord_sim* s) {
    if (!s) return CORD_OK;
    if (s->d_inst) (void)hipFree(s->d_inst);
    for (Group& g : s->groups)
        if (g.d_ids) (void)hipFree(g.d_ids);
    for (auto& kv : s->ckpt_dev) (void)hipFree(kv.second);
    if (s->seg) (void)hipFree(s->seg);
    if (s->seg_off) (void)hipFree(s->seg_off);
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
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    hipStream_t st = (hipStream_t)stream;
    for (const Group& g : s->groups) {
        a.ids = g.d_ids;
        a.n_ids = (int)g.ids.size();
        CORD_HIP(cfg[g.cfg].rollout(a, a.n_ids, st));
    }
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
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    hipStream_t st = (hipStream_t)stream;
    for (const Group& g : s->groups) {
        a.ids = g.d_ids;
        a.n_ids = (int)g.ids.size();
        CORD_HIP(cfg[g.cfg].backward(a, a.n_ids, st));
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
    if (jvp) { a.jvp_k = jvp->k; a.jvp_ds = jvp->ds; a.jvp_du = jvp->du; a.jvp_out = jvp->out; }
    hipStream_t st = (hipStream_t)stream;
    if (inst_status) CORD_HIP(launch_fill_i32(inst_status, s->info.n_inst, 0, st));
    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    for (const Group& g : s->groups) {
        a.ids = g.d_ids;
        a.n_ids = (int)g.ids.size();
        CORD_HIP(cfg[g.cfg].linearize(a, a.n_ids, g.tmax, st));
    }
    return CORD_OK;
}

}  // extern "C"
