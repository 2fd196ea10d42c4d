// Planning server: continuous batching of gradient-based planning requests.
//
// One scheduler thread owns every HIP call of the server.  Requests wait in
// a FIFO; the scheduler admits a request when a slot (device stream) is free
// and its device footprint fits in the remaining budget (a request that does
// not fit may be overtaken by at most kSkipAhead later ones).  Device memory
// is sub-allocated from one arena reserved at start, so admission and
// completion never call hipMalloc/hipFree (which would synchronise the device
// and serialise the slots).  Each slot owns pinned host staging: uploads and
// the result download are asynchronous copies on the slot's stream, queued
// with the request's kernels, so the scheduler never waits on the device.
// Completion is detected by polling one event per request; results are then
// copied from the slot's staging to host buffers owned by the request.  The
// server mutex guards only the queues and counters: staging, uploads, kernel
// launches and result copies run without it, so submit/poll/wait never wait
// for device work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/cord.h"
#include "cord_host.h"
#include "cord_internal.h"
#include "cord_kernels.h"

namespace cord {
hipError_t plan_cost(const InstDev* inst, int n_cand, const float* traj, const float* u, int goal_node,
                     const float goal[3], float reg, float* cost, float* sT_bar, hipStream_t s);
hipError_t plan_update(float* u, const float* ubar, int64_t n, float step, float reg, float umax, hipStream_t s);
hipError_t plan_argmin(const float* cost, int n, int32_t* best, float* best_cost, hipStream_t s);
hipError_t plan_gather(const float* src, int64_t stride, int64_t len, const int32_t* best, float* dst,
                       hipStream_t s);
hipError_t plan_status(const int32_t* st, int n, int32_t* out, hipStream_t s);
}  // namespace cord

using namespace cord;

namespace {

constexpr int kSkipAhead = 8;
constexpr size_t kAlign = 256;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit sub-allocator over one device reservation.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    void init(char* b, size_t c) {
        base = b;
        cap = c;
        free_.clear();
        free_[0] = c;
    }
    bool alloc(size_t sz, size_t* off) {
        sz = (sz + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= sz) {
                *off = it->first;
                const size_t rest = it->second - sz, o = it->first;
                free_.erase(it);
                if (rest) free_[o + sz] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t sz) {
        sz = (sz + kAlign - 1) / kAlign * kAlign;
        auto it = free_.emplace(off, sz).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum State { kQueued = 0, kRunning = 1, kDone = 2 };

struct Req {
    uint64_t ticket = 0;
    cord_plan_request r{};
    std::vector<float> s0, u_warm, u_init;
    int state = kQueued;
    int T = 0, n = 0, ns = 0, nu = 0, C = 0, cfg = -1;
    size_t footprint = 0;
    std::vector<std::pair<size_t, size_t>> blocks;
    int slot = -1;
    hipEvent_t ev = nullptr;
    // device pointers
    InstDev* d_inst = nullptr;
    int32_t *d_ids = nullptr, *d_status = nullptr, *d_best = nullptr, *d_simst = nullptr, *d_redo = nullptr;
    float *d_s0 = nullptr, *d_u = nullptr, *d_traj = nullptr, *d_sT = nullptr, *d_s0b = nullptr, *d_ub = nullptr;
    float *d_cost = nullptr, *d_bcost = nullptr, *d_ubest = nullptr, *d_tbest = nullptr, *d_A = nullptr, *d_B = nullptr;
    float* d_aux = nullptr;   // step internals of the candidates' rollouts
    // results
    cord_plan_result res{};
    std::vector<float> h_u, h_traj, h_A, h_B, h_costs;
};

size_t al(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

size_t footprint_of(int C, int T, int n, int ns, int nu, bool ab) {
    size_t f = 0;
    f += al(4ull * C * T * n * kAuxFields);        // step internals
    f += al(sizeof(InstDev) * C) + al(4 * C) * 3 + al(8) * 2;
    f += al(4ull * C * ns) * 3;                     // s0, sT_bar, s0_bar
    f += al(4ull * C * T * nu) * 2;                 // u, u_bar
    f += al(4ull * C * (T + 1) * ns);               // trajectories
    f += al(4ull * C);                              // costs
    f += al(4ull * T * nu) + al(4ull * (T + 1) * ns);
    if (ab) f += al(4ull * T * ns * ns) + al(4ull * T * ns * nu) + al(4ull * T);   // + per-step redo flags
    return f;
}

// SplitMix64 (Steele, Lea, Flood 2014) and Box-Muller for the candidate noise.
uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double unit_open(uint64_t& x) { return ((double)(splitmix64(x) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

// Pinned host staging of one slot, grown on demand (only while the slot is
// idle, so no copy on its stream can still be reading or writing it).
struct Staging {
    char* up = nullptr;
    size_t up_cap = 0;
    char* down = nullptr;
    size_t down_cap = 0;
};

bool grow_pinned(char** p, size_t* cap, size_t need) {
    if (need <= *cap) return true;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t n = std::max(need, (size_t)1 << 20);
    if (hipHostMalloc((void**)p, n, hipHostMallocDefault) != hipSuccess) {
        *p = nullptr;
        return false;
    }
    *cap = n;
    return true;
}

// Byte offsets of the pieces of one request inside its slot's staging.
struct UpLayout {
    size_t inst, ids, s0, u, total;
};
struct DownLayout {
    size_t best, simst, bcost, costs, u, traj, A, B, total;
};

UpLayout up_layout(int C, int T, int ns, int nu) {
    UpLayout L;
    size_t o = 0;
    L.inst = o; o += al(sizeof(InstDev) * C);
    L.ids = o; o += al(4ull * C);
    L.s0 = o; o += al(4ull * C * ns);
    L.u = o; o += al(4ull * C * T * nu);
    L.total = o;
    return L;
}

DownLayout down_layout(int C, int T, int ns, int nu, bool ab) {
    DownLayout L;
    size_t o = 0;
    L.best = o; o += al(4);
    L.simst = o; o += al(4);
    L.bcost = o; o += al(4);
    L.costs = o; o += al(4ull * C);
    L.u = o; o += al(4ull * T * nu);
    L.traj = o; o += al(4ull * (T + 1) * ns);
    L.A = o; o += ab ? al(4ull * T * ns * ns) : 0;
    L.B = o; o += ab ? al(4ull * T * ns * nu) : 0;
    L.total = o;
    return L;
}

}  // namespace

struct cord_server {
    int device = 0;
    size_t budget = 0, used = 0;
    int max_slots = 1;
    int queue_cap = 1024;
    char* pool = nullptr;
    Arena arena;
    std::vector<hipStream_t> slots;
    std::vector<Staging> staging;
    std::vector<int> slot_busy;
    std::deque<Req*> queue;
    std::vector<Req*> running;
    std::map<uint64_t, Req*> reqs;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::thread th;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t n_sub = 0, n_adm = 0, n_done = 0, n_fail = 0, peak_q = 0;
};

namespace {

template <class T>
T* carve(cord_server* s, Req* q, size_t bytes) {
    size_t off = 0;
    if (!s->arena.alloc(bytes, &off)) return nullptr;
    q->blocks.emplace_back(off, bytes);
    return reinterpret_cast<T*>(s->pool + off);
}

void release_blocks(cord_server* s, Req* q) {
    for (auto& b : q->blocks) s->arena.release(b.first, b.second);
    q->blocks.clear();
    s->used -= q->footprint;
}

#define SRV_HIP(call)                          \
    do {                                       \
        if ((call) != hipSuccess) return false; \
    } while (0)

// Carve every device buffer of the request from the arena; false (and
// nothing held) if the free space is too fragmented.
float* no_kept(void*, size_t) { return nullptr; }

bool carve_all(cord_server* s, Req* q) {
    const int C = q->C, T = q->T, ns = q->ns, nu = q->nu;
    const bool ab = q->r.want_AB != 0;
    q->d_inst = carve<InstDev>(s, q, sizeof(InstDev) * C);
    q->d_ids = carve<int32_t>(s, q, 4ull * C);
    q->d_status = carve<int32_t>(s, q, 4ull * C);
    q->d_best = carve<int32_t>(s, q, 8);
    q->d_simst = carve<int32_t>(s, q, 8);
    q->d_s0 = carve<float>(s, q, 4ull * C * ns);
    q->d_sT = carve<float>(s, q, 4ull * C * ns);
    q->d_s0b = carve<float>(s, q, 4ull * C * ns);
    q->d_u = carve<float>(s, q, 4ull * C * T * nu);
    q->d_ub = carve<float>(s, q, 4ull * C * T * nu);
    q->d_traj = carve<float>(s, q, 4ull * C * (T + 1) * ns);
    q->d_aux = carve<float>(s, q, 4ull * C * T * q->n * kAuxFields);
    q->d_cost = carve<float>(s, q, 4ull * C);
    q->d_bcost = q->d_cost ? carve<float>(s, q, 8) : nullptr;
    q->d_ubest = carve<float>(s, q, 4ull * T * nu);
    q->d_tbest = carve<float>(s, q, 4ull * (T + 1) * ns);
    if (ab) {
        q->d_A = carve<float>(s, q, 4ull * T * ns * ns);
        q->d_B = carve<float>(s, q, 4ull * T * ns * nu);
        q->d_redo = carve<int32_t>(s, q, 4ull * T);
    }
    if (!q->d_inst || !q->d_ids || !q->d_status || !q->d_best || !q->d_simst || !q->d_s0 || !q->d_sT ||
        !q->d_s0b || !q->d_u || !q->d_ub || !q->d_traj || !q->d_cost || !q->d_bcost || !q->d_ubest ||
        !q->d_tbest || !q->d_aux || (ab && (!q->d_A || !q->d_B || !q->d_redo))) {
        for (auto& b : q->blocks) s->arena.release(b.first, b.second);
        q->blocks.clear();
        return false;
    }
    return true;
}

// Stage the inputs in the slot's pinned buffer and enqueue, on the slot's
// stream: uploads, the whole plan, the result download and the completion
// event.  Returns without waiting for the device.
bool enqueue(cord_server* s, Req* q) {
    hipStream_t st = s->slots[q->slot];
    Staging& sg = s->staging[q->slot];
    const int C = q->C, T = q->T, ns = q->ns, nu = q->nu;
    const bool ab = q->r.want_AB != 0;
    const UpLayout U = up_layout(C, T, ns, nu);
    const DownLayout D = down_layout(C, T, ns, nu, ab);
    if (!grow_pinned(&sg.up, &sg.up_cap, U.total) || !grow_pinned(&sg.down, &sg.down_cap, D.total)) return false;
    // candidate table, replicated start state, candidate controls
    InstDev* inst = reinterpret_cast<InstDev*>(sg.up + U.inst);
    InstDev base;
    fill_instdev(q->r.inst, base);
    for (int c = 0; c < C; ++c) {
        inst[c] = base;
        inst[c].s_off = (int64_t)c * ns;
        inst[c].u_off = (int64_t)c * T * nu;
        inst[c].traj_off = (int64_t)c * (T + 1) * ns;
        inst[c].tns_off = (int64_t)c * T * ns;
        inst[c].A_off = 0;
        inst[c].B_off = 0;
        inst[c].aux_off = (int64_t)c * T * q->n * kAuxFields;
        inst[c].t_off = 0;   // only the winner is linearized: its steps index the redo flags
    }
    int32_t* ids = reinterpret_cast<int32_t*>(sg.up + U.ids);
    for (int c = 0; c < C; ++c) ids[c] = c;
    float* s0 = reinterpret_cast<float*>(sg.up + U.s0);
    float* u = reinterpret_cast<float*>(sg.up + U.u);
    for (int c = 0; c < C; ++c) std::memcpy(&s0[(size_t)c * ns], q->s0.data(), sizeof(float) * ns);
    if (!q->u_init.empty()) {
        std::memcpy(u, q->u_init.data(), sizeof(float) * (size_t)C * T * nu);
    } else {
        uint64_t state = q->r.seed;
        for (int c = 0; c < C; ++c)
            for (int i = 0; i < T * nu; ++i) {
                const float w = q->u_warm.empty() ? 0.f : q->u_warm[i];
                float z = 0.f;
                if (c > 0) {
                    const double u1 = unit_open(state), u2 = unit_open(state);
                    z = (float)(std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
                }
                u[(size_t)c * T * nu + i] = w + q->r.sigma * z;
            }
    }
    SRV_HIP(hipMemcpyAsync(q->d_inst, inst, sizeof(InstDev) * C, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(q->d_ids, ids, 4ull * C, hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(q->d_s0, s0, 4ull * C * ns, hipMemcpyHostToDevice, st));
    if (T * nu > 0) SRV_HIP(hipMemcpyAsync(q->d_u, u, 4ull * C * T * nu, hipMemcpyHostToDevice, st));

    int count = 0;
    const KernelCfg* cfg = kernel_configs(&count);
    const KernelCfg& K = cfg[q->cfg];
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.inst = q->d_inst;
    a.ids = q->d_ids;
    a.n_ids = C;
    a.ckpt_every = 1;
    a.status = q->d_status;
    const float reg = q->r.u_reg;
    const bool fric = q->r.inst.params.mu > 0.f;
    const auto roll = fric ? K.rollout_f : K.rollout;
    const auto back = fric ? K.backward_f : K.backward;
    for (int it = 0; it < q->r.iters; ++it) {
        KArgs f = a;
        f.store = CORD_STORE_FULL;
        f.s0 = q->d_s0; f.u = q->d_u; f.traj = q->d_traj;
        f.aux = q->d_aux; f.aux_mode = 1;
        SRV_HIP(roll(f, C, st));
        SRV_HIP(plan_cost(q->d_inst, C, q->d_traj, q->d_u, q->r.goal_node, q->r.goal, reg, q->d_cost, q->d_sT, st));
        KArgs b = a;
        b.store = CORD_STORE_FULL;
        b.u = q->d_u; b.traj_in = q->d_traj; b.sT_bar = q->d_sT; b.s0_bar = q->d_s0b; b.u_bar = q->d_ub;
        b.aux = q->d_aux; b.aux_mode = 2;
        SRV_HIP(back(b, C, st));
        SRV_HIP(plan_update(q->d_u, q->d_ub, (int64_t)C * T * nu, q->r.step, reg, q->r.u_max, st));
    }
    KArgs f = a;
    f.store = CORD_STORE_FULL;
    f.s0 = q->d_s0; f.u = q->d_u; f.traj = q->d_traj;
    f.aux = q->d_aux; f.aux_mode = 1;
    SRV_HIP(roll(f, C, st));
    SRV_HIP(plan_cost(q->d_inst, C, q->d_traj, q->d_u, q->r.goal_node, q->r.goal, reg, q->d_cost, nullptr, st));
    SRV_HIP(plan_argmin(q->d_cost, C, q->d_best, q->d_bcost, st));
    SRV_HIP(plan_status(q->d_status, C, q->d_simst, st));
    SRV_HIP(plan_gather(q->d_u, (int64_t)T * nu, (int64_t)T * nu, q->d_best, q->d_ubest, st));
    SRV_HIP(plan_gather(q->d_traj, (int64_t)(T + 1) * ns, (int64_t)(T + 1) * ns, q->d_best, q->d_tbest, st));
    if (ab) {
        KArgs l = a;
        l.ids = q->d_best;   // the winner's index, read on the device
        l.n_ids = 1;
        l.traj_in = q->d_traj; l.u = q->d_u; l.A = q->d_A; l.Bm = q->d_B;
        l.lin_zero_off = 1;
        l.status = nullptr;
        l.aux = q->d_aux; l.aux_mode = 2;
        l.redo = q->d_redo;
        SRV_HIP(launch_fill_i32(q->d_redo, T, 0, st));
        const int topo = q->r.inst.kind == CORD_ROPE ? kRope : kCloth;
        // one instance: the direct kernel keeps its vectors inside A (no scratch)
        SRV_HIP(launch_linearize(q->cfg, topo, bucket_of(topo, q->n), q->r.inst.grip_mode == CORD_GRIP_PENALTY, fric,
                                 l, 1, T, st, KeptSource{&no_kept, nullptr}));
    }
    // result download into the slot's staging
    char* h = sg.down;
    SRV_HIP(hipMemcpyAsync(h + D.best, q->d_best, 4, hipMemcpyDeviceToHost, st));
    SRV_HIP(hipMemcpyAsync(h + D.simst, q->d_simst, 4, hipMemcpyDeviceToHost, st));
    SRV_HIP(hipMemcpyAsync(h + D.bcost, q->d_bcost, 4, hipMemcpyDeviceToHost, st));
    SRV_HIP(hipMemcpyAsync(h + D.costs, q->d_cost, 4ull * C, hipMemcpyDeviceToHost, st));
    if (T * nu) SRV_HIP(hipMemcpyAsync(h + D.u, q->d_ubest, 4ull * T * nu, hipMemcpyDeviceToHost, st));
    SRV_HIP(hipMemcpyAsync(h + D.traj, q->d_tbest, 4ull * (T + 1) * ns, hipMemcpyDeviceToHost, st));
    if (ab) {
        SRV_HIP(hipMemcpyAsync(h + D.A, q->d_A, 4ull * T * ns * ns, hipMemcpyDeviceToHost, st));
        if (T * nu) SRV_HIP(hipMemcpyAsync(h + D.B, q->d_B, 4ull * T * ns * nu, hipMemcpyDeviceToHost, st));
    }
    SRV_HIP(hipEventRecord(q->ev, st));
    return true;
}

// Copy a finished request's results out of its slot's staging (host only).
void collect(cord_server* s, Req* q) {
    const int C = q->C, T = q->T, ns = q->ns, nu = q->nu;
    const bool ab = q->r.want_AB != 0;
    const DownLayout D = down_layout(C, T, ns, nu, ab);
    const char* h = s->staging[q->slot].down;
    auto take = [&](std::vector<float>& v, size_t off, size_t n) {
        v.resize(n);
        if (n) std::memcpy(v.data(), h + off, 4 * n);
    };
    take(q->h_costs, D.costs, C);
    take(q->h_u, D.u, (size_t)T * nu);
    take(q->h_traj, D.traj, (size_t)(T + 1) * ns);
    if (ab) {
        take(q->h_A, D.A, (size_t)T * ns * ns);
        take(q->h_B, D.B, (size_t)T * ns * nu);
    }
    std::memcpy(&q->res.best, h + D.best, 4);
    std::memcpy(&q->res.sim_status, h + D.simst, 4);
    std::memcpy(&q->res.cost, h + D.bcost, 4);
}

void finish(cord_server* s, Req* q, int status) {
    q->res.status = status;
    q->res.T = q->T; q->res.n_s = q->ns; q->res.n_u = q->nu; q->res.n_cand = q->C;
    q->res.u = q->h_u.empty() ? nullptr : q->h_u.data();
    q->res.traj = q->h_traj.empty() ? nullptr : q->h_traj.data();
    q->res.A = q->h_A.empty() ? nullptr : q->h_A.data();
    q->res.B = q->h_B.empty() ? nullptr : q->h_B.data();
    q->res.costs = q->h_costs.empty() ? nullptr : q->h_costs.data();
    q->res.t_done = now_s();
    q->state = kDone;
    if (status == CORD_OK) ++s->n_done;
    else ++s->n_fail;
}

void scheduler(cord_server* s) {
    (void)hipSetDevice(s->device);
    std::vector<Req*> done, admitted;
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        // completions (the running list and the arena belong to this thread)
        done.clear();
        for (size_t i = 0; i < s->running.size();) {
            Req* q = s->running[i];
            const hipError_t e = hipEventQuery(q->ev);
            if (e == hipErrorNotReady) { ++i; continue; }
            q->res.status = e == hipSuccess ? CORD_OK : CORD_EHIP;
            done.push_back(q);
            s->running.erase(s->running.begin() + i);
        }
        // admissions: FIFO with bounded skip-ahead
        admitted.clear();
        if (!s->stop) {
            int scanned = 0;
            for (auto it = s->queue.begin(); it != s->queue.end() && scanned <= kSkipAhead; ++scanned) {
                int slot = -1;
                for (int k = 0; k < s->max_slots; ++k)
                    if (!s->slot_busy[k]) { slot = k; break; }
                if (slot < 0) break;
                Req* q = *it;
                if (q->footprint > s->budget - s->used || !carve_all(s, q)) { ++it; continue; }
                q->slot = slot;
                s->slot_busy[slot] = 1;
                s->used += q->footprint;
                q->res.t_admit = now_s();
                q->state = kRunning;
                ++s->n_adm;
                it = s->queue.erase(it);
                admitted.push_back(q);
            }
        }
        if (done.empty() && admitted.empty()) {
            if (s->stop && s->running.empty()) break;
            s->cv.wait_for(lk, std::chrono::microseconds(s->running.empty() ? 2000 : 50));
            continue;
        }
        // device and host copies without the lock
        lk.unlock();
        for (Req* q : done)
            if (q->res.status == CORD_OK) collect(s, q);
        std::vector<int> ok(admitted.size(), 1);
        for (size_t i = 0; i < admitted.size(); ++i) {
            if (!enqueue(s, admitted[i])) {
                (void)hipStreamSynchronize(s->slots[admitted[i]->slot]);
                ok[i] = 0;
            }
        }
        lk.lock();
        for (Req* q : done) {
            release_blocks(s, q);
            s->slot_busy[q->slot] = 0;
            finish(s, q, q->res.status);
        }
        for (size_t i = 0; i < admitted.size(); ++i) {
            Req* q = admitted[i];
            if (ok[i]) {
                s->running.push_back(q);
            } else {
                release_blocks(s, q);
                s->slot_busy[q->slot] = 0;
                finish(s, q, CORD_EHIP);
            }
        }
        s->done_cv.notify_all();
    }
}

}  // namespace

extern "C" {

int cord_server_create(int32_t device, size_t hbm_budget, int32_t max_slots, int32_t queue_cap, cord_server** out) {
    if (!out || max_slots < 1 || max_slots > 64 || queue_cap < 1 || hbm_budget < (1u << 20))
        return set_error(CORD_EINVAL, "cord_server_create: bad arguments");
    cord_server* s = new (std::nothrow) cord_server();
    if (!s) return set_error(CORD_ENOMEM, "host allocation");
    s->device = device;
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->queue_cap = queue_cap;
    if (hipSetDevice(device) != hipSuccess) { delete s; return set_error(CORD_EHIP, "hipSetDevice failed"); }
    if (hipMalloc(&s->pool, hbm_budget) != hipSuccess) { delete s; return set_error(CORD_ENOMEM, "server memory pool"); }
    s->arena.init(s->pool, hbm_budget);
    for (int k = 0; k < max_slots; ++k) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {   // default priority
            cord_server_destroy(s);
            return set_error(CORD_EHIP, "stream creation failed");
        }
        s->slots.push_back(st);
        s->staging.emplace_back();
        s->slot_busy.push_back(0);
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return CORD_OK;
}

int cord_server_destroy(cord_server* s) {
    if (!s) return CORD_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Req* q : s->queue) finish(s, q, CORD_EAGAIN);
        s->queue.clear();
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    for (auto& kv : s->reqs) {
        if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
        delete kv.second;
    }
    for (hipStream_t st : s->slots) (void)hipStreamDestroy(st);
    for (Staging& g : s->staging) {
        if (g.up) (void)hipHostFree(g.up);
        if (g.down) (void)hipHostFree(g.down);
    }
    if (s->pool) (void)hipFree(s->pool);
    delete s;
    return CORD_OK;
}

int cord_plan_submit(cord_server* s, const cord_plan_request* r, uint64_t* ticket) {
    if (!s || !r || !ticket || !r->s0) return set_error(CORD_EINVAL, "cord_plan_submit: NULL argument");
    int rc = validate(r->inst, 0);
    if (rc) return rc;
    const cord_instance_desc& d = r->inst;
    const int n = d.nx * d.ny;
    if (r->n_cand < 1 || r->iters < 0 || !(r->u_max > 0.f) || r->goal_node < 0 || r->goal_node >= n ||
        !(r->u_reg >= 0.f) || !std::isfinite(r->step))
        return set_error(CORD_EINVAL, "cord_plan_submit: bad planner parameters");
    Req* q = new (std::nothrow) Req();
    if (!q) return set_error(CORD_ENOMEM, "host allocation");
    q->r = *r;
    q->T = d.T;
    q->n = n;
    q->ns = 6 * n + (d.grip_mode == CORD_GRIP_PENALTY ? 3 * d.n_grip : 0);
    q->nu = 3 * d.n_grip;
    q->C = r->n_cand;
    const int topo = d.kind == CORD_ROPE ? kRope : kCloth;
    q->cfg = default_config(topo, bucket_of(topo, n));
    q->footprint = footprint_of(q->C, q->T, q->n, q->ns, q->nu, r->want_AB != 0);
    q->s0.assign(r->s0, r->s0 + q->ns);
    if (r->u_warm) q->u_warm.assign(r->u_warm, r->u_warm + (size_t)q->T * q->nu);
    if (r->u_init) q->u_init.assign(r->u_init, r->u_init + (size_t)q->C * q->T * q->nu);
    q->r.s0 = nullptr; q->r.u_warm = nullptr; q->r.u_init = nullptr;
    if (q->footprint > s->budget) {
        delete q;
        return set_error(CORD_ETOOBIG, "cord_plan_submit: request footprint exceeds the server budget");
    }
    if (hipEventCreateWithFlags(&q->ev, hipEventDisableTiming) != hipSuccess) {
        delete q;
        return set_error(CORD_EHIP, "event creation failed");
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop || (int)s->queue.size() >= s->queue_cap) {
            (void)hipEventDestroy(q->ev);
            delete q;
            return set_error(CORD_EAGAIN, "cord_plan_submit: queue full");
        }
        q->ticket = s->next_ticket++;
        q->res.t_submit = now_s();
        s->queue.push_back(q);
        s->reqs[q->ticket] = q;
        ++s->n_sub;
        s->peak_q = std::max<int64_t>(s->peak_q, (int64_t)s->queue.size());
        *ticket = q->ticket;
    }
    s->cv.notify_all();
    return CORD_OK;
}

int cord_plan_poll(cord_server* s, uint64_t ticket, cord_plan_result* out) {
    if (!s || !out) return set_error(CORD_EINVAL, "cord_plan_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(CORD_EINVAL, "cord_plan_poll: unknown ticket");
    if (it->second->state != kDone) return CORD_EAGAIN;
    *out = it->second->res;
    return CORD_OK;
}

int cord_plan_wait(cord_server* s, uint64_t ticket, int32_t timeout_ms, cord_plan_result* out) {
    if (!s || !out) return set_error(CORD_EINVAL, "cord_plan_wait: NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(CORD_EINVAL, "cord_plan_wait: unknown ticket");
    Req* q = it->second;
    auto pred = [&] { return q->state == kDone; };
    if (timeout_ms < 0) s->done_cv.wait(lk, pred);
    else if (!s->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) return CORD_EAGAIN;
    *out = q->res;
    return CORD_OK;
}

int cord_plan_release(cord_server* s, uint64_t ticket) {
    if (!s) return set_error(CORD_EINVAL, "cord_plan_release: NULL server");
    Req* q = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return set_error(CORD_EINVAL, "cord_plan_release: unknown ticket");
        if (it->second->state != kDone) return set_error(CORD_EAGAIN, "cord_plan_release: request not finished");
        q = it->second;
        s->reqs.erase(it);
    }
    if (q->ev) (void)hipEventDestroy(q->ev);
    delete q;
    return CORD_OK;
}

int cord_server_stats(cord_server* s, int64_t* out8) {
    if (!s || !out8) return set_error(CORD_EINVAL, "cord_server_stats: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out8[0] = s->n_sub; out8[1] = s->n_adm; out8[2] = s->n_done; out8[3] = s->n_fail;
    out8[4] = (int64_t)s->queue.size(); out8[5] = (int64_t)s->running.size();
    out8[6] = s->peak_q; out8[7] = (int64_t)s->used;
    return CORD_OK;
}

}  // extern "C"
