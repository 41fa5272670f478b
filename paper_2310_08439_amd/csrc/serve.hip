// Persistent request loop over resident systems: energy/force requests and
// velocity-Verlet NVE runs (the MD protocol of Sec. IV.D), served by a pool of
// worker threads with one HIP stream and one workspace each, so that requests
// admitted together run concurrently on the device.
//
// Admission: a queued request is taken by a free worker when no earlier
// request on the same system is still queued or running (requests on one
// system keep their order) and the system's neighbour list fits in the memory
// budget; idle systems' lists are evicted, least recently used first.  System
// state (positions, velocities, forces, reference positions of the last list
// build) stays resident from registration to destruction.
#include "tmd_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <thread>

namespace tmd {
namespace {

constexpr double kAccConv = 9.648533e-3;  // (eV/A)/amu -> A/fs^2

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct System {
    int64_t id = 0, n = 0;
    double box[3] = {0, 0, 0};
    double* x = nullptr;       // [n][3] positions (not wrapped)
    double* v = nullptr;       // [n][3] velocities
    double* xref = nullptr;    // [n][3] positions at the last list build
    float* F = nullptr;        // [n][3] forces at x
    int32_t* sp = nullptr;     // [n]
    double* acc = nullptr;     // [S] kAccConv / m_s
    double* mass = nullptr;    // [S]
    size_t state_bytes = 0;
    tmd_nlist* nl = nullptr;
    int cap = 0;
    size_t nl_bytes = 0;
    bool nl_valid = false;     // built for the current positions (within skin/2)
    bool busy = false;
    uint64_t last_use = 0;
};

struct Pending {
    uint64_t ticket = 0;
    tmd_request req{};
    std::vector<double> vel;
    double t_submit = 0.0;
};

struct Finished {
    tmd_result res{};
    std::vector<float> F;
    std::vector<double> x, v, epot, ekin;
};

}  // namespace
}  // namespace tmd

struct tmd_server {
    const tmd_model* model = nullptr;
    tmd_serve_opts opts{};
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<tmd::Pending> queue;
    std::set<uint64_t> running;
    std::map<uint64_t, tmd::Finished> done;
    std::map<int64_t, std::unique_ptr<tmd::System>> systems;
    int64_t next_system = 0;
    uint64_t next_ticket = 1;
    uint64_t clock = 0;
    int64_t mem_in_use = 0, mem_peak = 0;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::vector<tmd_context*> ctxs;
    std::vector<hipEvent_t> events;  // two per slot: the ends of an MD request's last two queued chunks
    // lists evicted under the lock, destroyed by a worker after it releases the
    // lock (destroying a list waits for the whole device)
    std::vector<tmd_nlist*> retired;
    // builds the lists of newly registered systems (under admin_mu), so that
    // requests on them neither allocate nor build a first list
    tmd_context* admin = nullptr;
    hipStream_t admin_stream = nullptr;
    std::mutex admin_mu;
    bool stop = false;
    std::string last_error;
};

namespace tmd {
namespace {

// An MD request queues its steps in chunks of at least this many atom-steps
// and keeps at most two chunks on its stream: streams share the device's few
// hardware queues, whose packets run in order, so a request submitted on
// another slot waits behind at most two chunks of a long MD request rather
// than behind all of its steps.
constexpr int64_t kMdChunkAtomSteps = 65536;

void account(tmd_server* sv, int64_t delta) {
    sv->mem_in_use += delta;
    sv->mem_peak = std::max(sv->mem_peak, sv->mem_in_use);
}

int density_capacity(int64_t n, const double* box, double rlist, int S) {
    const double vol = box[0] * box[1] * box[2];
    const double mean = (double)n / vol * 4.0 / 3.0 * M_PI * rlist * rlist * rlist;
    int cap = (int)(mean * (1.0 / S + 0.3)) + 16;
    return std::max(16, (cap + 7) / 8 * 8);
}

// Device bytes of a system's neighbour list; with a skin, evaluations also keep
// the rows pruned to the cutoff (same size as the rows and counts).
size_t nlist_bytes(int64_t n, int S, int cap, bool pruned) {
    const size_t rows = (size_t)n * S * cap * 8 + (size_t)S * n * 4;
    return (size_t)n * 61 + rows * (pruned ? 2 : 1) + 8 * (size_t)(4 * n + 65);
}

// Build (or rebuild) sys's list on ctx, growing it on overflow.
tmd_status build_list(tmd_server* sv, tmd_context* ctx, System* sys, int* rebuilds) {
    const tmd_model* m = sv->model;
    tmd_system_view v{};
    v.n_atoms = sys->n;
    v.pos = sys->x;
    v.species = sys->sp;
    for (int a = 0; a < 3; ++a) v.box[a] = sys->box[a];
    for (int attempt = 0; attempt < 4; ++attempt) {
        int32_t need = 0;
        tmd_status st = tmd_build_neighbors(ctx, &v, m->rcut, sv->opts.skin, sys->nl, &need);
        if (st == TMD_OK) {
            TMD_HIP(ctx, hipMemcpyAsync(sys->xref, sys->x, 24 * (size_t)sys->n, hipMemcpyDeviceToDevice, ctx->stream));
            sys->nl_valid = true;
            ++*rebuilds;
            return TMD_OK;
        }
        if (st != TMD_ERR_CAPACITY) return st;
        // grow: the budget is exceeded briefly rather than failing the request
        const int cap = (need + 8 + 7) / 8 * 8;
        tmd_nlist* nl = nullptr;
        if ((st = tmd_nlist_create(ctx, sys->n, m->S, cap, &nl)) != TMD_OK) return st;
        tmd_nlist_destroy(sys->nl);
        sys->nl = nl;
        const size_t nb = nlist_bytes(sys->n, m->S, nl->cap, sv->opts.skin > 0.0);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            account(sv, (int64_t)nb - (int64_t)sys->nl_bytes);
        }
        sys->nl_bytes = nb;
        sys->cap = nl->cap;
    }
    return fail(ctx, TMD_ERR_CAPACITY, "neighbour list kept overflowing");
}

// At registration, when the budget has room: allocate the new system's list
// (with its pruned rows) and build it on the admission context, so that the
// first request on the system neither allocates (an allocation can wait for
// the whole device, i.e. for every other slot's work) nor builds.  On any
// failure the list is left to the first request, as for an evicted one.
void admit_list(tmd_server* sv, System* sys) {
    const int S = sv->model->S;
    const bool skin = sv->opts.skin > 0.0;
    const size_t lb = nlist_bytes(sys->n, S, sys->cap, skin);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->mem_in_use + (int64_t)lb > sv->opts.hbm_budget_bytes) return;
        account(sv, (int64_t)lb);
    }
    std::lock_guard<std::mutex> ak(sv->admin_mu);
    tmd_context* ctx = sv->admin;
    tmd_nlist* nl = nullptr;
    tmd_status st = tmd_nlist_create(ctx, sys->n, S, sys->cap, &nl);
    int rebuilds = 0;
    if (st == TMD_OK) {
        sys->nl = nl;
        sys->nl_bytes = lb;
        sys->nl_valid = false;
        st = build_list(sv, ctx, sys, &rebuilds);  // may grow the list (and its accounted bytes)
    }
    if (st == TMD_OK && skin) st = reserve_pruned_rows(ctx, sys->nl);
    if (st == TMD_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = TMD_ERR_DEVICE;
    if (st == TMD_OK) return;
    const size_t held = sys->nl ? sys->nl_bytes : lb;
    if (sys->nl) tmd_nlist_destroy(sys->nl);
    std::lock_guard<std::mutex> lk(sv->mu);
    account(sv, -(int64_t)held);
    sys->nl = nullptr;
    sys->nl_bytes = 0;
    sys->nl_valid = false;
}

struct SlotBuffers {
    double* tot = nullptr;                 // [7 (n_steps + 1)]
    double* ekin = nullptr;                // [4 (n_steps + 1)] kinetic tensor diagonal and total
    double* part = nullptr;                // [3 kKeBlocks]
    unsigned long long* maxd2 = nullptr;   // [n_steps + 1] largest squared displacement since the build, per step
    unsigned long long* flag = nullptr;    // [1] nonzero: some step moved an atom beyond skin/2
    double* x0 = nullptr;                  // [n][3] positions and velocities at the start of an MD request
    double* v0 = nullptr;
};

tmd_status slot_buffers(tmd_context* ctx, int n_steps, int64_t n, SlotBuffers* b) {
    hipError_t e = hipSuccess;
    b->tot = (double*)ctx->ws.get("md.tot", sizeof(double) * 7 * (size_t)(n_steps + 1), &e);
    b->ekin = (double*)ctx->ws.get("md.ekin", sizeof(double) * 4 * (size_t)(n_steps + 1), &e);
    b->part = (double*)ctx->ws.get("md.part", sizeof(double) * 3 * kKeBlocks, &e);
    b->maxd2 = (unsigned long long*)ctx->ws.get("md.maxd2", sizeof(unsigned long long) * (size_t)(n_steps + 1), &e);
    b->flag = (unsigned long long*)ctx->ws.get("md.flag", sizeof(unsigned long long), &e);
    b->x0 = (double*)ctx->ws.get("md.x0", 24 * (size_t)n, &e);
    b->v0 = (double*)ctx->ws.get("md.v0", 24 * (size_t)n, &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "MD workspace");
    return TMD_OK;
}

tmd_status kinetic(tmd_context* ctx, const System* sys, double* part, double* out4) {
    return launch_kinetic(ctx, sys->n, sys->v, sys->sp, sys->mass, part, out4);
}

// The steps of an MD request with no host synchronisation between them: each
// step's largest displacement since the list build (maxd2[s]) gates the
// reuse of pruned rows on the device, and a sticky device flag records
// whether any step moved an atom beyond skin/2, which would have made the
// list incomplete.  The caller reads the flag with the results.  The steps go
// out in chunks of kMdChunkAtomSteps: after queueing chunk c the host waits
// for the end of chunk c - 1 (ev[0], ev[1] alternate), which leaves chunk c
// queued, so the device never idles for the wait.
tmd_status md_steps_device_gated(tmd_server* sv, tmd_context* ctx, System* sys, const tmd_system_view& view,
                                 const SlotBuffers& b, int nsteps, double dt, hipEvent_t* ev) {
    const tmd_model* m = sv->model;
    const double half_skin2 = 0.25 * sv->opts.skin * sv->opts.skin;
    tmd_status st;
    if ((st = launch_zero_u64(ctx, b.maxd2, nsteps + 1)) != TMD_OK) return st;
    int64_t queued = 0;  // atom-steps queued since the last chunk end
    int chunk = 0;
    for (int s = 1; s <= nsteps; ++s) {
        if ((st = launch_kick_drift(ctx, sys->n, sys->x, sys->v, sys->F, sys->sp, sys->acc, dt, sys->xref,
                                    b.maxd2 + s)) != TMD_OK)
            return st;
        if ((st = launch_displacement_check(ctx, b.maxd2 + s, half_skin2, b.flag)) != TMD_OK) return st;
        PruneGate gate;
        gate.maxd2 = b.maxd2 + s;
        gate.margin = 0.2 * sv->opts.skin;
        if ((st = energy_forces_gated(ctx, m, &view, sys->nl, b.tot + 7 * s, nullptr, sys->F, &gate)) != TMD_OK)
            return st;
        if ((st = launch_kick(ctx, sys->n, sys->v, sys->F, sys->sp, sys->acc, dt)) != TMD_OK) return st;
        if ((st = kinetic(ctx, sys, b.part, b.ekin + 4 * s)) != TMD_OK) return st;
        queued += sys->n;
        if (queued >= kMdChunkAtomSteps && s < nsteps) {
            TMD_HIP(ctx, hipEventRecord(ev[chunk & 1], ctx->stream));
            if (chunk > 0) TMD_HIP(ctx, hipEventSynchronize(ev[(chunk - 1) & 1]));
            ++chunk;
            queued = 0;
        }
    }
    return TMD_OK;
}

// The same steps with a host synchronisation per step, rebuilding the list
// whenever an atom has moved more than skin/2 since the last build.
tmd_status md_steps_host_checked(tmd_server* sv, tmd_context* ctx, System* sys, const tmd_system_view& view,
                                 const SlotBuffers& b, int nsteps, double dt, int* rebuilds) {
    const tmd_model* m = sv->model;
    const double half_skin2 = 0.25 * sv->opts.skin * sv->opts.skin;
    tmd_status st;
    for (int s = 1; s <= nsteps; ++s) {
        if ((st = launch_zero_u64(ctx, b.maxd2 + s, 1)) != TMD_OK) return st;
        if ((st = launch_kick_drift(ctx, sys->n, sys->x, sys->v, sys->F, sys->sp, sys->acc, dt, sys->xref,
                                    b.maxd2 + s)) != TMD_OK)
            return st;
        unsigned long long bits = 0;
        TMD_HIP(ctx, hipMemcpyAsync(ctx->h_flags, b.maxd2 + s, sizeof(bits), hipMemcpyDeviceToHost, ctx->stream));
        TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
        std::memcpy(&bits, ctx->h_flags, sizeof(bits));
        double d2;
        std::memcpy(&d2, &bits, sizeof(d2));
        if (!(d2 <= half_skin2)) {
            sys->nl_valid = false;
            if ((st = build_list(sv, ctx, sys, rebuilds)) != TMD_OK) return st;
        }
        // b.maxd2[s] now holds this system's displacement since its build: the
        // pruned rows are reused while it allows (the request's first
        // evaluation pruned to the cutoff, so the first step here prunes)
        PruneGate gate;
        gate.maxd2 = b.maxd2 + s;
        gate.margin = 0.2 * sv->opts.skin;
        if ((st = energy_forces_gated(ctx, m, &view, sys->nl, b.tot + 7 * s, nullptr, sys->F,
                                      sv->opts.skin > 0.0 ? &gate : nullptr)) != TMD_OK)
            return st;
        if ((st = launch_kick(ctx, sys->n, sys->v, sys->F, sys->sp, sys->acc, dt)) != TMD_OK) return st;
        if ((st = kinetic(ctx, sys, b.part, b.ekin + 4 * s)) != TMD_OK) return st;
    }
    return TMD_OK;
}

// Run one request to completion on the worker's context.  An MD request on a
// list with a skin first runs all its steps without host synchronisation
// (md_steps_device_gated); if the device flag shows that some step moved an
// atom beyond skin/2 (so that a list rebuild was due), the request restarts
// from its saved positions and velocities and runs with a check per step.
tmd_status run_request(tmd_server* sv, tmd_context* ctx, hipEvent_t* ev, System* sys, const Pending& p,
                       Finished* out) {
    const tmd_model* m = sv->model;
    tmd_result& r = out->res;
    tmd_status st;
    tmd_system_view view{};
    view.n_atoms = sys->n;
    view.pos = sys->x;
    view.species = sys->sp;
    for (int a = 0; a < 3; ++a) view.box[a] = sys->box[a];
    int rebuilds = 0;
    const bool md = p.req.kind == TMD_REQ_MD;
    const int nsteps = md ? p.req.n_steps : 0;
    SlotBuffers b;
    if ((st = slot_buffers(ctx, nsteps, sys->n, &b)) != TMD_OK) return st;
    if (md && !p.vel.empty())
        TMD_HIP(ctx, hipMemcpyAsync(sys->v, p.vel.data(), 24 * (size_t)sys->n, hipMemcpyHostToDevice, ctx->stream));
    if (!sys->nl_valid && (st = build_list(sv, ctx, sys, &rebuilds)) != TMD_OK) return st;
    const bool fast = md && nsteps > 0 && sv->opts.skin > 0.0;
    if (fast) {
        TMD_HIP(ctx, hipMemcpyAsync(b.x0, sys->x, 24 * (size_t)sys->n, hipMemcpyDeviceToDevice, ctx->stream));
        TMD_HIP(ctx, hipMemcpyAsync(b.v0, sys->v, 24 * (size_t)sys->n, hipMemcpyDeviceToDevice, ctx->stream));
        if ((st = launch_zero_u64(ctx, b.flag, 1)) != TMD_OK) return st;
    }
    if ((st = tmd_energy_forces_async(ctx, m, &view, sys->nl, b.tot, nullptr, sys->F)) != TMD_OK) return st;
    if (md) {
        if ((st = kinetic(ctx, sys, b.part, b.ekin)) != TMD_OK) return st;  // slot 0
        const double dt = p.req.dt_fs;
        bool done = false;
        if (fast) {
            if ((st = md_steps_device_gated(sv, ctx, sys, view, b, nsteps, dt, ev)) != TMD_OK) return st;
            TMD_HIP(ctx, hipMemcpyAsync(ctx->h_flags, b.flag, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                        ctx->stream));
            TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
            done = ctx->h_flags[0] == 0 && ctx->h_flags[1] == 0;
            if (!done) {  // restart with a check per step
                TMD_HIP(ctx, hipMemcpyAsync(sys->x, b.x0, 24 * (size_t)sys->n, hipMemcpyDeviceToDevice, ctx->stream));
                TMD_HIP(ctx, hipMemcpyAsync(sys->v, b.v0, 24 * (size_t)sys->n, hipMemcpyDeviceToDevice, ctx->stream));
                if ((st = tmd_energy_forces_async(ctx, m, &view, sys->nl, b.tot, nullptr, sys->F)) != TMD_OK)
                    return st;
                if ((st = kinetic(ctx, sys, b.part, b.ekin)) != TMD_OK) return st;
            }
        }
        if (!done && (st = md_steps_host_checked(sv, ctx, sys, view, b, nsteps, dt, &rebuilds)) != TMD_OK)
            return st;
    }
    std::vector<double> tot(7 * (size_t)(nsteps + 1));
    out->F.resize(3 * (size_t)sys->n);
    TMD_HIP(ctx, hipMemcpyAsync(tot.data(), b.tot, sizeof(double) * tot.size(), hipMemcpyDeviceToHost, ctx->stream));
    TMD_HIP(ctx, hipMemcpyAsync(out->F.data(), sys->F, 12 * (size_t)sys->n, hipMemcpyDeviceToHost, ctx->stream));
    if (md) {
        out->ekin.resize(4 * (size_t)(nsteps + 1));
        out->x.resize(3 * (size_t)sys->n);
        out->v.resize(3 * (size_t)sys->n);
        TMD_HIP(ctx, hipMemcpyAsync(out->ekin.data(), b.ekin, sizeof(double) * 4 * (nsteps + 1),
                                    hipMemcpyDeviceToHost, ctx->stream));
        TMD_HIP(ctx, hipMemcpyAsync(out->x.data(), sys->x, 24 * (size_t)sys->n, hipMemcpyDeviceToHost, ctx->stream));
        TMD_HIP(ctx, hipMemcpyAsync(out->v.data(), sys->v, 24 * (size_t)sys->n, hipMemcpyDeviceToHost, ctx->stream));
    }
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out->epot.resize(nsteps + 1);
    for (int s = 0; s <= nsteps; ++s) out->epot[s] = tot[7 * s];
    r.energy = tot[7 * nsteps];
    for (int j = 0; j < 6; ++j) r.virial[j] = tot[7 * nsteps + 1 + j];
    if (md) {
        // keep the totals only
        for (int s = 0; s <= nsteps; ++s) out->ekin[s] = out->ekin[4 * (size_t)s + 3];
        out->ekin.resize(nsteps + 1);
    }
    r.kinetic = md ? out->ekin[nsteps] : 0.0;
    r.rebuilds = rebuilds;
    return TMD_OK;
}

// Energy-and-force requests of several small systems with resident lists in
// one tmd_energy_forces_batch call (lists rebuilt first where positions have
// moved beyond skin/2).  outs[i] gets request i's result.
tmd_status run_batch(tmd_server* sv, tmd_context* ctx, const std::vector<System*>& systems,
                     std::vector<Finished>& outs) {
    const tmd_model* m = sv->model;
    const int nb = (int)systems.size();
    std::vector<tmd_system_view> views((size_t)nb);
    std::vector<const tmd_nlist*> lists((size_t)nb);
    std::vector<float*> forces((size_t)nb);
    std::vector<int> rebuilds((size_t)nb, 0);
    std::vector<size_t> foff((size_t)nb + 1, 0);  // each system's slice of one staging array
    for (int i = 0; i < nb; ++i) foff[i + 1] = foff[i] + 3 * (size_t)systems[i]->n;
    hipError_t e = hipSuccess;
    // totals [nb][7], then the forces of every system (an MD request recomputes
    // its starting forces, so the resident force arrays need not be written)
    double* tot = (double*)ctx->ws.get("serve.batch_out", sizeof(double) * 7 * (size_t)nb + 4 * foff[nb], &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch outputs");
    float* fst = reinterpret_cast<float*>(tot + 7 * (size_t)nb);
    tmd_status st;
    for (int i = 0; i < nb; ++i) {
        System* sys = systems[i];
        if (!sys->nl_valid && (st = build_list(sv, ctx, sys, &rebuilds[i])) != TMD_OK) return st;
        tmd_system_view& v = views[i];
        v.n_atoms = sys->n;
        v.pos = sys->x;
        v.species = sys->sp;
        for (int a = 0; a < 3; ++a) v.box[a] = sys->box[a];
        lists[i] = sys->nl;
        forces[i] = fst + foff[i];
    }
    if ((st = tmd_energy_forces_batch(ctx, m, nb, views.data(), lists.data(), tot, forces.data())) != TMD_OK)
        return st;
    std::vector<double> h((size_t)7 * nb + (4 * foff[nb] + 7) / 8);
    TMD_HIP(ctx, hipMemcpyAsync(h.data(), tot, sizeof(double) * 7 * (size_t)nb + 4 * foff[nb], hipMemcpyDeviceToHost,
                                ctx->stream));
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const float* hf = reinterpret_cast<const float*>(h.data() + 7 * (size_t)nb);
    for (int i = 0; i < nb; ++i) outs[i].F.assign(hf + foff[i], hf + foff[i + 1]);
    for (int i = 0; i < nb; ++i) {
        tmd_result& r = outs[i].res;
        r.energy = h[7 * (size_t)i];
        for (int j = 0; j < 6; ++j) r.virial[j] = h[7 * (size_t)i + 1 + j];
        r.kinetic = 0.0;
        r.rebuilds = rebuilds[i];
        outs[i].epot.assign(1, r.energy);
    }
    return TMD_OK;
}

// Systems of at most this many atoms (and padded batches of at most
// kServeBatchAtoms atoms, kServeBatchSystems systems) are batched.
constexpr int kServeBatchSystems = 64;
constexpr int64_t kServeBatchAtoms = 65536;

// With `first` (an energy-and-force request on a small system with a resident
// list) admitted, also take the other such requests from the queue: the first
// queued request of each idle system.  Caller holds sv->mu.
void pick_batch(tmd_server* sv, System* first, std::vector<Pending>& reqs, std::vector<System*>& systems) {
    const int64_t lim = std::min<int64_t>(sv->opts.max_atoms, kServeBatchAtoms);
    int64_t atoms = (first->n + kBlock - 1) / kBlock * kBlock;
    std::set<int64_t> seen{first->id};
    for (auto it = sv->queue.begin(); it != sv->queue.end() && (int)systems.size() < kServeBatchSystems;) {
        const int64_t sid = it->req.system_id;
        System* s2 = sv->systems.at(sid).get();
        const int64_t padded = (s2->n + kBlock - 1) / kBlock * kBlock;
        const bool take = !seen.count(sid) && it->req.kind == TMD_REQ_ENERGY_FORCES && !s2->busy && s2->nl &&
                          s2->n <= sv->opts.batch_atoms && atoms + padded <= lim;
        seen.insert(sid);  // later requests of this system wait for the first one
        if (!take) {
            ++it;
            continue;
        }
        atoms += padded;
        s2->busy = true;
        sv->running.insert(it->ticket);
        reqs.push_back(std::move(*it));
        systems.push_back(s2);
        it = sv->queue.erase(it);
    }
}

// Next admissible request (queue order, one per system at a time, list memory
// within budget after evicting idle lists).  Caller holds sv->mu.
bool pick(tmd_server* sv, Pending* out, System** sys_out, bool* rejected, Finished* rej) {
    std::set<int64_t> blocked;
    const int64_t budget = sv->opts.hbm_budget_bytes;
    for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it) {
        const int64_t sid = it->req.system_id;
        if (blocked.count(sid)) continue;
        System* sys = sv->systems.at(sid).get();
        if (sys->busy) {
            blocked.insert(sid);
            continue;
        }
        int64_t need = sys->nl ? 0 : (int64_t)nlist_bytes(sys->n, sv->model->S, sys->cap, sv->opts.skin > 0.0);
        if (need > 0 && sv->mem_in_use + need > budget) {
            // evict idle lists, least recently used first
            std::vector<System*> idle;
            for (auto& kv : sv->systems)
                if (!kv.second->busy && kv.second->nl && kv.second.get() != sys) idle.push_back(kv.second.get());
            std::sort(idle.begin(), idle.end(), [](System* a, System* b) { return a->last_use < b->last_use; });
            for (System* s : idle) {
                if (sv->mem_in_use + need <= budget) break;
                sv->retired.push_back(s->nl);
                s->nl = nullptr;
                s->nl_valid = false;
                account(sv, -(int64_t)s->nl_bytes);
                s->nl_bytes = 0;
            }
        }
        if (need > 0 && sv->mem_in_use + need > budget) {
            if (sv->running.empty()) {
                // nothing will ever free more: the request cannot be served
                *rejected = true;
                rej->res.status = TMD_ERR_REJECTED;
                rej->res.kind = it->req.kind;
                rej->res.system_id = sid;
                rej->res.n_atoms = sys->n;
                rej->res.t_submit = it->t_submit;
                rej->res.t_start = rej->res.t_done = now_s(sv->t0);
                *out = *it;
                sv->queue.erase(it);
                return true;
            }
            blocked.insert(sid);
            continue;
        }
        *out = std::move(*it);
        sv->queue.erase(it);
        sys->busy = true;
        *sys_out = sys;
        *rejected = false;
        if (need > 0) account(sv, need);  // reserved now, allocated by the worker
        return true;
    }
    return false;
}

// Run a batch taken by pick_batch and publish each request's result.
void serve_batch(tmd_server* sv, tmd_context* ctx, std::vector<Pending>& reqs, std::vector<System*>& systems) {
    const double t_start = now_s(sv->t0);
    std::vector<Finished> outs(reqs.size());
    for (size_t i = 0; i < reqs.size(); ++i) {
        Finished& f = outs[i];
        f.res.kind = reqs[i].req.kind;
        f.res.system_id = systems[i]->id;
        f.res.n_atoms = systems[i]->n;
        f.res.n_steps = 0;
        f.res.t_submit = reqs[i].t_submit;
        f.res.t_start = t_start;
        f.res.batch_size = (int32_t)reqs.size();
    }
    const tmd_status st = run_batch(sv, ctx, systems, outs);
    const double t_done = now_s(sv->t0);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (st != TMD_OK) sv->last_error = ctx->last_error;
        for (size_t i = 0; i < reqs.size(); ++i) {
            outs[i].res.status = st;
            outs[i].res.t_done = t_done;
            systems[i]->busy = false;
            systems[i]->last_use = ++sv->clock;
            sv->running.erase(reqs[i].ticket);
            sv->done[reqs[i].ticket] = std::move(outs[i]);
        }
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
}

void destroy_lists(std::vector<tmd_nlist*>& lists) {
    for (tmd_nlist* nl : lists) tmd_nlist_destroy(nl);
    lists.clear();
}

void worker_main(tmd_server* sv, int slot) {
    (void)hipSetDevice(sv->opts.device);
    tmd_context* ctx = sv->ctxs[slot];
    for (;;) {
        Pending p;
        System* sys = nullptr;
        bool rejected = false;
        Finished fin;
        std::vector<tmd_nlist*> dead;  // lists that pick() evicted, freed once the lock is released
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return sv->stop || pick(sv, &p, &sys, &rejected, &fin); });
            if (sv->stop) break;
            dead.swap(sv->retired);
            if (rejected) {
                sv->done[p.ticket] = std::move(fin);
                sv->cv_done.notify_all();
                lk.unlock();
                destroy_lists(dead);
                continue;
            }
            sv->running.insert(p.ticket);
            if (sv->opts.batch_atoms > 0 && p.req.kind == TMD_REQ_ENERGY_FORCES && sys->nl &&
                sys->n <= sv->opts.batch_atoms) {
                std::vector<Pending> reqs;
                std::vector<System*> systems;
                reqs.push_back(std::move(p));
                systems.push_back(sys);
                pick_batch(sv, sys, reqs, systems);
                if (systems.size() > 1) {
                    lk.unlock();
                    destroy_lists(dead);
                    serve_batch(sv, ctx, reqs, systems);
                    continue;
                }
                p = std::move(reqs[0]);
            }
        }
        destroy_lists(dead);
        Finished f;
        f.res.kind = p.req.kind;
        f.res.system_id = sys->id;
        f.res.n_atoms = sys->n;
        f.res.n_steps = p.req.kind == TMD_REQ_MD ? p.req.n_steps : 0;
        f.res.t_submit = p.t_submit;
        f.res.t_start = now_s(sv->t0);
        f.res.batch_size = 1;
        tmd_status st = TMD_OK;
        if (!sys->nl) {
            tmd_nlist* nl = nullptr;
            st = tmd_nlist_create(ctx, sys->n, sv->model->S, sys->cap, &nl);
            if (st == TMD_OK) {
                sys->nl = nl;
                sys->nl_bytes = nlist_bytes(sys->n, sv->model->S, sys->cap, sv->opts.skin > 0.0);
                sys->nl_valid = false;
            }
        }
        if (st == TMD_OK) st = run_request(sv, ctx, sv->events.data() + 2 * slot, sys, p, &f);
        f.res.status = st;
        f.res.t_done = now_s(sv->t0);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (st != TMD_OK) {
                sv->last_error = ctx->last_error;
                if (!sys->nl_bytes && sys->nl == nullptr)
                    account(sv, -(int64_t)nlist_bytes(sys->n, sv->model->S, sys->cap, sv->opts.skin > 0.0));
            }
            sys->busy = false;
            sys->last_use = ++sv->clock;
            sv->running.erase(p.ticket);
            sv->done[p.ticket] = std::move(f);
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();
    }
}

void release_slots(tmd_server* sv) {
    for (tmd_context* c : sv->ctxs)
        if (c) tmd_context_destroy(c);
    for (hipStream_t st : sv->streams)
        if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t e : sv->events)
        if (e) (void)hipEventDestroy(e);
    if (sv->admin) tmd_context_destroy(sv->admin);
    if (sv->admin_stream) (void)hipStreamDestroy(sv->admin_stream);
    sv->ctxs.clear();
    sv->streams.clear();
    sv->events.clear();
    sv->admin = nullptr;
    sv->admin_stream = nullptr;
}

tmd_status sfail(tmd_server* sv, tmd_status st, const char* msg) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->last_error = msg;
    return st;
}

}  // namespace
}  // namespace tmd

using namespace tmd;

extern "C" {

tmd_status tmd_serve_create(const tmd_model* model, const tmd_serve_opts* opts, tmd_server** out) {
    if (!model || !out) return TMD_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    tmd_serve_opts o{};
    if (opts) o = *opts;
    if (o.hbm_budget_bytes <= 0) o.hbm_budget_bytes = (int64_t)32 << 30;
    if (o.max_slots <= 0) o.max_slots = 8;
    if (o.max_slots > 64) return TMD_ERR_INVALID_ARGUMENT;
    if (o.max_atoms <= 0) o.max_atoms = 262144;
    if (!(o.skin >= 0.0) || !std::isfinite(o.skin)) return TMD_ERR_INVALID_ARGUMENT;
    if (o.batch_atoms < 0) return TMD_ERR_INVALID_ARGUMENT;
    tmd_server* sv = new (std::nothrow) tmd_server();
    if (!sv) return TMD_ERR_OUT_OF_MEMORY;
    sv->model = model;
    sv->opts = o;
    sv->t0 = std::chrono::steady_clock::now();
    // one stream, context and workspace per slot, sized once for max_atoms
    if (hipSetDevice(o.device) != hipSuccess) {
        delete sv;
        return TMD_ERR_DEVICE;
    }
    account(sv, (int64_t)o.max_slots *
                        (int64_t)(eval_workspace_bytes(model, o.max_atoms) + nlist_workspace_bytes(o.max_atoms)) +
                    (int64_t)nlist_workspace_bytes(o.max_atoms));  // + the admission context's
    // merged lists of batched requests (rows estimated at 64 entries per species)
    if (o.batch_atoms > 0)
        account(sv, (int64_t)o.max_slots * std::min<int64_t>(o.max_atoms, kServeBatchAtoms) *
                        (68 + (int64_t)model->S * (64 * 8 + 4)));
    if (sv->mem_in_use > o.hbm_budget_bytes) {
        delete sv;
        return TMD_ERR_REJECTED;
    }
    tmd_status st = TMD_OK;
    for (int s = 0; s < o.max_slots && st == TMD_OK; ++s) {
        hipStream_t stream = nullptr;
        tmd_context* ctx = nullptr;
        if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
            st = TMD_ERR_DEVICE;
            break;
        }
        sv->streams.push_back(stream);
        for (int k = 0; k < 2; ++k) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                st = TMD_ERR_DEVICE;
                break;
            }
            sv->events.push_back(e);
        }
        if (st != TMD_OK) break;
        st = tmd_context_create(o.device, stream, &ctx);
        if (st != TMD_OK) break;
        sv->ctxs.push_back(ctx);
        if ((st = reserve_eval_workspace(ctx, model, o.max_atoms)) != TMD_OK) break;
        st = reserve_nlist_workspace(ctx, o.max_atoms, model->S);
    }
    if (st == TMD_OK) {
        if (hipStreamCreateWithFlags(&sv->admin_stream, hipStreamNonBlocking) != hipSuccess) st = TMD_ERR_DEVICE;
        if (st == TMD_OK) st = tmd_context_create(o.device, sv->admin_stream, &sv->admin);
        if (st == TMD_OK) st = reserve_nlist_workspace(sv->admin, o.max_atoms, model->S);
    }
    if (st != TMD_OK) {
        release_slots(sv);
        delete sv;
        return st;
    }
    for (int s = 0; s < o.max_slots; ++s) sv->workers.emplace_back(worker_main, sv, s);
    *out = sv;
    return TMD_OK;
}

tmd_status tmd_serve_add_system(tmd_server* sv, int64_t n, const double* pos, const int32_t* species,
                                const double box[3], const double* masses, int64_t* system_id) {
    if (!sv) return TMD_ERR_INVALID_ARGUMENT;
    if (!pos || !species || !box || !masses || !system_id) return sfail(sv, TMD_ERR_INVALID_ARGUMENT, "null argument");
    const int S = sv->model->S;
    if (n <= 0) return sfail(sv, TMD_ERR_INVALID_ARGUMENT, "n_atoms must be positive");
    if (n > sv->opts.max_atoms) return sfail(sv, TMD_ERR_REJECTED, "system larger than max_atoms");
    for (int a = 0; a < 3; ++a)
        if (!(box[a] > 0.0) || !std::isfinite(box[a])) return sfail(sv, TMD_ERR_INVALID_ARGUMENT, "bad box");
    for (int s = 0; s < S; ++s)
        if (!(masses[s] > 0.0) || !std::isfinite(masses[s])) return sfail(sv, TMD_ERR_INVALID_ARGUMENT, "bad mass");
    for (int64_t i = 0; i < n; ++i)
        if (species[i] < 0 || species[i] >= S) return sfail(sv, TMD_ERR_INVALID_ARGUMENT, "species out of range");
    auto sys = std::make_unique<System>();
    sys->n = n;
    for (int a = 0; a < 3; ++a) sys->box[a] = box[a];
    sys->cap = density_capacity(n, box, sv->model->rcut + sv->opts.skin, S);
    sys->state_bytes = (size_t)n * (24 * 3 + 12 + 4) + 16 * (size_t)S;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        // the resident lists can all be evicted to make room for this one
        int64_t lists = 0;
        for (auto& kv : sv->systems)
            if (kv.second->nl) lists += (int64_t)kv.second->nl_bytes;
        const int64_t need = (int64_t)sys->state_bytes + (int64_t)nlist_bytes(n, S, sys->cap, sv->opts.skin > 0.0);
        if (sv->mem_in_use - lists + need > sv->opts.hbm_budget_bytes) {
            sv->last_error = "system state does not fit in the memory budget";
            return TMD_ERR_REJECTED;
        }
        account(sv, (int64_t)sys->state_bytes);
    }
    std::vector<double> acc(S);
    for (int s = 0; s < S; ++s) acc[s] = kAccConv / masses[s];
    hipError_t e = hipSetDevice(sv->opts.device);
    auto alloc = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 256));
    };
    alloc((void**)&sys->x, 24 * (size_t)n);
    alloc((void**)&sys->v, 24 * (size_t)n);
    alloc((void**)&sys->xref, 24 * (size_t)n);
    alloc((void**)&sys->F, 12 * (size_t)n);
    alloc((void**)&sys->sp, 4 * (size_t)n);
    alloc((void**)&sys->acc, 8 * (size_t)S);
    alloc((void**)&sys->mass, 8 * (size_t)S);
    if (e == hipSuccess) e = hipMemcpy(sys->x, pos, 24 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sys->xref, pos, 24 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(sys->v, 0, 24 * (size_t)n);
    if (e == hipSuccess) e = hipMemcpy(sys->sp, species, 4 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sys->acc, acc.data(), 8 * (size_t)S, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sys->mass, masses, 8 * (size_t)S, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        for (void* p : {(void*)sys->x, (void*)sys->v, (void*)sys->xref, (void*)sys->F, (void*)sys->sp, (void*)sys->acc,
                        (void*)sys->mass})
            if (p) (void)hipFree(p);
        std::lock_guard<std::mutex> lk(sv->mu);
        account(sv, -(int64_t)sys->state_bytes);
        sv->last_error = std::string("system upload: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? TMD_ERR_OUT_OF_MEMORY : TMD_ERR_DEVICE;
    }
    admit_list(sv, sys.get());
    std::lock_guard<std::mutex> lk(sv->mu);
    sys->id = sv->next_system++;
    *system_id = sys->id;
    sv->systems[sys->id] = std::move(sys);
    return TMD_OK;
}

tmd_status tmd_serve_submit(tmd_server* sv, const tmd_request* req, uint64_t* ticket) {
    if (!sv) return TMD_ERR_INVALID_ARGUMENT;
    if (!req || !ticket) return sfail(sv, TMD_ERR_INVALID_ARGUMENT, "null argument");
    if (req->kind != TMD_REQ_ENERGY_FORCES && req->kind != TMD_REQ_MD)
        return sfail(sv, TMD_ERR_INVALID_ARGUMENT, "unknown request kind");
    if (req->kind == TMD_REQ_MD && (req->n_steps < 0 || req->n_steps > 1000000 || !(req->dt_fs > 0.0) ||
                                    !std::isfinite(req->dt_fs)))
        return sfail(sv, TMD_ERR_INVALID_ARGUMENT, "MD needs 0 <= n_steps and dt_fs > 0");
    Pending p;
    p.req = *req;
    p.req.velocities = nullptr;
    int64_t n = 0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->systems.find(req->system_id);
        if (it == sv->systems.end()) {
            sv->last_error = "unknown system id";
            return TMD_ERR_INVALID_ARGUMENT;
        }
        n = it->second->n;
    }
    if (req->kind == TMD_REQ_MD && req->velocities) p.vel.assign(req->velocities, req->velocities + 3 * n);
    std::lock_guard<std::mutex> lk(sv->mu);
    p.ticket = sv->next_ticket++;
    p.t_submit = now_s(sv->t0);
    *ticket = p.ticket;
    sv->queue.push_back(std::move(p));
    sv->cv_work.notify_one();
    return TMD_OK;
}

tmd_status tmd_serve_poll(tmd_server* sv, uint64_t ticket, tmd_result* result) {
    if (!sv || !result) return TMD_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) {
        if (ticket == 0 || ticket >= sv->next_ticket) {
            sv->last_error = "unknown ticket";
            return TMD_ERR_INVALID_ARGUMENT;
        }
        return TMD_ERR_NOT_READY;
    }
    *result = it->second.res;
    return TMD_OK;
}

tmd_status tmd_serve_wait(tmd_server* sv, uint64_t ticket, double timeout_s, tmd_result* result) {
    if (!sv || !result) return TMD_ERR_INVALID_ARGUMENT;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (ticket == 0 || ticket >= sv->next_ticket) {
        sv->last_error = "unknown ticket";
        return TMD_ERR_INVALID_ARGUMENT;
    }
    auto ready = [&] { return sv->done.count(ticket) > 0; };
    if (timeout_s < 0) sv->cv_done.wait(lk, ready);
    else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) return TMD_ERR_NOT_READY;
    *result = sv->done[ticket].res;
    return TMD_OK;
}

tmd_status tmd_serve_fetch(tmd_server* sv, uint64_t ticket, float* forces, double* pos, double* vel, double* epot,
                           double* ekin) {
    if (!sv) return TMD_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) {
        sv->last_error = "request not finished or unknown";
        return TMD_ERR_NOT_READY;
    }
    const Finished& f = it->second;
    if (f.res.status != TMD_OK) {
        sv->last_error = "request failed";
        return (tmd_status)f.res.status;
    }
    if (forces) std::memcpy(forces, f.F.data(), f.F.size() * sizeof(float));
    if (pos && !f.x.empty()) std::memcpy(pos, f.x.data(), f.x.size() * sizeof(double));
    if (vel && !f.v.empty()) std::memcpy(vel, f.v.data(), f.v.size() * sizeof(double));
    if (epot) std::memcpy(epot, f.epot.data(), f.epot.size() * sizeof(double));
    if (ekin && !f.ekin.empty()) std::memcpy(ekin, f.ekin.data(), f.ekin.size() * sizeof(double));
    return TMD_OK;
}

tmd_status tmd_serve_release(tmd_server* sv, uint64_t ticket) {
    if (!sv) return TMD_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->done.erase(ticket)) {
        sv->last_error = "request not finished or unknown";
        return TMD_ERR_INVALID_ARGUMENT;
    }
    return TMD_OK;
}

tmd_status tmd_serve_read_system(tmd_server* sv, int64_t system_id, double* pos, double* vel) {
    if (!sv) return TMD_ERR_INVALID_ARGUMENT;
    System* sys = nullptr;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->systems.find(system_id);
        if (it == sv->systems.end()) {
            sv->last_error = "unknown system id";
            return TMD_ERR_INVALID_ARGUMENT;
        }
        sys = it->second.get();
        // wait until no request on it is queued or running
        sv->cv_done.wait(lk, [&] {
            if (sys->busy) return false;
            for (const auto& q : sv->queue)
                if (q.req.system_id == system_id) return false;
            return true;
        });
        sys->busy = true;
    }
    hipError_t e = hipSetDevice(sv->opts.device);
    if (e == hipSuccess && pos) e = hipMemcpy(pos, sys->x, 24 * (size_t)sys->n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && vel) e = hipMemcpy(vel, sys->v, 24 * (size_t)sys->n, hipMemcpyDeviceToHost);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sys->busy = false;
    }
    sv->cv_work.notify_all();
    return e == hipSuccess ? TMD_OK : TMD_ERR_DEVICE;
}

tmd_status tmd_serve_memory(tmd_server* sv, int64_t* in_use, int64_t* peak) {
    if (!sv) return TMD_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (in_use) *in_use = sv->mem_in_use;
    if (peak) *peak = sv->mem_peak;
    return TMD_OK;
}

tmd_status tmd_serve_system_memory(tmd_server* sv, int64_t system_id, int64_t* state_bytes, int64_t* list_bytes) {
    if (!sv) return TMD_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->systems.find(system_id);
    if (it == sv->systems.end()) {
        sv->last_error = "unknown system id";
        return TMD_ERR_INVALID_ARGUMENT;
    }
    if (state_bytes) *state_bytes = (int64_t)it->second->state_bytes;
    if (list_bytes) *list_bytes = it->second->nl ? (int64_t)it->second->nl_bytes : 0;
    return TMD_OK;
}

const char* tmd_serve_last_error(tmd_server* sv) {
    if (!sv) return "null server";
    std::lock_guard<std::mutex> lk(sv->mu);
    return sv->last_error.c_str();
}

void tmd_serve_destroy(tmd_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->queue.clear();
    }
    sv->cv_work.notify_all();
    for (auto& t : sv->workers) t.join();
    (void)hipSetDevice(sv->opts.device);
    (void)hipDeviceSynchronize();
    destroy_lists(sv->retired);
    release_slots(sv);
    for (auto& kv : sv->systems) {
        System* s = kv.second.get();
        if (s->nl) tmd_nlist_destroy(s->nl);
        for (void* p : {(void*)s->x, (void*)s->v, (void*)s->xref, (void*)s->F, (void*)s->sp, (void*)s->acc,
                        (void*)s->mass})
            if (p) (void)hipFree(p);
    }
    delete sv;
}

}  // extern "C"
