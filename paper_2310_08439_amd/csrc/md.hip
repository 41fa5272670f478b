// Molecular dynamics on one system: velocity Verlet with an optional
// Nose-Hoover thermostat, the neighbour list rebuilt on a fixed period or when
// an atom has moved more than half the skin, and thermodynamic output
// (energies, temperature, pressure tensor) every few steps (the MD protocol of
// Sec. IV.D: NVT, 1 fs steps, a 1 A skin rebuilt every 5 steps, thermo output
// every 10 steps; the paper does not name its thermostat).  The velocity
// Verlet kernels here also serve the request loop.
//
// Thermostat: one Nose-Hoover variable xi with mass Q = g kB T tau^2
// (g = 3N) in the symmetric Trotter splitting
//   [xi += dt/4 G; v *= exp(-xi dt/2); eta += xi dt/2; xi += dt/4 G]  (half step)
//   velocity Verlet step
//   half step again,
// G = (2 KE - g kB T) / Q.  The extended energy PE + KE + Q xi^2/2 + g kB T eta
// is conserved.  All of it runs on the device; the host reads results only at
// output steps (and each step when the displacement criterion decides rebuilds).
#include "tmd_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace tmd {
namespace {

constexpr double kKeConv = 103.6427;       // amu (A/fs)^2 -> eV
constexpr double kKb = 8.617333262e-5;     // eV/K
constexpr double kEvA3ToGPa = 160.21766208;

// v += (dt/2) a; x += dt v; and (maxd2 non-null) the largest squared
// displacement since the last list build, as the bits of a non-negative
// double (ordered like the values).  Grid-stride over a few workgroups per CU,
// so that few workgroups meet at the one atomicMax.
__global__ void __launch_bounds__(256) k_kick_drift(int64_t n, double* __restrict__ x, double* __restrict__ v,
                                                    const float* __restrict__ F, const int32_t* __restrict__ sp,
                                                    const double* __restrict__ acc, double dt,
                                                    const double* __restrict__ xref,
                                                    unsigned long long* __restrict__ maxd2) {
    __shared__ double red[256];
    double d2 = 0.0;  // largest over this thread's atoms
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = acc[sp[i]];
        double di = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double vi = v[3 * i + c] + 0.5 * dt * a * (double)F[3 * i + c];
            const double xi = x[3 * i + c] + dt * vi;
            v[3 * i + c] = vi;
            x[3 * i + c] = xi;
            if (maxd2) {
                const double d = xi - xref[3 * i + c];
                di += d * d;
            }
        }
        d2 = fmax(d2, di);
    }
    if (!maxd2) return;  // uniform over the grid
    red[threadIdx.x] = d2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(maxd2, (unsigned long long)__double_as_longlong(red[0]));
}

// v += (dt/2) a
__global__ void k_kick(int64_t n, double* __restrict__ v, const float* __restrict__ F,
                       const int32_t* __restrict__ sp, const double* __restrict__ acc, double dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = acc[sp[i]];
    for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * dt * a * (double)F[3 * i + c];
}

// Kinetic energy tensor diagonal in two fixed-order passes: kKeBlocks strided
// partials, then compensated sums.
__global__ void __launch_bounds__(256) k_ke_partials(int64_t n, const double* __restrict__ v,
                                                     const int32_t* __restrict__ sp,
                                                     const double* __restrict__ mass, double* __restrict__ part) {
    __shared__ double red[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double hm = 0.5 * kKeConv * mass[sp[i]];
        for (int c = 0; c < 3; ++c) s[c] += hm * v[3 * i + c] * v[3 * i + c];
    }
    for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Sum of the nb (<= 256) block partials per component: one workgroup, a fixed
// pairwise tree of compensated (Neumaier) merges, so the result is the same
// run to run.
__global__ void __launch_bounds__(256) k_ke_total(const double* __restrict__ part, int nb, double* __restrict__ out4) {
    __shared__ double rs[3][256], rc[3][256];
    const int t = threadIdx.x;
    for (int c = 0; c < 3; ++c) {
        rs[c][t] = t < nb ? part[3 * t + c] : 0.0;
        rc[c][t] = 0.0;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int c = 0; c < 3; ++c) {
                const double x = rs[c][t], y = rs[c][t + w], s = x + y;
                const double e = fabs(x) >= fabs(y) ? (x - s) + y : (y - s) + x;
                rs[c][t] = s;
                rc[c][t] += rc[c][t + w] + e;
            }
        __syncthreads();
    }
    if (t == 0) {
        double tot = 0.0;
        for (int c = 0; c < 3; ++c) {
            out4[c] = rs[c][0] + rc[c][0];
            tot += out4[c];
        }
        out4[3] = tot;
    }
}

// Thermostat half step on the device: state = (xi, eta, scale); ke4 is the
// kinetic tensor before the scaling and is rescaled in place.
__global__ void k_nh_half(double* __restrict__ state, double* __restrict__ ke4, double g, double kT, double Q,
                          double dt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double xi = state[0], eta = state[1];
    double ke = ke4[3];
    xi += 0.25 * dt * (2.0 * ke - g * kT) / Q;
    const double s = exp(-xi * 0.5 * dt);
    ke *= s * s;
    eta += 0.5 * dt * xi;
    xi += 0.25 * dt * (2.0 * ke - g * kT) / Q;
    state[0] = xi;
    state[1] = eta;
    state[2] = s;
    for (int c = 0; c < 3; ++c) ke4[c] *= s * s;
    ke4[3] = ke;
}

__global__ void k_scale_v(int64_t n3, double* __restrict__ v, const double* __restrict__ state) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) v[i] *= state[2];
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

tmd_status launch_kick_drift(tmd_context* ctx, int64_t n, double* x, double* v, const float* F, const int32_t* sp,
                             const double* acc, double dt, const double* xref, unsigned long long* maxd2) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_of(n), 4 * (int64_t)ctx->num_cus));
    k_kick_drift<<<grid, kBlock, 0, ctx->stream>>>(n, x, v, F, sp, acc, dt, xref, maxd2);
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// flag |= (largest squared displacement > limit2); maxd2 holds the bits of a
// non-negative double, whose order is that of the bits.
__global__ void k_displacement_check(const unsigned long long* __restrict__ maxd2, double limit2,
                                     unsigned long long* __restrict__ flag) {
    if (threadIdx.x != 0) return;
    if (__longlong_as_double((long long)*maxd2) > limit2) *flag = 1ull;
}

tmd_status launch_zero_u64(tmd_context* ctx, unsigned long long* p, int64_t n) {
    if (n <= 0) return TMD_OK;
    k_zero_u64<<<blocks_of(n), kBlock, 0, ctx->stream>>>(p, n);
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status launch_displacement_check(tmd_context* ctx, const unsigned long long* maxd2, double limit2, unsigned long long* flag) {
    k_displacement_check<<<1, 64, 0, ctx->stream>>>(maxd2, limit2, flag);
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status launch_kick(tmd_context* ctx, int64_t n, double* v, const float* F, const int32_t* sp, const double* acc,
                       double dt) {
    k_kick<<<blocks_of(n), kBlock, 0, ctx->stream>>>(n, v, F, sp, acc, dt);
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

tmd_status launch_kinetic(tmd_context* ctx, int64_t n, const double* v, const int32_t* sp, const double* mass,
                          double* part, double* out4) {
    k_ke_partials<<<kKeBlocks, 256, 0, ctx->stream>>>(n, v, sp, mass, part);
    static_assert(kKeBlocks <= 256, "k_ke_total sums at most 256 partials");
    k_ke_total<<<1, 256, 0, ctx->stream>>>(part, kKeBlocks, out4);
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace tmd

struct tmd_md {
    tmd_context* ctx = nullptr;
    const tmd_model* model = nullptr;
    tmd_md_opts opts{};
    int64_t n = 0;
    int S = 0;
    double box[3] = {0, 0, 0};
    double g = 0.0, kT = 0.0, Q = 0.0;
    int64_t step = 0;
    bool started = false;
    int64_t steps_since_build = 0;
    int32_t rebuilds = 0;
    tmd_nlist* nl = nullptr;
    // device
    double* x = nullptr;
    double* v = nullptr;
    double* xref = nullptr;
    float* F = nullptr;
    int32_t* sp = nullptr;
    double* acc = nullptr;
    double* mass = nullptr;
    double* tot7 = nullptr;     // E, virial (xx, yy, zz, xy, xz, yz)
    double* ke4 = nullptr;      // kinetic tensor diagonal + total
    double* state = nullptr;    // xi, eta, scale
    double* part = nullptr;     // kinetic partials
    unsigned long long* maxd2 = nullptr;
};

namespace tmd {
namespace {

void md_free(tmd_md* md) {
    if (md->nl) tmd_nlist_destroy(md->nl);
    for (void* p : {(void*)md->x, (void*)md->v, (void*)md->xref, (void*)md->F, (void*)md->sp, (void*)md->acc,
                    (void*)md->mass, (void*)md->tot7, (void*)md->ke4, (void*)md->state, (void*)md->part,
                    (void*)md->maxd2})
        if (p) (void)hipFree(p);
}

tmd_system_view md_view(const tmd_md* md) {
    tmd_system_view v{};
    v.n_atoms = md->n;
    v.pos = md->x;
    v.species = md->sp;
    for (int a = 0; a < 3; ++a) v.box[a] = md->box[a];
    return v;
}

tmd_status md_build(tmd_md* md) {
    tmd_context* ctx = md->ctx;
    tmd_system_view v = md_view(md);
    for (int attempt = 0; attempt < 4; ++attempt) {
        int32_t need = 0;
        tmd_status st = tmd_build_neighbors(ctx, &v, md->model->rcut, md->opts.skin, md->nl, &need);
        if (st == TMD_OK) {
            TMD_HIP(ctx, hipMemcpyAsync(md->xref, md->x, 24 * (size_t)md->n, hipMemcpyDeviceToDevice, ctx->stream));
            md->steps_since_build = 0;
            ++md->rebuilds;
            return TMD_OK;
        }
        if (st != TMD_ERR_CAPACITY) return st;
        tmd_nlist* nl = nullptr;
        if ((st = tmd_nlist_create(ctx, md->n, md->S, (need + 8 + 7) / 8 * 8, &nl)) != TMD_OK) return st;
        tmd_nlist_destroy(md->nl);
        md->nl = nl;
    }
    return fail(ctx, TMD_ERR_CAPACITY, "neighbour list kept overflowing");
}

tmd_status md_thermo(tmd_md* md, tmd_thermo* out) {
    tmd_context* ctx = md->ctx;
    double h[14];
    TMD_HIP(ctx, hipMemcpyAsync(h, md->tot7, sizeof(double) * 7, hipMemcpyDeviceToHost, ctx->stream));
    TMD_HIP(ctx, hipMemcpyAsync(h + 7, md->ke4, sizeof(double) * 4, hipMemcpyDeviceToHost, ctx->stream));
    TMD_HIP(ctx, hipMemcpyAsync(h + 11, md->state, sizeof(double) * 3, hipMemcpyDeviceToHost, ctx->stream));
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double V = md->box[0] * md->box[1] * md->box[2];
    tmd_thermo t{};
    t.step = md->step;
    t.time_fs = (double)md->step * md->opts.dt_fs;
    t.epot = h[0];
    t.ekin = h[10];
    t.etotal = h[0] + h[10];
    t.temperature_K = 2.0 * h[10] / (md->g * kKb);
    t.volume_A3 = V;
    t.pxx_GPa = (2.0 * h[7] + h[1]) / V * kEvA3ToGPa;
    t.pyy_GPa = (2.0 * h[8] + h[2]) / V * kEvA3ToGPa;
    t.pzz_GPa = (2.0 * h[9] + h[3]) / V * kEvA3ToGPa;
    t.pressure_GPa = (t.pxx_GPa + t.pyy_GPa + t.pzz_GPa) / 3.0;
    t.xi = h[11];
    t.conserved = t.etotal;
    if (md->opts.ensemble == TMD_ENSEMBLE_NVT_NOSE_HOOVER)
        t.conserved += 0.5 * md->Q * h[11] * h[11] + md->g * md->kT * h[12];
    t.rebuilds = md->rebuilds;
    *out = t;
    return TMD_OK;
}

// Skin lists are pruned to the cutoff plus a fifth of the skin and reused
// while the displacements since the build allow (PruneGate); maxd2 holds the
// largest squared displacement since the build for the current positions.
PruneGate md_gate(const tmd_md* md) {
    PruneGate g;
    g.maxd2 = md->maxd2;
    g.margin = 0.2 * md->opts.skin;
    return g;
}

tmd_status md_energy_forces(tmd_md* md) {
    tmd_system_view v = md_view(md);
    const PruneGate g = md_gate(md);
    return energy_forces_gated(md->ctx, md->model, &v, md->nl, md->tot7, nullptr, md->F,
                               md->opts.skin > 0.0 ? &g : nullptr);
}

// Energy, forces and kinetic tensor at the current state.
tmd_status md_evaluate(tmd_md* md) {
    tmd_context* ctx = md->ctx;
    tmd_status st = md_energy_forces(md);
    if (st != TMD_OK) return st;
    return launch_kinetic(ctx, md->n, md->v, md->sp, md->mass, md->part, md->ke4);
}

tmd_status md_thermostat(tmd_md* md) {
    if (md->opts.ensemble != TMD_ENSEMBLE_NVT_NOSE_HOOVER) return TMD_OK;
    tmd_context* ctx = md->ctx;
    k_nh_half<<<1, 64, 0, ctx->stream>>>(md->state, md->ke4, md->g, md->kT, md->Q, md->opts.dt_fs);
    k_scale_v<<<blocks_of(3 * md->n), kBlock, 0, ctx->stream>>>(3 * md->n, md->v, md->state);
    TMD_HIP(ctx, hipGetLastError());
    return TMD_OK;
}

}  // namespace
}  // namespace tmd

using namespace tmd;

extern "C" {

tmd_status tmd_md_create(tmd_context* ctx, const tmd_model* model, const tmd_system_view* sys, const double* masses,
                         const double* velocities, const tmd_md_opts* opts, tmd_md** out) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    if (!model || !sys || !masses || !opts || !out) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null argument");
    *out = nullptr;
    if (!sys->pos || !sys->species || sys->n_atoms <= 0) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "bad system");
    if (!(opts->dt_fs > 0.0) || !std::isfinite(opts->dt_fs)) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "dt must be positive");
    if (!(opts->skin >= 0.0) || !std::isfinite(opts->skin)) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "skin must be >= 0");
    if (opts->rebuild_every < 0) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "rebuild_every must be >= 0");
    if (opts->ensemble != TMD_ENSEMBLE_NVE && opts->ensemble != TMD_ENSEMBLE_NVT_NOSE_HOOVER)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "unknown ensemble");
    if (opts->ensemble == TMD_ENSEMBLE_NVT_NOSE_HOOVER && !(opts->temperature_K > 0.0 && opts->tau_fs > 0.0))
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "NVT needs temperature and tau > 0");
    for (int s = 0; s < model->S; ++s)
        if (!(masses[s] > 0.0) || !std::isfinite(masses[s])) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "bad mass");
    tmd_md* md = new (std::nothrow) tmd_md();
    if (!md) return fail(ctx, TMD_ERR_OUT_OF_MEMORY, "host allocation");
    md->ctx = ctx;
    md->model = model;
    md->opts = *opts;
    md->n = sys->n_atoms;
    md->S = model->S;
    for (int a = 0; a < 3; ++a) md->box[a] = sys->box[a];
    md->g = 3.0 * (double)md->n;
    md->kT = kKb * opts->temperature_K;
    md->Q = md->g * md->kT * opts->tau_fs * opts->tau_fs;
    const size_t n = (size_t)md->n;
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 256));
    };
    alloc((void**)&md->x, 24 * n);
    alloc((void**)&md->v, 24 * n);
    alloc((void**)&md->xref, 24 * n);
    alloc((void**)&md->F, 12 * n);
    alloc((void**)&md->sp, 4 * n);
    alloc((void**)&md->acc, 8 * (size_t)md->S);
    alloc((void**)&md->mass, 8 * (size_t)md->S);
    alloc((void**)&md->tot7, 8 * 8);
    alloc((void**)&md->ke4, 8 * 4);
    alloc((void**)&md->state, 8 * 4);
    alloc((void**)&md->part, 8 * 3 * (size_t)kKeBlocks);
    alloc((void**)&md->maxd2, 8);
    std::vector<double> acc(md->S);
    for (int s = 0; s < md->S; ++s) acc[s] = 9.648533e-3 / masses[s];
    const double st0[4] = {0.0, 0.0, 1.0, 0.0};
    if (e == hipSuccess) e = hipMemcpyAsync(md->x, sys->pos, 24 * n, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(md->sp, sys->species, 4 * n, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess)
        e = velocities ? hipMemcpyAsync(md->v, velocities, 24 * n, hipMemcpyDeviceToDevice, ctx->stream)
                       : hipMemsetAsync(md->v, 0, 24 * n, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(md->acc, acc.data(), 8 * (size_t)md->S, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(md->mass, masses, 8 * (size_t)md->S, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(md->state, st0, sizeof(st0), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(md->maxd2, 0, 8, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    tmd_status st = e == hipSuccess ? TMD_OK : hip_fail(ctx, e, "MD allocation");
    if (st == TMD_OK) {
        const double vol = md->box[0] * md->box[1] * md->box[2];
        const double rl = model->rcut + opts->skin;
        const double mean = (double)md->n / vol * 4.0 / 3.0 * M_PI * rl * rl * rl;
        const int cap = std::max(16, ((int)(mean * (1.0 / md->S + 0.3)) + 16 + 7) / 8 * 8);
        st = tmd_nlist_create(ctx, md->n, md->S, cap, &md->nl);
    }
    if (st == TMD_OK) st = md_build(md);
    if (st == TMD_OK) st = md_evaluate(md);
    if (st != TMD_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        md_free(md);
        delete md;
        return st;
    }
    *out = md;
    return TMD_OK;
}

tmd_status tmd_md_run(tmd_md* md, int64_t n_steps, int32_t thermo_every, tmd_thermo* thermo, int32_t thermo_capacity,
                      int32_t* n_thermo) {
    if (!md) return TMD_ERR_INVALID_ARGUMENT;
    tmd_context* ctx = md->ctx;
    if (n_steps < 0 || thermo_every < 0 || (thermo_every > 0 && (!thermo || thermo_capacity < 0)))
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "bad run arguments");
    int32_t nt = 0;
    auto record = [&]() -> tmd_status {
        if (thermo_every <= 0 || md->step % thermo_every != 0 || nt >= thermo_capacity) return TMD_OK;
        return md_thermo(md, &thermo[nt++]);
    };
    tmd_status st = TMD_OK;
    if (!md->started) {
        md->started = true;
        if ((st = record()) != TMD_OK) return st;
    }
    const double dt = md->opts.dt_fs, half_skin2 = 0.25 * md->opts.skin * md->opts.skin;
    const bool by_distance = md->opts.rebuild_every == 0;
    for (int64_t s = 0; s < n_steps; ++s) {
        if ((st = md_thermostat(md)) != TMD_OK) return st;
        // the displacement since the build decides rebuilds (by_distance) and
        // whether the pruned rows can be reused
        TMD_HIP(ctx, hipMemsetAsync(md->maxd2, 0, 8, ctx->stream));
        if ((st = launch_kick_drift(ctx, md->n, md->x, md->v, md->F, md->sp, md->acc, dt, md->xref, md->maxd2)) !=
            TMD_OK)
            return st;
        ++md->steps_since_build;
        bool rebuild = false;
        if (by_distance) {
            TMD_HIP(ctx, hipMemcpyAsync(ctx->h_flags, md->maxd2, 8, hipMemcpyDeviceToHost, ctx->stream));
            TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
            double d2;
            std::memcpy(&d2, ctx->h_flags, sizeof(d2));
            rebuild = !(d2 <= half_skin2);
        } else {
            rebuild = md->steps_since_build >= md->opts.rebuild_every;
        }
        if (rebuild && (st = md_build(md)) != TMD_OK) return st;
        if ((st = md_energy_forces(md)) != TMD_OK) return st;
        if ((st = launch_kick(ctx, md->n, md->v, md->F, md->sp, md->acc, dt)) != TMD_OK) return st;
        if ((st = launch_kinetic(ctx, md->n, md->v, md->sp, md->mass, md->part, md->ke4)) != TMD_OK) return st;
        if ((st = md_thermostat(md)) != TMD_OK) return st;
        ++md->step;
        if ((st = record()) != TMD_OK) return st;
    }
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (n_thermo) *n_thermo = nt;
    return TMD_OK;
}

tmd_status tmd_md_read(tmd_md* md, double* pos, double* vel) {
    if (!md) return TMD_ERR_INVALID_ARGUMENT;
    tmd_context* ctx = md->ctx;
    if (pos) TMD_HIP(ctx, hipMemcpyAsync(pos, md->x, 24 * (size_t)md->n, hipMemcpyDeviceToDevice, ctx->stream));
    if (vel) TMD_HIP(ctx, hipMemcpyAsync(vel, md->v, 24 * (size_t)md->n, hipMemcpyDeviceToDevice, ctx->stream));
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return TMD_OK;
}

tmd_status tmd_md_thermostat_state(tmd_md* md, double* xi_eta) {
    if (!md || !xi_eta) return TMD_ERR_INVALID_ARGUMENT;
    tmd_context* ctx = md->ctx;
    TMD_HIP(ctx, hipMemcpyAsync(xi_eta, md->state, 16, hipMemcpyDeviceToHost, ctx->stream));
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return TMD_OK;
}

void tmd_md_destroy(tmd_md* md) {
    if (!md) return;
    (void)hipDeviceSynchronize();  // (not the context's stream: the handle does not keep its context alive)
    md_free(md);
    delete md;
}

}  // extern "C"
