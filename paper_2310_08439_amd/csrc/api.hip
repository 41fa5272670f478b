// C ABI of libtmd.so (declared in include/tmd.h): handle management, argument
// validation and the order of the kernels on the context's stream.
#include "tmd_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

namespace tmd {

void* Workspace::get(const std::string& key, size_t bytes, hipError_t* err) {
    if (*err != hipSuccess) return nullptr;
    bytes = std::max<size_t>(bytes, 256);
    auto it = bufs.find(key);
    if (it != bufs.end() && it->second.second >= bytes) return it->second.first;
    if (it != bufs.end()) {
        // the old buffer may still be read by queued work
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) { *err = e; return nullptr; }
        (void)hipFree(it->second.first);
        bufs.erase(it);
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    bufs[key] = {p, bytes};
    return p;
}

void Workspace::release() {
    for (auto& kv : bufs) (void)hipFree(kv.second.first);
    bufs.clear();
}

hipEvent_t Profiler::get_event() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void Profiler::collect() {
    for (auto& r : pending) {
        float ms = 0.0f;
        (void)hipEventSynchronize(r.stop);
        (void)hipEventElapsedTime(&ms, r.start, r.stop);
        size_t q = 0;
        while (q < names.size() && names[q] != r.name) ++q;
        if (q == names.size()) {
            names.push_back(r.name);
            total_ms.push_back(0.0);
            count.push_back(0);
        }
        total_ms[q] += ms;
        count[q] += 1;
        pool.push_back(r.start);
        pool.push_back(r.stop);
    }
    pending.clear();
}

void Profiler::release() {
    collect();
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
}

tmd_status fail(tmd_context* ctx, tmd_status st, const std::string& msg) {
    if (ctx) ctx->last_error = msg;
    return st;
}

tmd_status hip_fail(tmd_context* ctx, hipError_t e, const char* what) {
    const tmd_status st = (e == hipErrorOutOfMemory) ? TMD_ERR_OUT_OF_MEMORY : TMD_ERR_DEVICE;
    return fail(ctx, st, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

uint16_t float_to_bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);  // NaN
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int choose_kc(int K) {
    for (int kc : {8, 6, 4})
        if (K % kc == 0 && is_pow2(K / kc) && K / kc <= 64) return kc;
    return 0;
}

// Radial functions the kernels run for a model of K: the smallest 4, 6 or 8
// times a power of two that is at least K (so that K/kc chunks of kc radial
// functions cover them; at most 128).
int padded_k(int K) {
    for (int k = std::max(K, 4); k <= 128; ++k)
        if (choose_kc(k)) return k;
    return 0;
}

// Hidden width the kernels run: the widest layer rounded up to 32, 64 or 128.
int padded_h(const int* hid, int L) {
    int w = 0;
    for (int l = 0; l < L; ++l) w = std::max(w, hid[l]);
    for (int h : {32, 64, 128})
        if (w <= h) return h;
    return 0;
}

// The operand copies of every species (W, W^T in FP32 and BF16 at the padded
// sizes, biases, output layer) and the padded master copy, from ABI-layout
// parameters; every padded entry is zero.
tmd_status upload_params(tmd_model* m, const float* params) {
    tmd_context* ctx = m->ctx;
    const int S = m->S, L = m->L, H = m->H, Fpad = m->Fpad;
    const ParamMap pm = param_map(m);
    std::vector<float> w32((size_t)S * m->w_species_stride, 0.0f);
    std::vector<float> bias((size_t)S * L * H, 0.0f), wout((size_t)S * H, 0.0f), bout(S, 0.0f);
    std::vector<float> pint(m->padded ? (size_t)S * m->per_species_int : 0, 0.0f);
    for (int s = 0; s < S; ++s) {
        const float* p = params + (size_t)s * m->per_species;
        float* ws = w32.data() + (size_t)s * m->w_species_stride;
        for (int64_t q = 0; q < m->per_species; ++q) {
            int l, o, c, kind;
            const int64_t qi = pm.map(q, l, o, c, kind);
            const float v = p[q];
            if (m->padded) pint[(size_t)s * m->per_species_int + qi] = v;
            if (kind == 0) {
                const int in_pad = (l == 0) ? Fpad : H;
                ws[m->w_off[l] + (size_t)o * in_pad + c] = v;
                ws[m->wt_off[l] + (size_t)c * H + o] = v;
            } else if (kind == 1) {
                bias[((size_t)s * L + l) * H + o] = v;
            } else if (kind == 2) {
                wout[(size_t)s * H + o] = v;
            } else {
                bout[s] = v;
            }
        }
    }
    std::vector<uint16_t> wbf(w32.size());
    for (size_t q = 0; q < w32.size(); ++q) wbf[q] = float_to_bf16_rne(w32[q]);
    TMD_HIP(ctx, hipMemcpy(m->w32, w32.data(), w32.size() * 4, hipMemcpyHostToDevice));
    TMD_HIP(ctx, hipMemcpy(m->wbf, wbf.data(), wbf.size() * 2, hipMemcpyHostToDevice));
    TMD_HIP(ctx, hipMemcpy(m->bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice));
    TMD_HIP(ctx, hipMemcpy(m->wout, wout.data(), wout.size() * 4, hipMemcpyHostToDevice));
    TMD_HIP(ctx, hipMemcpy(m->bout, bout.data(), bout.size() * 4, hipMemcpyHostToDevice));
    TMD_HIP(ctx, hipMemcpy(m->params32, params, (size_t)S * m->per_species * 4, hipMemcpyHostToDevice));
    if (m->padded) TMD_HIP(ctx, hipMemcpy(m->params_int, pint.data(), pint.size() * 4, hipMemcpyHostToDevice));
    return TMD_OK;
}

tmd_status check_system(tmd_context* ctx, const tmd_system_view* sys) {
    if (!sys || !sys->pos || !sys->species) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null system pointer");
    if (sys->n_atoms <= 0) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "n_atoms must be positive");
    if (sys->n_atoms >= (int64_t)1 << 31) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "more than 2^31-1 atoms");
    for (int a = 0; a < 3; ++a)
        if (!(sys->box[a] > 0.0) || !std::isfinite(sys->box[a]))
            return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "box edges must be positive and finite");
    return TMD_OK;
}

tmd_status check_eval(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys, const tmd_nlist* nl) {
    if (!m || !nl) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null model or neighbour list");
    tmd_status st = check_system(ctx, sys);
    if (st != TMD_OK) return st;
    if (!nl->built) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "neighbour list has not been built");
    if (nl->n != sys->n_atoms) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "neighbour list built for another atom count");
    if (nl->S != m->S) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "neighbour list and model species counts differ");
    for (int a = 0; a < 3; ++a)
        if (nl->box[a] != sys->box[a])
            return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "box changed since the neighbour list was built");
    if (nl->rlist < m->rcut) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "neighbour list cutoff below the model cutoff");
    return TMD_OK;
}

struct EvalBuffers {
    float *G, *dG, *Ei, *P;
    unsigned long long* Fq;  // fixed-point force accumulators [n][3]
    double *vir, *totals, *part;
};

tmd_status eval_buffers(tmd_context* ctx, const tmd_model* m, const tmd_nlist* nl, EvalBuffers* b) {
    const int64_t n = nl->n;
    hipError_t e = hipSuccess;
    b->G = (float*)ctx->ws.get("ev.G", sizeof(float) * n * m->F, &e);
    b->dG = (float*)ctx->ws.get("ev.dG", sizeof(float) * n * m->F, &e);
    b->Ei = (float*)ctx->ws.get("ev.Ei", sizeof(float) * n, &e);
    b->Fq = (unsigned long long*)ctx->ws.get("ev.Fq", sizeof(unsigned long long) * 3 * n, &e);
    b->P = (float*)ctx->ws.get("ev.P", sizeof(float) * (size_t)p_slots(m, nl) * m->S * m->K * m->Dr, &e);
    b->vir = (double*)ctx->ws.get("ev.vir", sizeof(double) * kVirDoubles * (size_t)adjoint_max_partials(m, nl), &e);
    b->totals = (double*)ctx->ws.get("ev.totals", sizeof(double) * 8, &e);
    b->part = (double*)ctx->ws.get("ev.part", sizeof(double) * finalize_part_doubles(), &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "evaluation workspace allocation");
    return TMD_OK;
}

// Scratch of tmd_energy_forces_noalloc: one array per device (each device
// that loads the library holds its own copy until the process ends).  In host
// code `scratch` names a host-side stand-in, not device memory: host code uses
// only the address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::unordered_map<int, unsigned char*> g_scratch_addr;

// Device address of `scratch` on `device` (current), looked up once per
// device; nullptr when the lookup fails.
unsigned char* scratch_address(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) return it->second;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) ptr = nullptr;
    g_scratch_addr[device] = (unsigned char*)ptr;
    return (unsigned char*)ptr;
}

// Evaluation buffers carved from the scratch array, 256-byte aligned; the
// bytes they need in *need (more than kScratchBytes: nothing is carved).
void scratch_buffers(unsigned char* base, const tmd_model* m, const tmd_nlist* nl, EvalBuffers* b, size_t* need) {
    const int64_t n = nl->n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t oG = take(sizeof(float) * n * m->F), odG = take(sizeof(float) * n * m->F);
    const size_t oEi = take(sizeof(float) * n), oFq = take(sizeof(unsigned long long) * 3 * n);
    const size_t oP = take(sizeof(float) * (size_t)p_slots(m, nl) * m->S * m->K * m->Dr);
    const size_t ovir = take(sizeof(double) * kVirDoubles * (size_t)adjoint_max_partials(m, nl));
    const size_t opart = take(sizeof(double) * finalize_part_doubles());
    *need = off;
    if (off > kScratchBytes) return;
    b->G = (float*)(base + oG);
    b->dG = (float*)(base + odG);
    b->Ei = (float*)(base + oEi);
    b->Fq = (unsigned long long*)(base + oFq);
    b->P = (float*)(base + oP);
    b->vir = (double*)(base + ovir);
    b->part = (double*)(base + opart);
    b->totals = nullptr;
}

}  // namespace

tmd_status reserve_eval_workspace(tmd_context* ctx, const tmd_model* m, int64_t n) {
    hipError_t e = hipSuccess;
    const int64_t nch = m->K / m->kc;
    (void)ctx->ws.get("ev.G", sizeof(float) * n * m->F, &e);
    (void)ctx->ws.get("ev.dG", sizeof(float) * n * m->F, &e);
    (void)ctx->ws.get("ev.Ei", sizeof(float) * n, &e);
    (void)ctx->ws.get("ev.Fq", sizeof(unsigned long long) * 3 * n, &e);
    (void)ctx->ws.get("ev.P", sizeof(float) * (size_t)p_slots_reserve(n) * m->S * m->K * m->Dr, &e);
    (void)ctx->ws.get("ev.vir",
                      sizeof(double) * kVirDoubles * (size_t)std::max<int64_t>(4 * n + 64, (n * nch + kBlock - 1) / kBlock),
                      &e);
    (void)ctx->ws.get("ev.totals", sizeof(double) * 8, &e);
    (void)ctx->ws.get("ev.part", sizeof(double) * finalize_part_doubles(), &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "evaluation workspace allocation");
    return TMD_OK;
}

size_t eval_workspace_bytes(const tmd_model* m, int64_t n) {
    const int64_t nch = m->K / m->kc;
    return (size_t)n * (8 * m->F + 4 + 24) + (size_t)p_slots_reserve(n) * 4 * m->S * m->K * m->Dr +
           8 * kVirDoubles * (size_t)std::max<int64_t>(4 * n + 64, (n * nch + kBlock - 1) / kBlock) +
           8 * finalize_part_doubles() + 64;
}

namespace {

tmd_status run_energy_forces_in(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys,
                                const tmd_nlist* nl, const EvalBuffers& b, double* totals7_dev, float* atom_energy,
                                float* forces, const PruneGate* gate) {
    tmd_status st;
    if ((st = launch_refresh_positions(ctx, sys, nl)) != TMD_OK) return st;
    // A list with a skin carries ~(1 + skin/rc)^3 - 1 more entries than the
    // cutoff needs (60 % for 1 A on 6 A); the descriptor and adjoint loops
    // then run over rows pruned to the cutoff at the current positions.
    const tmd_nlist* use = nl;
    tmd_nlist pruned;
    if (nl->rlist > m->rcut * (1.0 + 1e-9)) {
        tmd_nlist* mnl = const_cast<tmd_nlist*>(nl);  // the pruned rows are scratch owned by the list
        st = gate ? launch_prune_gated(ctx, mnl, m->rcut, *gate) : launch_prune(ctx, mnl, m->rcut);
        if (st != TMD_OK) return st;
        pruned = *nl;  // a view: same atoms, cells and work order, pruned rows
        pruned.nbr = nl->pnbr;
        pruned.img = nl->pimg;
        pruned.cnt = nl->pcnt;
        use = &pruned;
    }
    // a BF16 MLP takes its operand as BF16 descriptors, stored in the first
    // half of the FP32 descriptor buffer
    uint16_t* Gb = m->prec == TMD_BF16_MLP ? reinterpret_cast<uint16_t*>(b.G) : nullptr;
    if ((st = launch_descriptors(ctx, m, use, b.G, b.P, Gb)) != TMD_OK) return st;
    if ((st = launch_mlp(ctx, m, species_groups(nl), m->prec, b.G, Gb, b.Ei, b.dG)) != TMD_OK) return st;
    int nvir = 0;
    if ((st = launch_adjoint(ctx, m, use, b.dG, b.P, b.Fq, b.vir, &nvir)) != TMD_OK) return st;
    return launch_finalize(ctx, nl, b.Ei, b.Fq, b.vir, nvir, atom_energy, forces, totals7_dev ? totals7_dev : b.totals,
                           b.part);
}

tmd_status run_energy_forces(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys, const tmd_nlist* nl,
                             double* totals7_dev, float* atom_energy, float* forces, const PruneGate* gate = nullptr) {
    EvalBuffers b;
    tmd_status st = eval_buffers(ctx, m, nl, &b);
    if (st != TMD_OK) return st;
    return run_energy_forces_in(ctx, m, sys, nl, b, totals7_dev, atom_energy, forces, gate);
}

}  // namespace
}  // namespace tmd

using namespace tmd;

extern "C" {

tmd_status tmd_context_create(int device, void* hip_stream, tmd_context** out) {
    if (!out) return TMD_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TMD_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return TMD_ERR_DEVICE;
    tmd_context* ctx = new (std::nothrow) tmd_context();
    if (!ctx) return TMD_ERR_OUT_OF_MEMORY;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        ctx->num_cus = cus;
    ctx->scratch = scratch_address(device);  // with `device` current
    if (hipHostMalloc((void**)&ctx->h_totals, sizeof(double) * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_flags, sizeof(int32_t) * 64, hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return TMD_ERR_OUT_OF_MEMORY;
    }
    *out = ctx;
    return TMD_OK;
}

void tmd_context_destroy(tmd_context* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->ws.release();
    ctx->prof.release();
    if (ctx->h_totals) (void)hipHostFree(ctx->h_totals);
    if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
    delete ctx;
}

tmd_status tmd_context_set_stream(tmd_context* ctx, void* hip_stream) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    ctx->stream = (hipStream_t)hip_stream;
    return TMD_OK;
}

const char* tmd_last_error(const tmd_context* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

tmd_status tmd_profile_enable(tmd_context* ctx, int on) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    ctx->prof.on = on != 0;
    return TMD_OK;
}

tmd_status tmd_profile_reset(tmd_context* ctx) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    ctx->prof.collect();
    ctx->prof.names.clear();
    ctx->prof.total_ms.clear();
    ctx->prof.count.clear();
    return TMD_OK;
}

int32_t tmd_profile_read(tmd_context* ctx, int32_t max_kernels, char* names, double* total_ms, int64_t* count) {
    if (!ctx) return 0;
    ctx->prof.collect();
    const int32_t n = (int32_t)ctx->prof.names.size();
    for (int32_t q = 0; q < n && q < max_kernels; ++q) {
        if (names) {
            std::memset(names + 32 * q, 0, 32);
            std::strncpy(names + 32 * q, ctx->prof.names[q].c_str(), 31);
        }
        if (total_ms) total_ms[q] = ctx->prof.total_ms[q];
        if (count) count[q] = ctx->prof.count[q];
    }
    return n;
}

tmd_status tmd_model_create(tmd_context* ctx, const tmd_model_spec* spec, const float* params, tmd_model** out) {
    if (!ctx || !spec || !params || !out) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null argument");
    *out = nullptr;
    const int S = spec->n_species, Kabi = spec->n_radial, M = spec->max_moment, L = spec->n_hidden;
    if (S < 1 || S > kMaxSpecies) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "n_species must be in 1..8");
    if (Kabi < 1 || Kabi > 128) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "n_radial must be in 1..128");
    if (M < 0 || M > 3) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "max_moment must be in 0..3");
    if (L < 1 || L > TMD_MAX_HIDDEN) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "n_hidden must be in 1..4");
    for (int l = 0; l < L; ++l)
        if (spec->hidden[l] < 1 || spec->hidden[l] > 128)
            return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "hidden widths must be in 1..128");
    if (spec->activation != TMD_ACT_TANH && spec->activation != TMD_ACT_SQUAREPLUS)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "unknown activation");
    if (!(spec->rcut > 0.0) || !std::isfinite(spec->rcut)) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "rcut must be positive");
    if (!spec->mu || !spec->eta) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null mu or eta");
    for (int k = 0; k < Kabi; ++k)
        if (!std::isfinite(spec->mu[k]) || !(spec->eta[k] >= 0.0) || !std::isfinite(spec->eta[k]))
            return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "mu must be finite and eta finite and non-negative");
    const int K = padded_k(Kabi), H = padded_h(spec->hidden, L);
    const int kc = choose_kc(K);
    tmd_model* m = new (std::nothrow) tmd_model();
    if (!m) return fail(ctx, TMD_ERR_OUT_OF_MEMORY, "host allocation");
    m->ctx = ctx;
    m->S = S;
    m->K = K;
    m->Kabi = Kabi;
    m->M = M;
    m->D = (M + 1) * (M + 2) * (M + 3) / 6;
    m->Dr = M == 3 ? 16 : (M == 2 ? 9 : m->D);
    m->F = S * K * (M + 1);
    m->Fabi = S * Kabi * (M + 1);
    m->Fpad = (m->F + 31) / 32 * 32;
    m->L = L;
    m->H = H;
    for (int l = 0; l < L; ++l) m->hid[l] = spec->hidden[l];
    m->act = spec->activation;
    m->kc = kc;
    m->rcut = spec->rcut;
    m->padded = K != Kabi;
    for (int l = 0; l < L; ++l) m->padded = m->padded || m->hid[l] != H;
    {
        int64_t per = 0, per_int = 0;
        int in = m->Fabi, in_int = m->F;
        for (int l = 0; l < L; ++l) {
            per += (int64_t)m->hid[l] * in + m->hid[l];
            per_int += (int64_t)H * in_int + H;
            in = m->hid[l];
            in_int = H;
        }
        m->per_species = per + in + 1;
        m->per_species_int = per_int + H + 1;
    }
    int64_t off = 0;
    m->w_off.resize(L);
    m->wt_off.resize(L);
    for (int l = 0; l < L; ++l) {
        const int in_pad = (l == 0) ? m->Fpad : H;
        m->w_off[l] = off;
        off += (int64_t)H * in_pad;
        m->wt_off[l] = off;
        off += (int64_t)H * in_pad;
    }
    m->w_species_stride = off;
    // radial functions past the model's K continue its grid (uniform grids
    // keep the two-exponential recurrence); their features meet zero weights
    std::vector<double> mu_d(K), eta_d(K);
    for (int k = 0; k < K; ++k) {
        if (k < Kabi) {
            mu_d[k] = spec->mu[k];
            eta_d[k] = spec->eta[k];
        } else {
            const double step = Kabi > 1 ? spec->mu[Kabi - 1] - spec->mu[Kabi - 2] : 0.0;
            mu_d[k] = spec->mu[Kabi - 1] + (k - Kabi + 1) * step;
            eta_d[k] = spec->eta[Kabi - 1];
        }
    }
    std::vector<float> mu(K), eta(K);
    m->mu_h = mu_d;
    m->eta_h = eta_d;
    for (int k = 0; k < K; ++k) {
        mu[k] = (float)mu_d[k];
        eta[k] = (float)eta_d[k];
    }
    {
        // recurrence for the Gaussians of a chunk on a uniform grid (see tmd_model)
        const double d = K > 1 ? mu_d[1] - mu_d[0] : 0.0, e0 = eta_d[0];
        bool ok = d > 0.0 && e0 > 0.0;
        for (int k = 0; k < K && ok; ++k)
            ok = std::fabs(mu_d[k] - mu_d[0] - k * d) <= 1e-9 * d && std::fabs(eta_d[k] - e0) <= 1e-12 * e0;
        for (int k0 = 0; k0 < K && ok; k0 += kc) {
            const double tmax = std::max(std::fabs(spec->rcut - mu_d[k0]), std::fabs(mu_d[k0]));
            ok = e0 * tmax * tmax <= 80.0 && 2.0 * e0 * d * tmax <= 80.0;
        }
        if (ok) {
            const double log2e = 1.4426950408889634;
            m->rec = true;
            m->rec_a = (float)(2.0 * e0 * d * log2e);
            m->rec_b = (float)(-e0 * d * d * log2e);
            m->rec_c = (float)std::exp(-2.0 * e0 * d * d);
            bool ok4 = K % 4 == 0;
            for (int k0 = 0; k0 < 4 && k0 < K && ok4; ++k0) {
                const double tmax = std::max(std::fabs(spec->rcut - mu_d[k0]), std::fabs(mu_d[k0]));
                ok4 = e0 * tmax * tmax <= 80.0 && 8.0 * e0 * d * tmax <= 80.0;
            }
            if (ok4) {
                m->rec4 = true;
                m->rec_c4 = (float)std::exp(-32.0 * e0 * d * d);
            }
        }
    }
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 256));
    };
    alloc((void**)&m->mu, 4 * K);
    alloc((void**)&m->eta, 4 * K);
    alloc((void**)&m->w32, 4 * (size_t)S * off);
    alloc((void**)&m->wbf, 2 * (size_t)S * off);
    alloc((void**)&m->bias, 4 * (size_t)S * L * H);
    alloc((void**)&m->wout, 4 * (size_t)S * H);
    alloc((void**)&m->bout, 4 * (size_t)S);
    alloc((void**)&m->params32, 4 * (size_t)S * m->per_species);
    if (m->padded) alloc((void**)&m->params_int, 4 * (size_t)S * m->per_species_int);
    else m->params_int = m->params32;
    if (e == hipSuccess) e = hipMemcpy(m->mu, mu.data(), 4 * K, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->eta, eta.data(), 4 * K, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        tmd_model_destroy(m);
        return hip_fail(ctx, e, "model allocation");
    }
    tmd_status st = upload_params(m, params);
    if (st != TMD_OK) {
        tmd_model_destroy(m);
        return st;
    }
    *out = m;
    return TMD_OK;
}

tmd_status tmd_model_set_params(tmd_model* m, const float* params) {
    if (!m || !params) return TMD_ERR_INVALID_ARGUMENT;
    TMD_HIP(m->ctx, hipStreamSynchronize(m->ctx->stream));
    // new weights restart the optimiser
    m->opt_t = 0;
    const size_t bytes = (size_t)m->S * m->per_species * 4;
    if (m->opt_m) TMD_HIP(m->ctx, hipMemset(m->opt_m, 0, bytes));
    if (m->opt_v) TMD_HIP(m->ctx, hipMemset(m->opt_v, 0, bytes));
    return upload_params(m, params);
}

tmd_status tmd_model_get_params(const tmd_model* m, float* params) {
    if (!m || !params) return TMD_ERR_INVALID_ARGUMENT;
    TMD_HIP(m->ctx, hipMemcpyAsync(params, m->params32, (size_t)m->S * m->per_species * 4, hipMemcpyDeviceToHost,
                                   m->ctx->stream));
    TMD_HIP(m->ctx, hipStreamSynchronize(m->ctx->stream));
    return TMD_OK;
}

tmd_status tmd_model_set_precision(tmd_model* m, tmd_precision precision) {
    if (!m) return TMD_ERR_INVALID_ARGUMENT;
    if (precision != TMD_FP32 && precision != TMD_BF16_MLP)
        return fail(m->ctx, TMD_ERR_INVALID_ARGUMENT, "unknown precision");
    m->prec = precision;
    return TMD_OK;
}

tmd_status tmd_model_tabulate(tmd_model* m, double dr) {
    if (!m) return TMD_ERR_INVALID_ARGUMENT;
    if (!std::isfinite(dr) || dr < 0.0 || dr > m->rcut)
        return fail(m->ctx, TMD_ERR_INVALID_ARGUMENT, "table spacing must be in [0, rcut]");
    const double nint_d = dr > 0.0 ? std::ceil(m->rcut / dr) : 0.0;
    if (nint_d > (double)(1 << 20)) return fail(m->ctx, TMD_ERR_INVALID_ARGUMENT, "more than 2^20 table intervals");
    TMD_HIP(m->ctx, hipStreamSynchronize(m->ctx->stream));
    if (dr == 0.0) {
        if (m->tab) TMD_HIP(m->ctx, hipFree(m->tab));
        m->tab = nullptr;
        m->tab_n = 0;
        m->tab_delta = 0.0;
        return TMD_OK;
    }
    const int n = (int)nint_d, K = m->K;
    const double rc = m->rcut, delta = rc / n;
    // node data: exact h_k and h_k' (FP64) at r_j = j delta, zero at r = 0 and r = rc
    std::vector<double> f((size_t)(n + 1) * K), df((size_t)(n + 1) * K);
    for (int j = 0; j <= n; ++j) {
        const double R = j * delta;
        const double fc = (j > 0 && j < n) ? 0.5 * (std::cos(M_PI * R / rc) + 1.0) : 0.0;
        const double dfc = (j > 0 && j < n) ? -0.5 * (M_PI / rc) * std::sin(M_PI * R / rc) : 0.0;
        for (int k = 0; k < K; ++k) {
            const double t = R - m->mu_h[k], e = std::exp(-m->eta_h[k] * t * t);
            f[(size_t)j * K + k] = e * fc;
            df[(size_t)j * K + k] = e * (dfc - 2.0 * m->eta_h[k] * t * fc);
        }
    }
    // per interval the cubic with these end values and slopes, in powers of t
    std::vector<float4> tab((size_t)(n + 1) * K, make_float4(0.f, 0.f, 0.f, 0.f));
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < K; ++k) {
            const double f0 = f[(size_t)j * K + k], f1 = f[(size_t)(j + 1) * K + k];
            const double s0 = delta * df[(size_t)j * K + k], s1 = delta * df[(size_t)(j + 1) * K + k];
            tab[(size_t)j * K + k] = make_float4((float)f0, (float)s0, (float)(3.0 * (f1 - f0) - 2.0 * s0 - s1),
                                                 (float)(2.0 * (f0 - f1) + s0 + s1));
        }
    float4* d = nullptr;
    const size_t bytes = tab.size() * sizeof(float4);
    if (hipMalloc((void**)&d, bytes) != hipSuccess) return fail(m->ctx, TMD_ERR_OUT_OF_MEMORY, "radial table");
    const hipError_t e = hipMemcpy(d, tab.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(m->ctx, e, "radial table upload");
    }
    if (m->tab) (void)hipFree(m->tab);
    m->tab = d;
    m->tab_n = n;
    m->tab_delta = delta;
    return TMD_OK;
}

double tmd_model_tab_spacing(const tmd_model* m) { return m ? m->tab_delta : 0.0; }

int64_t tmd_model_params_per_species(const tmd_model* m) { return m ? m->per_species : 0; }
int32_t tmd_model_n_features(const tmd_model* m) { return m ? m->Fabi : 0; }

void tmd_model_destroy(tmd_model* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    for (void* p : {(void*)m->mu, (void*)m->eta, (void*)m->w32, (void*)m->wbf, (void*)m->bias, (void*)m->wout,
                    (void*)m->bout, (void*)m->params32, (void*)m->opt_m, (void*)m->opt_v, (void*)m->tab,
                    (void*)(m->padded ? m->params_int : nullptr)})
        if (p) (void)hipFree(p);
    delete m;
}

tmd_status tmd_nlist_create(tmd_context* ctx, int64_t n_atoms, int32_t n_species, int32_t capacity,
                            tmd_nlist** out) {
    if (!ctx || !out) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null argument");
    *out = nullptr;
    if (n_atoms <= 0 || n_atoms >= ((int64_t)1 << 31)) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "bad n_atoms");
    if (n_species < 1 || n_species > kMaxSpecies) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "n_species must be in 1..8");
    if (capacity < 1 || capacity > 4096) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "capacity must be in 1..4096");
    tmd_nlist* nl = new (std::nothrow) tmd_nlist();
    if (!nl) return fail(ctx, TMD_ERR_OUT_OF_MEMORY, "host allocation");
    nl->ctx = ctx;
    nl->nmax = n_atoms;
    nl->S = n_species;
    nl->cap = (capacity + 3) / 4 * 4;  // rows start 16-byte aligned
    const size_t n = (size_t)n_atoms, lst = (size_t)n_species * nl->cap * n;
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 256));
    };
    alloc((void**)&nl->perm, 4 * n);
    alloc((void**)&nl->shift, 12 * n);
    alloc((void**)&nl->xs, 32 * n);
    alloc((void**)&nl->sp, 4 * n);
    alloc((void**)&nl->nbr, 4 * lst);
    alloc((void**)&nl->img, 4 * lst);
    alloc((void**)&nl->cnt, 4 * (size_t)n_species * n);
    alloc((void**)&nl->sp_idx, 4 * n);
    alloc((void**)&nl->wperm, 4 * n);
    alloc((void**)&nl->wcell, n);
    if (e != hipSuccess) {
        tmd_nlist_destroy(nl);
        return hip_fail(ctx, e, "neighbour list allocation");
    }
    *out = nl;
    return TMD_OK;
}

void tmd_nlist_destroy(tmd_nlist* nl) {
    if (!nl) return;
    (void)hipDeviceSynchronize();
    for (void* p : {(void*)nl->perm, (void*)nl->shift, (void*)nl->xs, (void*)nl->sp, (void*)nl->nbr, (void*)nl->img,
                    (void*)nl->cnt, (void*)nl->sp_idx, (void*)nl->cellstart, (void*)nl->wperm, (void*)nl->wcell,
                    (void*)nl->wbase, (void*)nl->pnbr, (void*)nl->pimg, (void*)nl->pcnt, (void*)nl->prune_state})
        if (p) (void)hipFree(p);
    delete nl;
}

int32_t tmd_nlist_capacity(const tmd_nlist* nl) { return nl ? nl->cap : 0; }

tmd_status tmd_nlist_stats(tmd_context* ctx, const tmd_nlist* nl, int64_t* total_pairs, int32_t* max_row) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    if (!nl || !nl->built) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "neighbour list has not been built");
    return launch_nlist_stats(ctx, nl, total_pairs, max_row);
}

tmd_status tmd_build_neighbors(tmd_context* ctx, const tmd_system_view* sys, double rcut, double skin, tmd_nlist* nl,
                               int32_t* required_capacity) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    if (!nl) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null neighbour list");
    tmd_status st = check_system(ctx, sys);
    if (st != TMD_OK) return st;
    if (sys->n_atoms > nl->nmax) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "more atoms than the list was created for");
    if (!(rcut > 0.0) || !std::isfinite(rcut)) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "rcut must be positive");
    if (!(skin >= 0.0) || !std::isfinite(skin)) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "skin must be non-negative");
    nl->built = false;
    return launch_build_neighbors(ctx, sys, rcut + skin, nl, required_capacity);
}

tmd_status tmd_nlist_export(tmd_context* ctx, const tmd_nlist* nl, int32_t* nbr, int32_t* img, int32_t* cnt) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    if (!nl || !nbr || !img || !cnt) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null argument");
    if (!nl->built) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "neighbour list has not been built");
    return launch_export_nlist(ctx, nl, nbr, img, cnt);
}

tmd_status tmd_descriptors(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys, const tmd_nlist* nl,
                           float* G) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    tmd_status st = check_eval(ctx, m, sys, nl);
    if (st != TMD_OK) return st;
    if (!G) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null G");
    hipError_t e = hipSuccess;
    float* Gs = (float*)ctx->ws.get("ev.G", sizeof(float) * nl->n * m->F, &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "descriptor workspace");
    if ((st = launch_refresh_positions(ctx, sys, nl)) != TMD_OK) return st;
    if ((st = launch_descriptors(ctx, m, nl, Gs, nullptr)) != TMD_OK) return st;
    return launch_permute_rows(ctx, nl, Gs, m, G);
}

tmd_status tmd_energy_forces(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys, const tmd_nlist* nl,
                             double* energy, float* atom_energy, float* forces, double* virial6) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    tmd_status st = check_eval(ctx, m, sys, nl);
    if (st != TMD_OK) return st;
    if (!energy || !forces) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null energy or forces");
    hipError_t e = hipSuccess;
    double* tot = (double*)ctx->ws.get("ev.totals", sizeof(double) * 8, &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "totals workspace");
    if ((st = run_energy_forces(ctx, m, sys, nl, tot, atom_energy, forces)) != TMD_OK) return st;
    TMD_HIP(ctx, hipMemcpyAsync(ctx->h_totals, tot, sizeof(double) * 7, hipMemcpyDeviceToHost, ctx->stream));
    TMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *energy = ctx->h_totals[0];
    if (virial6)
        for (int j = 0; j < 6; ++j) virial6[j] = ctx->h_totals[1 + j];
    return TMD_OK;
}

tmd_status tmd_energy_forces_async(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys,
                                   const tmd_nlist* nl, double* totals7, float* atom_energy, float* forces) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    tmd_status st = check_eval(ctx, m, sys, nl);
    if (st != TMD_OK) return st;
    if (!totals7 || !forces) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null totals or forces");
    return run_energy_forces(ctx, m, sys, nl, totals7, atom_energy, forces);
}

tmd_status tmd_energy_forces_batch(tmd_context* ctx, const tmd_model* m, int32_t n_systems,
                                   const tmd_system_view* systems, const tmd_nlist* const* lists, double* totals7,
                                   float* const* forces) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    if (n_systems <= 0 || n_systems > kMaxBatchSystems || !systems || !lists || !totals7 || !forces)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT,
                    "tmd_energy_forces_batch: 1.." + std::to_string(kMaxBatchSystems) +
                        " systems with non-null views, lists, totals and force arrays");
    std::vector<BatchSeg> segs((size_t)n_systems);
    int64_t N = 0, counts[kMaxSpecies] = {0};
    int cap = 4;
    for (int s = 0; s < n_systems; ++s) {
        tmd_status st = check_eval(ctx, m, &systems[s], lists[s]);
        if (st != TMD_OK) return st;
        if (!forces[s]) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null force array");
        const tmd_nlist* nl = lists[s];
        BatchSeg& g = segs[s];
        g.off = N;
        g.n = nl->n;
        g.npad = (nl->n + kBlock - 1) / kBlock * kBlock;
        N += g.npad;
        g.cap = nl->cap;
        cap = std::max(cap, nl->cap);
        for (int a = 0; a < 3; ++a) g.L[a] = systems[s].box[a];
        g.pos = systems[s].pos;
        g.perm = nl->perm;
        g.shift = nl->shift;
        g.nbr = nl->nbr;
        g.img = nl->img;
        g.cnt = nl->cnt;
        g.sp_idx = nl->sp_idx;
        for (int b = 0; b <= m->S; ++b) g.sp_off[b] = nl->sp_off[b];
        for (int b = 0; b < m->S; ++b) counts[b] += nl->sp_off[b + 1] - nl->sp_off[b];
        g.forces = forces[s];
    }
    if (N >= (int64_t)1 << 31) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "batch of more than 2^31-1 atoms");
    tmd_nlist v;  // the merged list: a view over workspace arrays
    v.ctx = ctx;
    v.nmax = v.n = N;
    v.S = m->S;
    v.cap = cap;
    v.built = true;
    v.rlist = m->rcut;
    v.sp_off[0] = 0;
    for (int b = 0; b < m->S; ++b) {
        v.sp_count[b] = counts[b];
        v.sp_off[b + 1] = v.sp_off[b] + counts[b];
    }
    for (int b = 0; b < m->S; ++b) {
        int64_t at = v.sp_off[b];
        for (auto& g : segs) {
            g.dst_off[b] = at;
            at += g.sp_off[b + 1] - g.sp_off[b];
        }
    }
    const int nch = m->K / m->kc;  // chunk lanes per atom in the adjoint: 256 / nch atoms per virial partial
    hipError_t e = hipSuccess;
    BatchSeg* dsegs = (BatchSeg*)ctx->ws.get("batch.segs", sizeof(BatchSeg) * segs.size(), &e);
    v.xs = (double4*)ctx->ws.get("batch.xs", sizeof(double4) * N, &e);
    double4* boxes = (double4*)ctx->ws.get("batch.boxes", sizeof(double4) * N, &e);
    v.boxes = boxes;
    v.nbr = (int32_t*)ctx->ws.get("batch.nbr", sizeof(int32_t) * (size_t)N * m->S * cap, &e);
    v.img = (int32_t*)ctx->ws.get("batch.img", sizeof(int32_t) * (size_t)N * m->S * cap, &e);
    v.cnt = (int32_t*)ctx->ws.get("batch.cnt", sizeof(int32_t) * (size_t)N * m->S, &e);
    v.sp_idx = (int32_t*)ctx->ws.get("batch.sp_idx", sizeof(int32_t) * (size_t)N, &e);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch workspace allocation");
    EvalBuffers b;
    tmd_status st = eval_buffers(ctx, m, &v, &b);
    if (st != TMD_OK) return st;
    // pageable source: the copy is staged before the call returns
    TMD_HIP(ctx, hipMemcpyAsync(dsegs, segs.data(), sizeof(BatchSeg) * segs.size(), hipMemcpyHostToDevice,
                                ctx->stream));
    if ((st = launch_batch_merge(ctx, dsegs, n_systems, &v, boxes)) != TMD_OK) return st;
    uint16_t* Gb = m->prec == TMD_BF16_MLP ? reinterpret_cast<uint16_t*>(b.G) : nullptr;
    if ((st = launch_descriptors(ctx, m, &v, b.G, b.P, Gb)) != TMD_OK) return st;
    if ((st = launch_mlp(ctx, m, species_groups(&v), m->prec, b.G, Gb, b.Ei, b.dG)) != TMD_OK) return st;
    int nvir = 0;
    if ((st = launch_adjoint(ctx, m, &v, b.dG, b.P, b.Fq, b.vir, &nvir)) != TMD_OK) return st;
    return launch_batch_finalize(ctx, dsegs, n_systems, N, b.Fq, b.Ei, b.vir, kBlock / nch, totals7);
}

tmd_status tmd_energy_forces_noalloc(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys,
                                     const tmd_nlist* nl, double* totals7, float* atom_energy, float* forces) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    tmd_status st = check_eval(ctx, m, sys, nl);
    if (st != TMD_OK) return st;
    if (!totals7 || !forces) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null totals or forces");
    if (nl->rlist > m->rcut * (1.0 + 1e-9))
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT,
                    "tmd_energy_forces_noalloc takes lists built with rlist = rcut (a skin list needs pruned-row "
                    "memory)");
    if (!ctx->scratch) return fail(ctx, TMD_ERR_DEVICE, "the scratch array's device address is unavailable");
    EvalBuffers b{};
    size_t need = 0;
    scratch_buffers(ctx->scratch, m, nl, &b, &need);
    if (need > kScratchBytes)
        return fail(ctx, TMD_ERR_INVALID_ARGUMENT,
                    "system too large for tmd_energy_forces_noalloc: needs " + std::to_string(need) +
                        " bytes of scratch, the limit is " + std::to_string(kScratchBytes));
    // per-kernel timing would create events; it is suspended for this call
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    st = run_energy_forces_in(ctx, m, sys, nl, b, totals7, atom_energy, forces, nullptr);
    ctx->prof.on = prof;
    return st;
}

int64_t tmd_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }

}  // extern "C"

namespace tmd {

tmd_status energy_forces_gated(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys, const tmd_nlist* nl,
                               double* totals7, float* atom_energy, float* forces, const PruneGate* gate) {
    if (!ctx) return TMD_ERR_INVALID_ARGUMENT;
    tmd_status st = check_eval(ctx, m, sys, nl);
    if (st != TMD_OK) return st;
    if (!totals7 || !forces) return fail(ctx, TMD_ERR_INVALID_ARGUMENT, "null totals or forces");
    return run_energy_forces(ctx, m, sys, nl, totals7, atom_energy, forces, gate);
}

}  // namespace tmd
