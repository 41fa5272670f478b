// Internal declarations of libtmd.so: handle layouts, kernel launch entry
// points and small device helpers.  Not part of the public ABI (include/tmd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/tmd.h"

namespace tmd {

constexpr int kMaxSpecies = 8;
// Preferred cell block of the blocked adjoint (cells per axis, clamped to the grid).
constexpr int kBlockShape[3] = {4, 4, 2};
// Further block shapes whose largest halos the build counts exactly, taken in
// turn when the previous one's halo does not fit the LDS budget (dense
// systems, large cells such as lists with a skin).
constexpr int kBlockShape2[3] = {4, 2, 2};
constexpr int kBlockShape3[3] = {3, 2, 2};
constexpr int kBlock = 256;

// Workgroups are dispatched to the eight XCDs round-robin (workgroup b runs on
// XCD b mod 8, each XCD with its own L2).  The logical block of a workgroup is
// chosen so that each XCD walks one contiguous eighth of the blocks: sorted
// atoms are cell-major, so an XCD's neighbour gathers stay in a compact slab
// that its L2 holds.  The grid is rounded up to a multiple of 8; the padding
// workgroups get -1.
__device__ __forceinline__ int64_t xcd_block(int64_t nblocks) {
    const int64_t b = blockIdx.x, per = (nblocks + 7) / 8;
    const int64_t l = (b % 8) * per + b / 8;
    return l < nblocks ? l : -1;
}
inline unsigned xcd_grid(int64_t nblocks) { return (unsigned)((nblocks + 7) / 8 * 8); }

// Grow-only device buffers owned by a context, keyed by purpose.
struct Workspace {
    std::unordered_map<std::string, std::pair<void*, size_t>> bufs;
    void* get(const std::string& key, size_t bytes, hipError_t* err);
    void release();
};

}  // namespace tmd

namespace tmd {
// Optional per-kernel timing with HIP events recorded on the context's stream.
struct ProfRec {
    const char* name;
    hipEvent_t start, stop;
};
struct Profiler {
    bool on = false;
    std::vector<ProfRec> pending;
    std::vector<hipEvent_t> pool;
    std::vector<std::string> names;
    std::vector<double> total_ms;
    std::vector<int64_t> count;
    hipEvent_t get_event();
    void collect();  // synchronises on the pending events
    void release();
};
}  // namespace tmd

struct tmd_context {
    int device = 0;
    int num_cus = 256;  // compute units of the device
    hipStream_t stream = nullptr;
    std::string last_error;
    tmd::Workspace ws;
    tmd::Profiler prof;
    double* h_totals = nullptr;  // pinned host [8]
    int32_t* h_flags = nullptr;  // pinned host [64]
    // device address of the library's static scratch array on this context's
    // device (tmd_energy_forces_noalloc), looked up once per device at creation
    unsigned char* scratch = nullptr;
};

namespace tmd {
// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
    tmd_context* ctx;
    ProfRec rec{};
    ProfScope(tmd_context* c, const char* name) : ctx(c) {
        if (!ctx->prof.on) return;
        rec.name = name;
        rec.start = ctx->prof.get_event();
        rec.stop = ctx->prof.get_event();
        (void)hipEventRecord(rec.start, ctx->stream);
    }
    ~ProfScope() {
        if (!ctx->prof.on || !rec.name) return;
        (void)hipEventRecord(rec.stop, ctx->stream);
        ctx->prof.pending.push_back(rec);
    }
};
}  // namespace tmd

// The kernels run a padded copy of the model: K radial functions rounded up to
// 4, 6 or 8 times a power of two (so that each thread takes a whole chunk of
// them) and every hidden layer at one width H in {32, 64, 128}.  The padded
// radial functions continue the model's grid and the padded hidden units sit
// behind zero weights, so that neither reaches an atomic energy, a force or
// the virial: the first layer's columns of padded features, and every row
// and column of a padded unit, are zero.  K, F and H below are the padded
// sizes; Kabi, Fabi and hid[] are the model's own.
struct tmd_model {
    tmd_context* ctx = nullptr;
    int S = 0, K = 0, M = 0, D = 0, F = 0, Fpad = 0, L = 0, H = 0, act = 0;
    int Dr = 0;  // moment components of P the evaluation path stores (the unit-norm identity drops the rest)
    int Kabi = 0, Fabi = 0;
    int hid[TMD_MAX_HIDDEN] = {0, 0, 0, 0};
    int kc = 8;  // radial functions per thread in the descriptor / adjoint kernels
    double rcut = 0.0;
    tmd_precision prec = TMD_FP32;
    int64_t per_species = 0;      // floats per species in the ABI parameter layout
    int64_t per_species_int = 0;  // the same layout at the padded sizes
    bool padded = false;          // the padded sizes differ from the model's
    // device parameters
    float* mu = nullptr;   // [K]
    float* eta = nullptr;  // [K]
    // Uniform radial grid (mu_k = mu_0 + k Delta, one eta): consecutive
    // Gaussians differ by the factor r_k = exp2(rec_a t_k + rec_b), t_k = R - mu_k,
    // with r_{k+1} = r_k * rec_c, so a chunk needs two exponentials.  Set only
    // when no value of a chunk can underflow before the chunk's last one.
    bool rec = false;
    float rec_a = 0.0f, rec_b = 0.0f, rec_c = 0.0f;
    // The same in steps of four radial functions (ratio exp2(4 rec_a t_k +
    // 16 rec_b), which gains rec_c4 = rec_c^16 per step), set when none of
    // those ratios or the first Gaussian of a lane (k = 0..3) can leave the
    // FP32 range.
    bool rec4 = false;
    float rec_c4 = 0.0f;
    std::vector<double> mu_h, eta_h;  // host FP64 copies (table construction)
    // Tabulated radial functions (cubic Hermite on nodes tab_delta apart):
    // tab [(tab_n + 1)][K] float4 = (c0, c1, c2, c3) of h_k = c0 + t(c1 + t(c2 + t c3))
    // on interval j, t = R/delta - j; row tab_n is all zero (R >= rcut).
    float4* tab = nullptr;
    int tab_n = 0;
    double tab_delta = 0.0;
    // Per species, per layer l = 0..L-1: forward W_l [H][in_pad] and transposed
    // W_l^T [in_pad][H] (in_pad = Fpad for l = 0, H otherwise), FP32 and BF16 copies.
    float* w32 = nullptr;
    __hip_bfloat16* wbf = nullptr;
    int64_t w_species_stride = 0;         // elements per species in w32 / wbf
    std::vector<int64_t> w_off, wt_off;   // per layer offsets inside a species block
    float* bias = nullptr;   // [S][L][H]
    float* wout = nullptr;   // [S][H]
    float* bout = nullptr;   // [S]
    // master copy in the ABI layout [S][per_species] and optimiser state;
    // params_int: the master copy in the padded layout [S][per_species_int]
    // (zero at every padded entry; == params32 when nothing is padded)
    float* params32 = nullptr;
    float* params_int = nullptr;
    float* opt_m = nullptr;
    float* opt_v = nullptr;
    int64_t opt_t = 0;
};

namespace tmd {
// Position of an ABI-layout parameter in the padded layout.  Both layouts
// hold, per species, W_l [out][in] then b_l [out] for each hidden layer, then
// the output weights [width] and bias; the padded one at the padded sizes.
// Returns the offset inside the species block and, for a weight, its row o
// and padded column c (layer l; -1 for the output layer and biases).
struct ParamMap {
    int L, H, F, Fabi, K, Kabi, M1;
    int hid[TMD_MAX_HIDDEN];
    __host__ __device__ int64_t map(int64_t q, int& l, int& o, int& c, int& kind) const {
        int64_t base = 0;
        int in_abi = Fabi, in_int = F;
        for (l = 0; l < L; ++l) {
            const int out = hid[l];
            if (q < (int64_t)out * in_abi) {
                o = (int)(q / in_abi);
                const int ca = (int)(q - (int64_t)o * in_abi);
                if (l == 0) {
                    const int per_b = Kabi * M1, b = ca / per_b, r = ca - b * per_b;
                    c = (b * K + r / M1) * M1 + r % M1;
                } else {
                    c = ca;
                }
                kind = 0;
                return base + (int64_t)o * in_int + c;
            }
            q -= (int64_t)out * in_abi;
            base += (int64_t)H * in_int;
            if (q < out) {
                o = (int)q;
                c = -1;
                kind = 1;
                return base + q;
            }
            q -= out;
            base += H;
            in_abi = out;
            in_int = H;
        }
        c = -1;
        if (q < in_abi) {
            o = (int)q;
            kind = 2;
            return base + q;
        }
        o = 0;
        kind = 3;
        return base + H;
    }
};
inline ParamMap param_map(const tmd_model* m) {
    ParamMap pm{};
    pm.L = m->L;
    pm.H = m->H;
    pm.F = m->F;
    pm.Fabi = m->Fabi;
    pm.K = m->K;
    pm.Kabi = m->Kabi;
    pm.M1 = m->M + 1;
    for (int l = 0; l < TMD_MAX_HIDDEN; ++l) pm.hid[l] = m->hid[l];
    return pm;
}
}  // namespace tmd

struct tmd_nlist {
    tmd_context* ctx = nullptr;
    int64_t nmax = 0;
    int S = 1;
    int cap = 0;
    // state of the last successful build
    int64_t n = 0;
    bool built = false;
    double box[3] = {0, 0, 0};
    double rlist = 0.0;
    int nc[3] = {1, 1, 1};
    int reach[3] = {1, 1, 1};
    int64_t sp_count[tmd::kMaxSpecies] = {0};
    int64_t sp_off[tmd::kMaxSpecies + 1] = {0};
    // device arrays, sorted (cell-major) atom order
    int32_t* perm = nullptr;     // [n]   sorted -> original index
    int32_t* shift = nullptr;    // [n][3] wrap shift: x_wrapped = x + shift * L
    double4* xs = nullptr;       // [n]   positions used by the kernels
    const double4* boxes = nullptr;  // [n] per-atom box edges of a merged multi-system list (else box)
    int32_t* sp = nullptr;       // [n]   species
    int32_t* nbr = nullptr;      // [n][S][cap] neighbour (sorted index), row-major per atom
    int32_t* img = nullptr;      // [n][S][cap] image word (pack_img)
    int32_t* cnt = nullptr;      // [S][n]
    int32_t* sp_idx = nullptr;   // [n] sorted indices grouped by species
    // cell structure of the last build (sorted atoms are cell-major)
    int32_t* cellstart = nullptr;  // [ncells + 1]
    int64_t cellstart_cap = 0;
    int64_t ncells = 0;
    int max_occ = 0;               // most atoms in one cell
    int halo_max = -1;             // most atoms in one kBlockShape block plus halo (-1: not counted)
    int halo_max2 = -1;            // the same for kBlockShape2
    int halo_max3 = -1;            // and for kBlockShape3
    bool narrow = false;           // 3x3x3 stencil (every reach is 1)
    // Work order of the descriptor and adjoint kernels, set by every build
    // when the adjoint runs over cell blocks (wo_valid): blocks of wo_B cells
    // in block-major order, each block's atoms by descending species-0 row
    // length (so that a wave's rows are alike);
    // wperm[w] = sorted atom index of work slot w, wcell[w] = its cell inside
    // the block, wbase[blk] = first slot of block blk, and after those
    // (wbase + blocks + 1) the first 16-atom group of each block (the
    // matrix-core kernels' P layout).  P is stored by slot or by group.
    bool wo_valid = false;
    int wo_B[3] = {1, 1, 1}, wo_nb[3] = {1, 1, 1}, wo_hmax = 0;
    int32_t* wperm = nullptr;      // [nmax]
    uint8_t* wcell = nullptr;      // [nmax]
    int32_t* wbase = nullptr;      // [wbase_cap]
    int64_t wbase_cap = 0;
    // Rows pruned for lists built with a skin (same layout as nbr / img /
    // cnt, allocated on first use): to the model cutoff at every evaluation,
    // or, when the caller tracks displacements (PruneGate), to the cutoff plus
    // a margin and only when the last such copy may have lost a pair.
    int32_t* pnbr = nullptr;
    int32_t* pimg = nullptr;
    int32_t* pcnt = nullptr;
    double* prune_state = nullptr;  // device: displacement since the build at the last margin prune
    int32_t* prune_flag = nullptr;  // device: 1 when this evaluation prunes
    int64_t build_id = 0;           // count of builds
    int64_t pruned_build_id = -1;   // build the pruned rows come from (margin prunes only)
    double pruned_margin = -1.0;    // margin of the pruned rows (-1: pruned to the cutoff)
};

namespace tmd {

// Status helpers ------------------------------------------------------------
tmd_status fail(tmd_context* ctx, tmd_status st, const std::string& msg);
tmd_status hip_fail(tmd_context* ctx, hipError_t e, const char* what);

#define TMD_HIP(ctx, call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return tmd::hip_fail((ctx), e_, #call); \
    } while (0)

// Image word of a list entry: three signed 8-bit image components and, in the
// top byte, the entry's stencil cell offset (ox, oy, oz in -1..1 as the
// two-bit fields ox+1, oy+1, oz+1 at bits 0, 2, 4 of the byte; 255 when
// unused, i.e. when the stencil is wider than 3x3x3).
__host__ __device__ inline int stencil_bits(int o) {  // o = (ox+1) + 3 (oy+1) + 9 (oz+1)
    return (o % 3) | (((o / 3) % 3) << 2) | ((o / 9) << 4);
}
__host__ __device__ inline int32_t pack_img(int nx, int ny, int nz, int ocode = 255) {
    return (int32_t)((uint32_t)(nx & 0xff) | ((uint32_t)(ny & 0xff) << 8) | ((uint32_t)(nz & 0xff) << 16) |
                     ((uint32_t)(ocode & 0xff) << 24));
}
__host__ __device__ inline int img_ocode(int32_t c) { return (int)(((uint32_t)c >> 24) & 0xff); }
// ox+1, oy+1, oz+1 of an entry's stencil offset (0..2 each).
__device__ inline int img_sx(int32_t c) { return (int)__builtin_amdgcn_ubfe((uint32_t)c, 24, 2); }
__device__ inline int img_sy(int32_t c) { return (int)__builtin_amdgcn_ubfe((uint32_t)c, 26, 2); }
__device__ inline int img_sz(int32_t c) { return (int)__builtin_amdgcn_ubfe((uint32_t)c, 28, 2); }
__host__ __device__ inline void unpack_img(int32_t c, int& nx, int& ny, int& nz) {
    nx = (int)(int8_t)(c & 0xff);
    ny = (int)(int8_t)((c >> 8) & 0xff);
    nz = (int)(int8_t)((c >> 16) & 0xff);
}

// Launchers (each enqueues on ctx->stream) ---------------------------------
tmd_status launch_build_neighbors(tmd_context* ctx, const tmd_system_view* sys, double rlist, tmd_nlist* nl,
                                  int32_t* required_capacity);
tmd_status launch_refresh_positions(tmd_context* ctx, const tmd_system_view* sys, const tmd_nlist* nl);
// Descriptors G [n][F] (sorted order); when Pbuf is non-null the per-atom P
// tensors (kept components) are kept there for the adjoint: p_slots(m, nl)
// x S x K x Dr floats.  When Gb is non-null G is stored there instead, as the
// bits of (__bf16)G (nearest-even): the operand a BF16 MLP takes, at half the
// bytes.
tmd_status launch_descriptors(tmd_context* ctx, const tmd_model* m, const tmd_nlist* nl, float* G, float* Pbuf,
                              uint16_t* Gb = nullptr);
// Atom slots of the P buffer for this model and list (the matrix-core
// kernels pad each work-order block to whole 16-atom groups), and a bound for
// reserving workspace before any list exists (blocks of 128 atoms or more on
// average, or up to 1,024 blocks; a list needing more grows the buffer at its
// first evaluation).
int64_t p_slots(const tmd_model* m, const tmd_nlist* nl);
int64_t p_slots_reserve(int64_t n);
// Atoms grouped by species: idx[off[s] .. off[s+1]) are the atoms of species s
// (row indices into G, Ei and dG).
struct SpeciesGroups {
    int S = 1;
    int64_t off[kMaxSpecies + 1] = {0};
    const int32_t* idx = nullptr;
};
SpeciesGroups species_groups(const tmd_nlist* nl);
// Per-element MLP: E_i and dE/dG for every grouped atom, in precision prec:
// TMD_FP32 reads the FP32 descriptors G, TMD_BF16_MLP the BF16 ones Gb (the
// other pointer may be null).
tmd_status launch_mlp(tmd_context* ctx, const tmd_model* m, const SpeciesGroups& g, tmd_precision prec,
                      const float* G, const uint16_t* Gb, float* Ei, float* dG);
// Forces are accumulated as 64-bit fixed-point integers with 32 fractional
// bits (F = q 2^-32, |F| < 2^31 eV/A): integer additions are associative, so
// the sums do not depend on the order of the scatter's atomic adds and the
// forces are reproducible bit for bit.
constexpr double kForceFixedScale = 4294967296.0;  // 2^32
// Virial partials: per block, 6 compensated FP64 sums (value, compensation).
constexpr int kVirDoubles = 12;
// Adjoint: forces accumulated into Fq [n][3] (fixed point, zeroed by the
// launcher), virial block partials [blocks][6][2] into vir_partials (count in
// *nvir_out).
tmd_status launch_adjoint(tmd_context* ctx, const tmd_model* m, const tmd_nlist* nl, const float* dG, float* Pbuf,
                          unsigned long long* Fq, double* vir_partials, int* nvir_out);
// part: device scratch of finalize_part_doubles() doubles.
constexpr int64_t finalize_part_doubles() { return 256 * 14; }
tmd_status launch_finalize(tmd_context* ctx, const tmd_nlist* nl, const float* Ei, const unsigned long long* Fq,
                           const double* vir_partials, int nvir, float* atom_energy, float* forces, double* totals7,
                           double* part);
// Descriptor rows [n][F] (sorted order, padded radial functions) to the
// caller's order and the model's own F columns.
tmd_status launch_permute_rows(tmd_context* ctx, const tmd_nlist* nl, const float* in, const tmd_model* m, float* out);
// Rows [n][F] at the padded radial functions (F features, K radial
// functions) to the model's Fabi columns (Kabi radial functions), same rows.
tmd_status launch_compact_features(tmd_context* ctx, int64_t n, const float* in, int F, int Fabi, int K, int Kabi,
                                   int M1, float* out);
tmd_status launch_export_nlist(tmd_context* ctx, const tmd_nlist* nl, int32_t* nbr, int32_t* img, int32_t* cnt);
tmd_status launch_nlist_stats(tmd_context* ctx, const tmd_nlist* nl, int64_t* total_pairs, int32_t* max_row);

// Regenerate the MLP operand copies (W, W^T in FP32 and BF16, biases, output
// layer) of every species from the master parameters m->params32.
tmd_status launch_unpack_params(tmd_context* ctx, tmd_model* m);

// Pre-size a context's evaluation workspace for n atoms (avoids growth, and
// the device-wide synchronisation it implies, later), and its size in bytes.
tmd_status reserve_eval_workspace(tmd_context* ctx, const tmd_model* m, int64_t n);
size_t eval_workspace_bytes(const tmd_model* m, int64_t n);
tmd_status reserve_nlist_workspace(tmd_context* ctx, int64_t n, int S);
size_t nlist_workspace_bytes(int64_t n);
// Allocate a list's rows pruned to the cutoff now rather than at its first
// evaluation (a no-op once they exist).
tmd_status reserve_pruned_rows(tmd_context* ctx, tmd_nlist* nl);

// Velocity Verlet pieces (md.hip).  acc[S] = 9.648533e-3 / m_s; maxd2
// (nullable) receives the largest squared displacement from xref as ordered
// bits; the kinetic tensor out4 = (KE_xx, KE_yy, KE_zz, KE) in eV, FP64 fixed
// order, with part a [3 * kKeBlocks] scratch.
constexpr int kKeBlocks = 256;
tmd_status launch_kick_drift(tmd_context* ctx, int64_t n, double* x, double* v, const float* F, const int32_t* sp,
                             const double* acc, double dt, const double* xref, unsigned long long* maxd2);
tmd_status launch_kick(tmd_context* ctx, int64_t n, double* v, const float* F, const int32_t* sp, const double* acc,
                       double dt);
tmd_status launch_kinetic(tmd_context* ctx, int64_t n, const double* v, const int32_t* sp, const double* mass,
                          double* part, double* out4);
// p[0 .. n) = 0 (a kernel, not a memset).
tmd_status launch_zero_u64(tmd_context* ctx, unsigned long long* p, int64_t n);
// *flag = 1 when the squared displacement whose bits maxd2 holds exceeds
// limit2 (flag is sticky: never cleared here).
tmd_status launch_displacement_check(tmd_context* ctx, const unsigned long long* maxd2, double limit2, unsigned long long* flag);

// Copy of the list's rows keeping only the entries within rcut (times 1 + 1e-6)
// at the current positions, into nl->pnbr / pimg / pcnt (allocated on first
// use).  Every entry the kernels would use survives, in the same order.
tmd_status launch_prune(tmd_context* ctx, tmd_nlist* nl, double rcut);

// Displacement tracking that lets pruned rows be reused: maxd2 (device) holds
// the bits of the largest squared displacement of any atom since the list was
// built, for the positions being evaluated.  Rows pruned to rcut + margin when
// the largest displacement since the build was d_p keep every pair within
// rcut while d + d_p < margin / 2 (each of a pair's atoms moved by at most
// d + d_p since the prune), so they are rebuilt only when that fails.
struct PruneGate {
    const unsigned long long* maxd2;
    double margin;
};
// launch_prune with a gate: the decision is taken on the device (no host
// synchronisation); a new build always prunes.
tmd_status launch_prune_gated(tmd_context* ctx, tmd_nlist* nl, double rcut, const PruneGate& g);
// E+F on the stream with device-resident totals (totals7: E, W[6]); gate may
// be null (skin lists are then pruned to the cutoff at every call).
tmd_status energy_forces_gated(tmd_context* ctx, const tmd_model* m, const tmd_system_view* sys, const tmd_nlist* nl,
                               double* totals7, float* atom_energy, float* forces, const PruneGate* gate);

// Work order for the descriptor and adjoint (see tmd_nlist::wo_valid); called
// at the end of every successful list build.
tmd_status launch_work_order(tmd_context* ctx, tmd_nlist* nl);

constexpr int kMaxBatchSystems = 4096;
// Several systems' lists merged into one (tmd_energy_forces_batch): segment s
// covers combined atoms [off, off + n) followed by padding up to off + npad
// (npad a multiple of 256).
struct BatchSeg {
    int64_t off = 0, n = 0, npad = 0;
    int cap = 0;
    double L[3] = {0, 0, 0};
    const double* pos = nullptr;     // system positions [n][3], original order
    const int32_t* perm = nullptr;   // the system list's sorted -> original index
    const int32_t* shift = nullptr;  // and its wrap shifts
    const int32_t* nbr = nullptr;    // its rows (unpruned; skin entries are skipped by the kernels)
    const int32_t* img = nullptr;
    const int32_t* cnt = nullptr;
    const int32_t* sp_idx = nullptr;  // its species grouping
    int64_t sp_off[kMaxSpecies + 1] = {0};
    int64_t dst_off[kMaxSpecies] = {0};  // first slot of its species-b atoms in the merged grouping
    float* forces = nullptr;          // output [n][3], original order
};
// Merged positions, per-atom boxes, rows and species grouping into vnl's arrays.
tmd_status launch_batch_merge(tmd_context* ctx, const BatchSeg* segs, int nseg, tmd_nlist* vnl, double4* boxes);
// Forces to each segment's output and per-segment totals [nseg][7]; the adjoint
// wrote one virial partial per vir_atoms combined atoms.
tmd_status launch_batch_finalize(tmd_context* ctx, const BatchSeg* segs, int nseg, int64_t N,
                                 const unsigned long long* Fq, const float* Ei, const double* vir, int vir_atoms,
                                 double* totals);

// Upper bound on the virial partials the adjoint writes.
int64_t adjoint_max_partials(const tmd_model* m, const tmd_nlist* nl);

}  // namespace tmd
