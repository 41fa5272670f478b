/*
 * FP64 CPU oracle for the TensorMD energy / force / virial evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * It is deliberately plain: brute-force neighbour enumeration, explicit loops
 * over every tensor index, every step evaluated in double precision in the
 * order the paper states it:
 *   - atomic descriptor as a squared sum of neighbour moment tensors weighted
 *     by radial functions (Sec. II.A, eqn original_tensormd_formalism);
 *   - tensor form P = sum_c H M, S = T P^2, G = sigma(S) with the
 *     multiplicity table T_dm and the sqrt-on-m=0 function sigma
 *     (Sec. III.A, eqns T_dm, tensor_formalism, sigma_function);
 *   - atomic energies from a per-element MLP, E = sum_a E_a (Sec. III.A);
 *   - forces through the adjoint chain P' = 2 T sigma' P, U = P' M,
 *     V = P' H, F1 = U H' R', F2 = V M' and the scattered sum over pairs
 *     (Sec. III.A, eqns dP_abkd, U_abck, F1_abcx, F2_abcx);
 *   - optionally, radial functions interpolated from a table of nodes with
 *     the cutoff folded in (Sec. III.B), by cubic Hermite interpolation;
 *   - beyond the paper (its potentials were trained elsewhere): the
 *     force-matching loss and its parameter gradient, with the descriptor
 *     tangent and a second-order network pass written from their definitions,
 *     and a velocity-Verlet NVE integrator for the MD protocol (Sec. IV.D).
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 * Gaussian radial functions exp(-eta_k (R - mu_k)^2); cosine cutoff
 * 0.5 (cos(pi R / rc) + 1) for R < rc, else exactly 0; D = x_j + n*L - x_i
 * (neighbour minus centre); b = species of the neighbour; the squared sum
 * keeps the j = k self terms; sigma'(0) = 0; forces F_i += g, F_j -= g with
 * g = dE/dD; virial W_ab = -sum_pairs D_a g_b.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (oracle/build.py).
 * -ffp-contract=off keeps every product and sum separately rounded, which the
 * bit-exact neighbour-list comparison relies on.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_CAP 2
#define ORC_ERR_MEM 3
#define ORC_ERR_NUM 4

#define MAXW 1024   /* widest MLP layer the oracle accepts */
#define MAXL 8      /* most hidden layers */

typedef struct {
    int32_t n_species;     /* S */
    int32_t n_radial;      /* K */
    int32_t max_moment;    /* M in 0..3 */
    int32_t n_hidden;      /* number of hidden layers */
    int32_t hidden[MAXL];  /* hidden widths */
    int32_t activation;    /* 0 tanh, 1 squareplus */
    int32_t mlp_bf16;      /* 1: MLP matrix-product operands rounded to BF16 (see mlp_eval) */
    double rcut;
    double tab_dr;         /* > 0: radial functions from a table of this spacing (at most) */
    const double* mu;      /* [K] */
    const double* eta;     /* [K] */
    const double* params;  /* per-species packed MLP parameters */
} orc_model;

/* Exponents (p_x, p_y, p_z) of the moment components in the row order of the
 * multiplicity table T_dm: 1; x, y, z; xx, xy, xz, yy, yz, zz; xxx, xxy, xxz,
 * xyy, xyz, xzz, yyy, yyz, yzz, zzz. */
static const int MONO[20][3] = {
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2},
    {3, 0, 0}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 1, 1}, {1, 0, 2},
    {0, 3, 0}, {0, 2, 1}, {0, 1, 2}, {0, 0, 3}};

/* Multiplicities T_dm, one non-zero per row, as printed in the paper's table
 * (Sec. III.A, eqn T_dm). */
static const double TDM[20] = {1, 1, 1, 1, 1, 2, 2, 1, 2, 1, 1, 3, 3, 3, 6, 3, 1, 3, 3, 1};

static int n_moments(int M) { return (M + 1) * (M + 2) * (M + 3) / 6; }
static int order_of(int d) { return MONO[d][0] + MONO[d][1] + MONO[d][2]; }

int orc_n_features(const orc_model* m) { return m->n_species * m->n_radial * (m->max_moment + 1); }

int orc_params_per_species(const orc_model* m) {
    int prev = orc_n_features(m), tot = 0;
    for (int l = 0; l < m->n_hidden; ++l) { tot += m->hidden[l] * prev + m->hidden[l]; prev = m->hidden[l]; }
    return tot + prev + 1;
}

/* ------------------------------------------------------------------ */
/* Neumaier-compensated summation                                       */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;
static void nsum_add(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x; else a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum* a) { return a->s + a->c; }

double orc_neumaier_sum(int64_t n, const double* x) {
    nsum a = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nsum_add(&a, x[i]);
    return nsum_get(&a);
}

/* ------------------------------------------------------------------ */
/* Periodic wrap into [0, L)                                            */
/* ------------------------------------------------------------------ */
static double wrap1(double x, double L) {
    double w = x - L * floor(x / L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    return w;
}

void orc_wrap_positions(int64_t n, const double* pos, const double* box, double* out) {
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) out[3 * i + a] = wrap1(pos[3 * i + a], box[a]);
}

/* ------------------------------------------------------------------ */
/* Brute-force neighbour enumeration                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t j, sj;
    int32_t n[3];
    double d[3];   /* D = (x_j - x_i) + n*L */
} orc_pair;

static int pair_cmp(const void* pa, const void* pb) {
    const orc_pair* a = (const orc_pair*)pa;
    const orc_pair* b = (const orc_pair*)pb;
    if (a->sj != b->sj) return a->sj < b->sj ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    for (int q = 0; q < 3; ++q)
        if (a->n[q] != b->n[q]) return a->n[q] < b->n[q] ? -1 : 1;
    return 0;
}

/* Every (j, n) != (i, 0) with |(x_j - x_i) + n*L|^2 < rlist^2, over all atoms j
 * and every periodic image n that can lie within rlist.  Positions must be
 * wrapped.  The returned array is malloc'ed (caller frees), canonical order
 * (species of j, j, n_x, n_y, n_z). */
static orc_pair* atom_pairs(int64_t i, int64_t n, const double* w, const int32_t* sp, const double* box,
                            double rlist, int* count) {
    int cap = 64, cnt = 0;
    orc_pair* out = (orc_pair*)malloc(sizeof(orc_pair) * cap);
    const double r2 = rlist * rlist;
    for (int64_t j = 0; j < n; ++j) {
        double d0[3];
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            d0[a] = w[3 * j + a] - w[3 * i + a];
            lo[a] = (int)ceil((-rlist - d0[a]) / box[a] - 1e-6);
            hi[a] = (int)floor((rlist - d0[a]) / box[a] + 1e-6);
        }
        for (int nx = lo[0]; nx <= hi[0]; ++nx)
            for (int ny = lo[1]; ny <= hi[1]; ++ny)
                for (int nz = lo[2]; nz <= hi[2]; ++nz) {
                    if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
                    double dx = d0[0] + (double)nx * box[0];
                    double dy = d0[1] + (double)ny * box[1];
                    double dz = d0[2] + (double)nz * box[2];
                    double dd = dx * dx + dy * dy + dz * dz;
                    if (!(dd < r2)) continue;
                    if (cnt == cap) { cap *= 2; out = (orc_pair*)realloc(out, sizeof(orc_pair) * cap); }
                    orc_pair* p = &out[cnt++];
                    p->j = (int32_t)j; p->sj = sp[j];
                    p->n[0] = nx; p->n[1] = ny; p->n[2] = nz;
                    p->d[0] = dx; p->d[1] = dy; p->d[2] = dz;
                }
    }
    qsort(out, cnt, sizeof(orc_pair), pair_cmp);
    *count = cnt;
    return out;
}

/* Full neighbour list, row-major [n][cap] in canonical order.  Returns the
 * largest count; rows longer than cap are truncated (the caller compares the
 * return value with cap). */
int orc_neighbors(int64_t n, const double* pos, const int32_t* sp, const double* box, double rlist, int cap,
                  int32_t* nbr, int32_t* img, int32_t* cnt) {
    double* w = (double*)malloc(sizeof(double) * 3 * n);
    orc_wrap_positions(n, pos, box, w);
    int maxc = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : maxc)
    for (int64_t i = 0; i < n; ++i) {
        int c;
        orc_pair* pr = atom_pairs(i, n, w, sp, box, rlist, &c);
        cnt[i] = c;
        if (c > maxc) maxc = c;
        for (int q = 0; q < cap; ++q) {
            if (q < c) {
                nbr[i * cap + q] = pr[q].j;
                for (int a = 0; a < 3; ++a) img[(i * cap + q) * 3 + a] = pr[q].n[a];
            } else {
                nbr[i * cap + q] = -1;
                for (int a = 0; a < 3; ++a) img[(i * cap + q) * 3 + a] = 0;
            }
        }
        free(pr);
    }
    free(w);
    return maxc;
}

/* Neighbours of one atom (canonical order); returns the count, writes up to cap
 * entries of j, n[3] and D[3]. */
int orc_atom_neighbors(int64_t i, int64_t n, const double* pos, const int32_t* sp, const double* box,
                       double rlist, int cap, int32_t* js, int32_t* imgs, double* ds) {
    double* w = (double*)malloc(sizeof(double) * 3 * n);
    orc_wrap_positions(n, pos, box, w);
    int c;
    orc_pair* pr = atom_pairs(i, n, w, sp, box, rlist, &c);
    for (int q = 0; q < c && q < cap; ++q) {
        js[q] = pr[q].j;
        for (int a = 0; a < 3; ++a) { imgs[3 * q + a] = pr[q].n[a]; ds[3 * q + a] = pr[q].d[a]; }
    }
    free(pr);
    free(w);
    return c;
}

/* ------------------------------------------------------------------ */
/* Radial functions, cutoff, moments                                    */
/* ------------------------------------------------------------------ */
static double cutoff_fc(double R, double rc) { return R < rc ? 0.5 * (cos(M_PI * R / rc) + 1.0) : 0.0; }
static double cutoff_dfc(double R, double rc) { return R < rc ? -0.5 * (M_PI / rc) * sin(M_PI * R / rc) : 0.0; }

static double ipow(double x, int p) {
    double r = 1.0;
    for (int q = 0; q < p; ++q) r *= x;
    return r;
}

/* Exact radial function h_k(R) = exp(-eta_k (R - mu_k)^2) f_c(R) and its
 * derivative (Sec. III.A, H_abck). */
static void radial_exact(const orc_model* m, int k, double R, double* h, double* dh) {
    const double t = R - m->mu[k];
    const double f = exp(-m->eta[k] * t * t);
    const double fc = cutoff_fc(R, m->rcut), dfc = cutoff_dfc(R, m->rcut);
    *h = f * fc;
    *dh = (-2.0 * m->eta[k] * t) * f * fc + f * dfc;
}

/* Tabulated radial functions (Sec. III.B, batch 1-D interpolation of H and
 * H' with the cutoff folded in).  The paper's rational scheme is not printed,
 * so this is piecewise cubic Hermite interpolation, a named substitute: nodes
 * r_j = j delta with delta = rc / ceil(rc / tab_dr) (so that rc is a node),
 * node data (h_k(r_j), h_k'(r_j)) exact, both forced to 0 at r = 0 as the
 * paper does, and 0 for R >= rc.  On [r_j, r_j+1) with t = R/delta - j:
 *   h  = H00(t) f_j + H10(t) delta f'_j + H01(t) f_j+1 + H11(t) delta f'_j+1,
 *   h' = dh/dR of the same cubic,
 * H00 = 2t^3 - 3t^2 + 1, H10 = t^3 - 2t^2 + t, H01 = 3t^2 - 2t^3, H11 = t^3 - t^2
 * (the textbook Hermite basis), so forces stay the exact gradient of the
 * interpolated energy. */
static void radial_node(const orc_model* m, int k, int64_t j, double delta, double* f, double* df) {
    if (j == 0) { *f = 0.0; *df = 0.0; return; }
    radial_exact(m, k, (double)j * delta, f, df);
}

static void radial(const orc_model* m, int k, double R, double* h, double* dh) {
    if (!(m->tab_dr > 0.0)) { radial_exact(m, k, R, h, dh); return; }
    if (!(R < m->rcut)) { *h = 0.0; *dh = 0.0; return; }
    const double nint = ceil(m->rcut / m->tab_dr);
    const double delta = m->rcut / nint;
    int64_t j = (int64_t)floor(R / delta);
    if (j > (int64_t)nint - 1) j = (int64_t)nint - 1;
    const double t = R / delta - (double)j;
    double f0, d0, f1, d1;
    radial_node(m, k, j, delta, &f0, &d0);
    radial_node(m, k, j + 1, delta, &f1, &d1);
    const double t2 = t * t, t3 = t2 * t;
    const double H00 = 2 * t3 - 3 * t2 + 1, H10 = t3 - 2 * t2 + t, H01 = 3 * t2 - 2 * t3, H11 = t3 - t2;
    const double D00 = 6 * t2 - 6 * t, D10 = 3 * t2 - 4 * t + 1, D01 = 6 * t - 6 * t2, D11 = 3 * t2 - 2 * t;
    *h = H00 * f0 + H10 * delta * d0 + H01 * f1 + H11 * delta * d1;
    *dh = (D00 * f0 + D10 * delta * d0 + D01 * f1 + D11 * delta * d1) / delta;
}

/* h_k(R) and h_k'(R) for k = 0..K-1, as the model evaluates them. */
void orc_radial(const orc_model* m, double R, double* h, double* dh) {
    for (int k = 0; k < m->n_radial; ++k) radial(m, k, R, &h[k], &dh[k]);
}

/* M_d(u) = u_x^px u_y^py u_z^pz */
static double moment(int d, const double* u) {
    return ipow(u[0], MONO[d][0]) * ipow(u[1], MONO[d][1]) * ipow(u[2], MONO[d][2]);
}

/* dM_d/du_a */
static double dmoment_du(int d, int a, const double* u) {
    int p[3] = {MONO[d][0], MONO[d][1], MONO[d][2]};
    if (p[a] == 0) return 0.0;
    double r = (double)p[a];
    for (int b = 0; b < 3; ++b) r *= ipow(u[b], b == a ? p[b] - 1 : p[b]);
    return r;
}

/* ------------------------------------------------------------------ */
/* MLP                                                                  */
/* ------------------------------------------------------------------ */
static double act_f(int act, double z) {
    if (act == 1) return 0.5 * (z + sqrt(z * z + 4.0));
    return tanh(z);
}
static double act_df(int act, double z) {
    if (act == 1) return 0.5 * (1.0 + z / sqrt(z * z + 4.0));
    double t = tanh(z);
    return 1.0 - t * t;
}

/* BF16 rounding of an FP32 operand: the value is first rounded to FP32 (the
 * precision the GPU path holds it in), then to the nearest number with an
 * 8-bit significand, ties to even (the IEEE rule; FE_TONEAREST is the default
 * rounding mode, under which nearbyint rounds halfway cases to even).
 * frexp gives x = f 2^e with 0.5 <= |f| < 1, so x 2^(8-e) has its 8
 * significant bits in the integer part.  Below 2^-126 BF16, like FP32, is
 * subnormal: a fixed spacing of 2^-133. */
static double round_bf16(double x) {
    const double xf = (double)(float)x;
    if (xf == 0.0 || !isfinite(xf)) return xf;
    int e;
    (void)frexp(xf, &e);
    if (e < -125) e = -125;
    return ldexp(nearbyint(ldexp(xf, 8 - e)), e - 8);
}

void orc_round_bf16(int64_t n, const double* in, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = round_bf16(in[i]);
}

/* Operand of an MLP matrix product: exact, or rounded to BF16 when the model
 * asks for the BF16 form (reading of the precision form: every operand of a
 * matrix product -- weights, descriptors, hidden activations, back-propagated
 * deltas -- is rounded to BF16 and products are accumulated exactly; biases,
 * activation functions, their derivatives and the output layer stay exact). */
static double opnd(const orc_model* m, double x) { return m->mlp_bf16 ? round_bf16(x) : x; }

/* Forward and input-gradient of the MLP of one species.
 * z_l = W_l a_{l-1} + b_l, a_l = act(z_l), E = w_out . a_L + b_out,
 * dE/dG by back-propagation. */
static double mlp_eval(const orc_model* m, int species, const double* G, double* dG) {
    const int F = orc_n_features(m);
    const double* p = m->params + (size_t)species * orc_params_per_species(m);
    double z[MAXL][MAXW], a[MAXL + 1][MAXW], delta[MAXW], tmp[MAXW];
    int widths[MAXL + 2];
    widths[0] = F;
    for (int l = 0; l < m->n_hidden; ++l) widths[l + 1] = m->hidden[l];
    const double* Wp[MAXL + 1];
    const double* bp[MAXL + 1];
    for (int q = 0; q < F; ++q) a[0][q] = G[q];
    for (int l = 0; l < m->n_hidden; ++l) {
        const int wi = widths[l], wo = widths[l + 1];
        Wp[l] = p; p += (size_t)wo * wi;
        bp[l] = p; p += wo;
        for (int o = 0; o < wo; ++o) {
            double s = bp[l][o];
            for (int q = 0; q < wi; ++q) s += opnd(m, Wp[l][(size_t)o * wi + q]) * opnd(m, a[l][q]);
            z[l][o] = s;
            a[l + 1][o] = act_f(m->activation, s);
        }
    }
    const int L = m->n_hidden, wl = widths[L];
    const double* wout = p;
    const double bout = p[wl];
    double E = bout;
    for (int q = 0; q < wl; ++q) E += wout[q] * a[L][q];
    if (dG) {
        for (int q = 0; q < wl; ++q) delta[q] = wout[q];
        for (int l = L - 1; l >= 0; --l) {
            const int wi = widths[l], wo = widths[l + 1];
            for (int o = 0; o < wo; ++o) delta[o] *= act_df(m->activation, z[l][o]);
            for (int q = 0; q < wi; ++q) {
                double s = 0.0;
                for (int o = 0; o < wo; ++o) s += opnd(m, Wp[l][(size_t)o * wi + q]) * opnd(m, delta[o]);
                tmp[q] = s;
            }
            for (int q = 0; q < wi; ++q) delta[q] = tmp[q];
        }
        for (int q = 0; q < F; ++q) dG[q] = delta[q];
    }
    return E;
}

int orc_mlp(const orc_model* m, int64_t n, const int32_t* species, const double* G, double* E, double* dG) {
    const int F = orc_n_features(m);
    for (int l = 0; l < m->n_hidden; ++l)
        if (m->hidden[l] > MAXW || m->hidden[l] < 1) return ORC_ERR_ARG;
    if (F > MAXW || m->n_hidden > MAXL) return ORC_ERR_ARG;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        E[i] = mlp_eval(m, species[i], G + (size_t)i * F, dG ? dG + (size_t)i * F : NULL);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* One centre atom: descriptor, energy and per-pair gradients          */
/* ------------------------------------------------------------------ */
typedef struct {
    int S, K, M, D, F;
} dims_t;

static dims_t dims_of(const orc_model* m) {
    dims_t d;
    d.S = m->n_species; d.K = m->n_radial; d.M = m->max_moment; d.D = n_moments(m->max_moment);
    d.F = orc_n_features(m);
    return d;
}

/* P[b][k][d] = sum over neighbours c of species b of h_k(R_c) M_d(u_c)
 * (the contraction of H_abck with M_abcd over c, Sec. III.A). */
static void atom_P(const orc_model* m, const orc_pair* pr, int cnt, double* P) {
    const dims_t dm = dims_of(m);
    memset(P, 0, sizeof(double) * dm.S * dm.K * dm.D);
    for (int c = 0; c < cnt; ++c) {
        const double* D = pr[c].d;
        const double R = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        if (!(R < m->rcut)) continue;
        const double u[3] = {D[0] / R, D[1] / R, D[2] / R};
        const int b = pr[c].sj;
        for (int k = 0; k < dm.K; ++k) {
            double h, dh;
            radial(m, k, R, &h, &dh);
            for (int d = 0; d < dm.D; ++d) P[(b * dm.K + k) * dm.D + d] += h * moment(d, u);
        }
    }
}

/* S[b][k][m] = sum_{d of order m} T_d P[b][k][d]^2 and G = sigma(S):
 * sqrt for m = 0, identity for m > 0 (eqns tensor_formalism, sigma_function).
 * Feature index ((b*K + k)*(M+1) + m). */
static void atom_G(const orc_model* m, const double* P, double* S, double* G) {
    const dims_t dm = dims_of(m);
    for (int b = 0; b < dm.S; ++b)
        for (int k = 0; k < dm.K; ++k)
            for (int mm = 0; mm <= dm.M; ++mm) {
                double s = 0.0;
                for (int d = 0; d < dm.D; ++d)
                    if (order_of(d) == mm) s += TDM[d] * P[(b * dm.K + k) * dm.D + d] * P[(b * dm.K + k) * dm.D + d];
                const int f = (b * dm.K + k) * (dm.M + 1) + mm;
                S[f] = s;
                G[f] = (mm == 0) ? sqrt(s) : s;
            }
}

/* Per-pair gradient g_c = dE_i/dD_c from the adjoint chain:
 *   sigma'_bkm = dE/dS_bkm = G'_bkm * dsigma/dS      (0 where S = 0, m = 0)
 *   P'_bkd     = 2 T_d sigma'_{b,k,m(d)} P_bkd        (eqn dP_abkd)
 *   U_ck       = sum_d P'_{b,k,d} M_cd                 (eqn U_abck)
 *   V_cd       = sum_k P'_{b,k,d} H_ck
 *   F1_cx      = sum_k U_ck H'_ck R'_cx,  R' = dR/dD   (eqn F1_abcx)
 *   F2_cx      = sum_d V_cd M'_cxd,      M' = dM/dD   (eqn F2_abcx) */
static void atom_pair_grads(const orc_model* m, const orc_pair* pr, int cnt, const double* P, const double* S,
                            const double* dG, double* g) {
    const dims_t dm = dims_of(m);
    double* Pbar = (double*)malloc(sizeof(double) * dm.S * dm.K * dm.D);
    for (int b = 0; b < dm.S; ++b)
        for (int k = 0; k < dm.K; ++k)
            for (int d = 0; d < dm.D; ++d) {
                const int mm = order_of(d);
                const int f = (b * dm.K + k) * (dm.M + 1) + mm;
                double sbar;
                if (mm == 0) sbar = S[f] > 0.0 ? dG[f] / (2.0 * sqrt(S[f])) : 0.0;
                else sbar = dG[f];
                Pbar[(b * dm.K + k) * dm.D + d] = 2.0 * TDM[d] * sbar * P[(b * dm.K + k) * dm.D + d];
            }
    for (int c = 0; c < cnt; ++c) {
        double* gc = g + 3 * c;
        gc[0] = gc[1] = gc[2] = 0.0;
        const double* D = pr[c].d;
        const double R = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        if (!(R < m->rcut)) continue;
        const double u[3] = {D[0] / R, D[1] / R, D[2] / R};
        const int b = pr[c].sj;
        double H[128], dH[128], Mv[20], dM[20][3];
        for (int k = 0; k < dm.K; ++k) radial(m, k, R, &H[k], &dH[k]);
        for (int d = 0; d < dm.D; ++d) {
            Mv[d] = moment(d, u);
            for (int x = 0; x < 3; ++x) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a) s += dmoment_du(d, a, u) * (((a == x) ? 1.0 : 0.0) - u[a] * u[x]) / R;
                dM[d][x] = s;
            }
        }
        double U[128], V[20];
        for (int k = 0; k < dm.K; ++k) {
            double s = 0.0;
            for (int d = 0; d < dm.D; ++d) s += Pbar[(b * dm.K + k) * dm.D + d] * Mv[d];
            U[k] = s;
        }
        for (int d = 0; d < dm.D; ++d) {
            double s = 0.0;
            for (int k = 0; k < dm.K; ++k) s += Pbar[(b * dm.K + k) * dm.D + d] * H[k];
            V[d] = s;
        }
        for (int x = 0; x < 3; ++x) {
            double f1 = 0.0, f2 = 0.0;
            for (int k = 0; k < dm.K; ++k) f1 += U[k] * dH[k] * u[x];
            for (int d = 0; d < dm.D; ++d) f2 += V[d] * dM[d][x];
            gc[x] = f1 + f2;
        }
    }
    free(Pbar);
}

static int check_model(const orc_model* m) {
    if (m->n_species < 1 || m->n_radial < 1 || m->n_radial > 128 || m->max_moment < 0 || m->max_moment > 3)
        return ORC_ERR_ARG;
    if (m->n_hidden < 0 || m->n_hidden > MAXL || orc_n_features(m) > MAXW || !(m->rcut > 0.0)) return ORC_ERR_ARG;
    for (int l = 0; l < m->n_hidden; ++l)
        if (m->hidden[l] < 1 || m->hidden[l] > MAXW) return ORC_ERR_ARG;
    if (!(m->tab_dr >= 0.0) || m->tab_dr > m->rcut) return ORC_ERR_ARG;
    return ORC_OK;
}

/* Descriptors G [nsel][F] of the selected atoms (all atoms if sel == NULL). */
int orc_descriptors(const orc_model* m, int64_t n, const double* pos, const int32_t* sp, const double* box,
                    int64_t nsel, const int64_t* sel, double* G) {
    if (check_model(m)) return ORC_ERR_ARG;
    const dims_t dm = dims_of(m);
    double* w = (double*)malloc(sizeof(double) * 3 * n);
    orc_wrap_positions(n, pos, box, w);
    if (!sel) nsel = n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nsel; ++q) {
        const int64_t i = sel ? sel[q] : q;
        int c;
        orc_pair* pr = atom_pairs(i, n, w, sp, box, m->rcut, &c);
        double* P = (double*)malloc(sizeof(double) * dm.S * dm.K * dm.D);
        double* S = (double*)malloc(sizeof(double) * dm.F);
        atom_P(m, pr, c, P);
        atom_G(m, P, S, G + (size_t)q * dm.F);
        free(P); free(S); free(pr);
    }
    free(w);
    return ORC_OK;
}

/* Per-atom state of a full evaluation. */
typedef struct {
    orc_pair* pr;
    int cnt;
    double E;
    double* g;   /* [cnt][3] */
} atom_state;

static void atom_evaluate(const orc_model* m, int64_t i, int64_t n, const double* w, const int32_t* sp,
                          const double* box, atom_state* st) {
    const dims_t dm = dims_of(m);
    st->pr = atom_pairs(i, n, w, sp, box, m->rcut, &st->cnt);
    double* P = (double*)malloc(sizeof(double) * dm.S * dm.K * dm.D);
    double* S = (double*)malloc(sizeof(double) * dm.F);
    double* G = (double*)malloc(sizeof(double) * dm.F);
    double* dG = (double*)malloc(sizeof(double) * dm.F);
    atom_P(m, st->pr, st->cnt, P);
    atom_G(m, P, S, G);
    st->E = mlp_eval(m, sp[i], G, dG);
    st->g = (double*)malloc(sizeof(double) * 3 * (st->cnt > 0 ? st->cnt : 1));
    atom_pair_grads(m, st->pr, st->cnt, P, S, dG, st->g);
    free(P); free(S); free(G); free(dG);
}

/* Total energy (Neumaier sum of atomic energies in atom order), atomic
 * energies, forces F = -dE/dx and the virial W_ab = -sum_pairs D_a g_b
 * (full 3x3, row-major).  Any output pointer except energy may be NULL. */
int orc_energy_forces(const orc_model* m, int64_t n, const double* pos, const int32_t* sp, const double* box,
                      double* energy, double* atom_energy, double* forces, double* virial9) {
    if (check_model(m)) return ORC_ERR_ARG;
    double* w = (double*)malloc(sizeof(double) * 3 * n);
    orc_wrap_positions(n, pos, box, w);
    atom_state* st = (atom_state*)calloc(n, sizeof(atom_state));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) atom_evaluate(m, i, n, w, sp, box, &st[i]);
    /* ScatterSum over pairs, serial in atom order (deterministic). */
    double* F = (double*)calloc(3 * n, sizeof(double));
    nsum W[9];
    memset(W, 0, sizeof(W));
    nsum Et = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        nsum_add(&Et, st[i].E);
        if (atom_energy) atom_energy[i] = st[i].E;
        for (int c = 0; c < st[i].cnt; ++c) {
            const double* g = st[i].g + 3 * c;
            const int64_t j = st[i].pr[c].j;
            for (int x = 0; x < 3; ++x) { F[3 * i + x] += g[x]; F[3 * j + x] -= g[x]; }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) nsum_add(&W[3 * a + b], -st[i].pr[c].d[a] * g[b]);
        }
        free(st[i].pr); free(st[i].g);
    }
    *energy = nsum_get(&Et);
    if (forces) memcpy(forces, F, sizeof(double) * 3 * n);
    if (virial9)
        for (int q = 0; q < 9; ++q) virial9[q] = nsum_get(&W[q]);
    free(F); free(st); free(w);
    return ORC_OK;
}

/* Atomic energies and forces of selected atoms only, for systems too large for
 * a full evaluation.  F_i = sum_c g_i(c) - sum over atoms j that list i of
 * g_j(c') for each of their entries c' pointing at i. */
int orc_forces_subset(const orc_model* m, int64_t n, const double* pos, const int32_t* sp, const double* box,
                      int64_t nsel, const int64_t* sel, double* atom_energy, double* forces) {
    if (check_model(m)) return ORC_ERR_ARG;
    double* w = (double*)malloc(sizeof(double) * 3 * n);
    orc_wrap_positions(n, pos, box, w);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nsel; ++q) {
        const int64_t i = sel[q];
        atom_state si;
        atom_evaluate(m, i, n, w, sp, box, &si);
        double F[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < si.cnt; ++c)
            for (int x = 0; x < 3; ++x) F[x] += si.g[3 * c + x];
        /* distinct neighbour atoms (the list is sorted by (species, j)) */
        for (int c = 0; c < si.cnt; ++c) {
            const int32_t j = si.pr[c].j;
            int seen = 0;
            for (int c2 = 0; c2 < c; ++c2)
                if (si.pr[c2].j == j) { seen = 1; break; }
            if (seen) continue;
            atom_state sj;
            if (j == i) sj = si;
            else atom_evaluate(m, j, n, w, sp, box, &sj);
            for (int c3 = 0; c3 < sj.cnt; ++c3)
                if (sj.pr[c3].j == i)
                    for (int x = 0; x < 3; ++x) F[x] -= sj.g[3 * c3 + x];
            if (j != i) { free(sj.pr); free(sj.g); }
        }
        if (atom_energy) atom_energy[q] = si.E;
        for (int x = 0; x < 3; ++x) forces[3 * q + x] = F[x];
        free(si.pr); free(si.g);
    }
    free(w);
    return ORC_OK;
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Force matching (training): descriptor tangent, second-order MLP,     */
/* loss and parameter gradient.  Not part of the paper's method (its    */
/* potentials were trained elsewhere); these are plain definitions.     */
/* ------------------------------------------------------------------ */

/* Tangent of one atom's descriptors along a displacement field r:
 * Gt = d/de G_i(x + e r) at e = 0.  For each pair c the tangent of
 * D_c = x_j + n L - x_i is t = r_j - r_i, and through the definition
 *   R_t = u . t,   u_t = (t - u (u . t)) / R,
 *   Pt_bkd = sum_c [ h_k'(R) R_t M_d(u) + h_k(R) (grad_u M_d) . u_t ],
 *   St_bkm = sum_{d of order m} 2 T_d P_bkd Pt_bkd,
 *   Gt = St / (2 sqrt S) for m = 0 (0 where S = 0), St otherwise. */
static void atom_G_tangent(const orc_model* m, int64_t i, const orc_pair* pr, int cnt, const double* r, double* Gt) {
    const dims_t dm = dims_of(m);
    double* P = (double*)malloc(sizeof(double) * dm.S * dm.K * dm.D);
    double* Pt = (double*)calloc((size_t)dm.S * dm.K * dm.D, sizeof(double));
    double* S = (double*)malloc(sizeof(double) * dm.F);
    double* G = (double*)malloc(sizeof(double) * dm.F);
    atom_P(m, pr, cnt, P);
    atom_G(m, P, S, G);
    for (int c = 0; c < cnt; ++c) {
        const double* D = pr[c].d;
        const double R = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        if (!(R < m->rcut)) continue;
        const double u[3] = {D[0] / R, D[1] / R, D[2] / R};
        const int64_t j = pr[c].j;
        const double t[3] = {r[3 * j] - r[3 * i], r[3 * j + 1] - r[3 * i + 1], r[3 * j + 2] - r[3 * i + 2]};
        const double Rt = u[0] * t[0] + u[1] * t[1] + u[2] * t[2];
        const double ut[3] = {(t[0] - u[0] * Rt) / R, (t[1] - u[1] * Rt) / R, (t[2] - u[2] * Rt) / R};
        const int b = pr[c].sj;
        for (int k = 0; k < dm.K; ++k) {
            double h, dh;
            radial(m, k, R, &h, &dh);
            for (int d = 0; d < dm.D; ++d) {
                double Mt = 0.0;
                for (int a = 0; a < 3; ++a) Mt += dmoment_du(d, a, u) * ut[a];
                Pt[(b * dm.K + k) * dm.D + d] += dh * Rt * moment(d, u) + h * Mt;
            }
        }
    }
    for (int b = 0; b < dm.S; ++b)
        for (int k = 0; k < dm.K; ++k)
            for (int mm = 0; mm <= dm.M; ++mm) {
                double st = 0.0;
                for (int d = 0; d < dm.D; ++d)
                    if (order_of(d) == mm)
                        st += 2.0 * TDM[d] * P[(b * dm.K + k) * dm.D + d] * Pt[(b * dm.K + k) * dm.D + d];
                const int f = (b * dm.K + k) * (dm.M + 1) + mm;
                Gt[f] = (mm == 0) ? (S[f] > 0.0 ? st / (2.0 * sqrt(S[f])) : 0.0) : st;
            }
    free(P); free(Pt); free(S); free(G);
}

/* Descriptor tangents w [n][F] of every atom along the field r [n][3]. */
int orc_descriptor_jvp(const orc_model* m, int64_t n, const double* pos, const int32_t* sp, const double* box,
                       const double* r, double* w) {
    if (check_model(m)) return ORC_ERR_ARG;
    const dims_t dm = dims_of(m);
    double* wp = (double*)malloc(sizeof(double) * 3 * n);
    orc_wrap_positions(n, pos, box, wp);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        int c;
        orc_pair* pr = atom_pairs(i, n, wp, sp, box, m->rcut, &c);
        atom_G_tangent(m, i, pr, c, r, w + (size_t)i * dm.F);
        free(pr);
    }
    free(wp);
    return ORC_OK;
}

static double act_d2f(int act, double z) {
    if (act == 1) return 2.0 / pow(z * z + 4.0, 1.5);
    double t = tanh(z);
    return -2.0 * t * (1.0 - t * t);
}

/* One atom of the second-order network pass.  Primal z_l = W_l a_{l-1} + b_l,
 * a_l = act(z_l), E = w_out . a_L + b_out; tangent along the input direction
 * w: zt_l = W_l at_{l-1}, at_l = act'(z_l) zt_l, q = w_out . at_L (so q is
 * grad_G E . w).  Reverse mode of J = e E - q through both graphs, adding
 * dJ/dtheta into g (this species' parameter block). */
static void mlp_second_atom(const orc_model* m, int species, const double* G, const double* w, double e,
                            double* E_out, double* q_out, double* g) {
    const int F = orc_n_features(m);
    const double* p = m->params + (size_t)species * orc_params_per_species(m);
    static __thread double z[MAXL][MAXW], zt[MAXL][MAXW], a[MAXL + 1][MAXW], at[MAXL + 1][MAXW];
    static __thread double ab[MAXW], atb[MAXW], zb[MAXW], ztb[MAXW], nab[MAXW], natb[MAXW];
    int widths[MAXL + 2];
    widths[0] = F;
    for (int l = 0; l < m->n_hidden; ++l) widths[l + 1] = m->hidden[l];
    size_t offW[MAXL], offb[MAXL];
    size_t off = 0;
    for (int l = 0; l < m->n_hidden; ++l) {
        offW[l] = off; off += (size_t)widths[l + 1] * widths[l];
        offb[l] = off; off += widths[l + 1];
    }
    const int L = m->n_hidden, wl = widths[L];
    const size_t off_wout = off, off_bout = off + wl;
    for (int q = 0; q < F; ++q) { a[0][q] = G[q]; at[0][q] = w[q]; }
    for (int l = 0; l < L; ++l) {
        const int wi = widths[l], wo = widths[l + 1];
        const double* W = p + offW[l];
        for (int o = 0; o < wo; ++o) {
            double s = p[offb[l] + o], st = 0.0;
            for (int q = 0; q < wi; ++q) {
                s += W[(size_t)o * wi + q] * a[l][q];
                st += W[(size_t)o * wi + q] * at[l][q];
            }
            z[l][o] = s;
            zt[l][o] = st;
            a[l + 1][o] = act_f(m->activation, s);
            at[l + 1][o] = act_df(m->activation, s) * st;
        }
    }
    double E = p[off_bout], q = 0.0;
    for (int o = 0; o < wl; ++o) {
        E += p[off_wout + o] * a[L][o];
        q += p[off_wout + o] * at[L][o];
    }
    *E_out = E;
    *q_out = q;
    /* output layer */
    for (int o = 0; o < wl; ++o) {
        g[off_wout + o] += e * a[L][o] - at[L][o];
        ab[o] = e * p[off_wout + o];
        atb[o] = -p[off_wout + o];
    }
    g[off_bout] += e;
    for (int l = L - 1; l >= 0; --l) {
        const int wi = widths[l], wo = widths[l + 1];
        const double* W = p + offW[l];
        for (int o = 0; o < wo; ++o) {
            const double d1 = act_df(m->activation, z[l][o]), d2 = act_d2f(m->activation, z[l][o]);
            ztb[o] = d1 * atb[o];
            zb[o] = d1 * ab[o] + d2 * zt[l][o] * atb[o];
        }
        for (int o = 0; o < wo; ++o) {
            for (int qq = 0; qq < wi; ++qq) g[offW[l] + (size_t)o * wi + qq] += zb[o] * a[l][qq] + ztb[o] * at[l][qq];
            g[offb[l] + o] += zb[o];
        }
        if (l > 0) {
            for (int qq = 0; qq < wi; ++qq) {
                double s = 0.0, st = 0.0;
                for (int o = 0; o < wo; ++o) {
                    s += W[(size_t)o * wi + qq] * zb[o];
                    st += W[(size_t)o * wi + qq] * ztb[o];
                }
                nab[qq] = s;
                natb[qq] = st;
            }
            for (int qq = 0; qq < wi; ++qq) { ab[qq] = nab[qq]; atb[qq] = natb[qq]; }
        }
    }
}

/* E_a, q_a and grad = d/dtheta sum_a (e_a E_a - q_a), grad [S * params per
 * species] overwritten; atoms are visited in index order. */
int orc_mlp_second(const orc_model* m, int64_t n, const int32_t* species, const double* G, const double* w,
                   const double* e, double* E, double* q, double* grad) {
    if (check_model(m)) return ORC_ERR_ARG;
    const int F = orc_n_features(m);
    const size_t np = (size_t)m->n_species * orc_params_per_species(m);
    memset(grad, 0, sizeof(double) * np);
    for (int64_t i = 0; i < n; ++i) {
        const int s = species[i];
        double* g = grad + (size_t)s * orc_params_per_species(m);
        mlp_second_atom(m, s, G + (size_t)i * F, w + (size_t)i * F, e[i], &E[i], &q[i], g);
    }
    return ORC_OK;
}

/* Force-matching loss over a batch of B periodic systems (system s holds atoms
 * sys_off[s] .. sys_off[s+1]-1 in a box boxes[3s..3s+2]):
 *   L = (1/B) sum_s ((E_s - Ehat_s)/N_s)^2 + lambda/(3 N) sum_i |F_i - Fhat_i|^2,
 * N = total atoms.  The gradient is assembled from
 *   dL/dE_a = e_a = (2/B)(E_s - Ehat_s)/N_s^2          (energy term)
 *   dL/dF_i = r_i = (2 lambda/(3N)) (F_i - Fhat_i)     (force term)
 * and F = -dE/dx: sum_i r_i . dF_i/dtheta = -d/dtheta sum_a q_a with q_a the
 * network tangent along the descriptor tangent of the field r.  loss_e and
 * loss_f receive the two terms (nullable); grad [S * params per species]. */
int orc_train_loss_grad(const orc_model* m, int32_t n_sys, const int64_t* sys_off, const double* pos,
                        const int32_t* sp, const double* boxes, const double* E_label, const double* F_label,
                        double lambda, double* loss, double* loss_e, double* loss_f, double* grad) {
    if (check_model(m) || n_sys < 1) return ORC_ERR_ARG;
    const int F = orc_n_features(m);
    const size_t np = (size_t)m->n_species * orc_params_per_species(m);
    const int64_t N = sys_off[n_sys] - sys_off[0];
    memset(grad, 0, sizeof(double) * np);
    double* gs = (double*)malloc(sizeof(double) * np);
    nsum le = {0.0, 0.0}, lf = {0.0, 0.0};
    for (int32_t s = 0; s < n_sys; ++s) {
        const int64_t o = sys_off[s], ns = sys_off[s + 1] - sys_off[s];
        const double* x = pos + 3 * o;
        const int32_t* spp = sp + o;
        const double* box = boxes + 3 * s;
        double Es;
        double* Fs = (double*)malloc(sizeof(double) * 3 * ns);
        double* r = (double*)malloc(sizeof(double) * 3 * ns);
        double* G = (double*)malloc(sizeof(double) * ns * F);
        double* w = (double*)malloc(sizeof(double) * ns * F);
        double* e = (double*)malloc(sizeof(double) * ns);
        double* Ea = (double*)malloc(sizeof(double) * ns);
        double* qa = (double*)malloc(sizeof(double) * ns);
        int st = orc_energy_forces(m, ns, x, spp, box, &Es, NULL, Fs, NULL);
        if (!st) st = orc_descriptors(m, ns, x, spp, box, 0, NULL, G);
        if (st) {
            free(Fs); free(r); free(G); free(w); free(e); free(Ea); free(qa); free(gs);
            return st;
        }
        const double de = (Es - E_label[s]) / (double)ns;
        nsum_add(&le, de * de / (double)n_sys);
        for (int64_t i = 0; i < ns; ++i)
            for (int a = 0; a < 3; ++a) {
                const double df = Fs[3 * i + a] - F_label[3 * (o + i) + a];
                nsum_add(&lf, lambda * df * df / (3.0 * (double)N));
                r[3 * i + a] = 2.0 * lambda / (3.0 * (double)N) * df;
            }
        for (int64_t i = 0; i < ns; ++i) e[i] = 2.0 / (double)n_sys * (Es - E_label[s]) / ((double)ns * (double)ns);
        orc_descriptor_jvp(m, ns, x, spp, box, r, w);
        orc_mlp_second(m, ns, spp, G, w, e, Ea, qa, gs);
        for (size_t q = 0; q < np; ++q) grad[q] += gs[q];
        free(Fs); free(r); free(G); free(w); free(e); free(Ea); free(qa);
    }
    free(gs);
    if (loss_e) *loss_e = nsum_get(&le);
    if (loss_f) *loss_f = nsum_get(&lf);
    *loss = nsum_get(&le) + nsum_get(&lf);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Velocity-Verlet NVE                                                  */
/* ------------------------------------------------------------------ */
#define ORC_ACC_CONV 9.648533e-3   /* (eV/A)/amu -> A/fs^2 */
#define ORC_KE_CONV 103.6427       /* amu (A/fs)^2 -> eV */

static double kinetic(int64_t n, const double* vel, const int32_t* sp, const double* mass) {
    nsum k = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        nsum_add(&k, 0.5 * ORC_KE_CONV * mass[sp[i]] *
                         (vel[3 * i] * vel[3 * i] + vel[3 * i + 1] * vel[3 * i + 1] + vel[3 * i + 2] * vel[3 * i + 2]));
    return nsum_get(&k);
}

/* n_steps of velocity Verlet in the microcanonical ensemble:
 *   v += (dt/2) a(x);  x += dt v;  v += (dt/2) a(x),   a = ACC_CONV F / m,
 * forces from the full FP64 evaluation at every step (neighbours rebuilt by
 * brute force each time).  pos and vel [n][3] are advanced in place and never
 * wrapped.  epot and ekin (nullable, n_steps + 1 entries) get the potential and
 * kinetic energy before the first step and after each step. */
int orc_nve(const orc_model* m, int64_t n, double* pos, double* vel, const int32_t* sp, const double* mass,
            const double* box, double dt, int n_steps, double* epot, double* ekin) {
    if (check_model(m) || n_steps < 0) return ORC_ERR_ARG;
    double* F = (double*)malloc(sizeof(double) * 3 * n);
    double E;
    int st = orc_energy_forces(m, n, pos, sp, box, &E, NULL, F, NULL);
    if (st) { free(F); return st; }
    if (epot) epot[0] = E;
    if (ekin) ekin[0] = kinetic(n, vel, sp, mass);
    for (int t = 0; t < n_steps; ++t) {
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                vel[3 * i + a] += 0.5 * dt * ORC_ACC_CONV * F[3 * i + a] / mass[sp[i]];
                pos[3 * i + a] += dt * vel[3 * i + a];
            }
        st = orc_energy_forces(m, n, pos, sp, box, &E, NULL, F, NULL);
        if (st) { free(F); return st; }
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) vel[3 * i + a] += 0.5 * dt * ORC_ACC_CONV * F[3 * i + a] / mass[sp[i]];
        if (epot) epot[t + 1] = E;
        if (ekin) ekin[t + 1] = kinetic(n, vel, sp, mass);
    }
    free(F);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Nose-Hoover NVT (the MD protocol of Sec. IV.D runs NVT at 300 K; the */
/* paper does not name its thermostat)                                  */
/* ------------------------------------------------------------------ */
#define ORC_KB 8.617333262e-5      /* eV/K */

/* Kinetic energy and its diagonal tensor components (eV). */
static void kinetic_tensor(int64_t n, const double* vel, const int32_t* sp, const double* mass, double* ke,
                           double* kxyz) {
    nsum k[3];
    memset(k, 0, sizeof(k));
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) nsum_add(&k[a], 0.5 * ORC_KE_CONV * mass[sp[i]] * vel[3 * i + a] * vel[3 * i + a]);
    for (int a = 0; a < 3; ++a) kxyz[a] = nsum_get(&k[a]);
    *ke = kxyz[0] + kxyz[1] + kxyz[2];
}

/* One thermostat half step of the Nose-Hoover Trotter splitting (one
 * thermostat variable xi with mass Q = g kB T tau^2, thermostat position eta):
 *   xi += (dt/4) G;  v *= exp(-xi dt/2), eta += xi dt/2;  xi += (dt/4) G,
 * G = (2 KE - g kB T) / Q with KE after the scaling for the second update.
 * ke is updated. */
static void nh_half(int64_t n, double* vel, double* ke, double g, double kT, double Q, double dt, double* xi,
                    double* eta) {
    *xi += 0.25 * dt * (2.0 * (*ke) - g * kT) / Q;
    const double s = exp(-(*xi) * 0.5 * dt);
    for (int64_t i = 0; i < 3 * n; ++i) vel[i] *= s;
    *ke *= s * s;
    *eta += 0.5 * dt * (*xi);
    *xi += 0.25 * dt * (2.0 * (*ke) - g * kT) / Q;
}

/* n_steps of Nose-Hoover NVT: thermostat half step, velocity Verlet
 * (v += dt/2 a, x += dt v, F(x), v += dt/2 a), thermostat half step.
 * g = 3n degrees of freedom; tau_fs the thermostat period.  xi_eta [2] holds
 * (xi, eta) in and out.  epot, ekin, conserved [n_steps + 1] (nullable):
 * potential, kinetic and the conserved H = PE + KE + Q xi^2 / 2 + g kB T eta. */
int orc_nvt(const orc_model* m, int64_t n, double* pos, double* vel, const int32_t* sp, const double* mass,
            const double* box, double dt, double T, double tau_fs, int n_steps, double* xi_eta, double* epot,
            double* ekin, double* conserved) {
    if (check_model(m) || n_steps < 0 || !(T > 0.0) || !(tau_fs > 0.0)) return ORC_ERR_ARG;
    const double g = 3.0 * (double)n, kT = ORC_KB * T, Q = g * kT * tau_fs * tau_fs;
    double xi = xi_eta[0], eta = xi_eta[1];
    double* F = (double*)malloc(sizeof(double) * 3 * n);
    double E, ke, kx[3];
    int st = orc_energy_forces(m, n, pos, sp, box, &E, NULL, F, NULL);
    if (st) { free(F); return st; }
    kinetic_tensor(n, vel, sp, mass, &ke, kx);
    if (epot) epot[0] = E;
    if (ekin) ekin[0] = ke;
    if (conserved) conserved[0] = E + ke + 0.5 * Q * xi * xi + g * kT * eta;
    for (int t = 0; t < n_steps; ++t) {
        nh_half(n, vel, &ke, g, kT, Q, dt, &xi, &eta);
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                vel[3 * i + a] += 0.5 * dt * ORC_ACC_CONV * F[3 * i + a] / mass[sp[i]];
                pos[3 * i + a] += dt * vel[3 * i + a];
            }
        st = orc_energy_forces(m, n, pos, sp, box, &E, NULL, F, NULL);
        if (st) { free(F); return st; }
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) vel[3 * i + a] += 0.5 * dt * ORC_ACC_CONV * F[3 * i + a] / mass[sp[i]];
        kinetic_tensor(n, vel, sp, mass, &ke, kx);
        nh_half(n, vel, &ke, g, kT, Q, dt, &xi, &eta);
        if (epot) epot[t + 1] = E;
        if (ekin) ekin[t + 1] = ke;
        if (conserved) conserved[t + 1] = E + ke + 0.5 * Q * xi * xi + g * kT * eta;
    }
    xi_eta[0] = xi;
    xi_eta[1] = eta;
    free(F);
    return ORC_OK;
}

/* Instantaneous pressure tensor diagonal and pressure (GPa) from velocities and
 * the virial: p_aa = (2 KE_aa + W_aa) / V, P = (p_xx + p_yy + p_zz)/3. */
int orc_pressure(const orc_model* m, int64_t n, const double* pos, const double* vel, const int32_t* sp,
                 const double* mass, const double* box, double* p4) {
    if (check_model(m)) return ORC_ERR_ARG;
    double E, W[9], ke, kx[3];
    int st = orc_energy_forces(m, n, pos, sp, box, &E, NULL, NULL, W);
    if (st) return st;
    kinetic_tensor(n, vel, sp, mass, &ke, kx);
    const double V = box[0] * box[1] * box[2], conv = 160.21766208; /* eV/A^3 -> GPa */
    for (int a = 0; a < 3; ++a) p4[a] = (2.0 * kx[a] + W[4 * a]) / V * conv;
    p4[3] = (p4[0] + p4[1] + p4[2]) / 3.0;
    return ORC_OK;
}
