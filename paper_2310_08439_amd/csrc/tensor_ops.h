// Per-pair tensor algebra shared by the energy/force kernels and the
// training kernels: the moment monomials M_d(u) in the row order of the
// multiplicity table T_dm (Sec. III.A, eqn T_dm), their adjoint (the F2 term
// of the force, eqn F2_abcx) and their directional derivative (the descriptor
// tangent used by force matching).
#pragma once

#include <hip/hip_runtime.h>

namespace tmd {
namespace ops {

constexpr float kLog2e = 1.4426950408889634f;

template <int M>
struct Moments {
    static constexpr int D = (M + 1) * (M + 2) * (M + 3) / 6;
    // Components left once the unit-norm identity z^2 = 1 - x^2 - y^2 has
    // removed zz (M >= 2) and xzz, yzz, zzz (M = 3); see reduced_monomials.
    static constexpr int DR = M == 3 ? 16 : (M == 2 ? 9 : D);
};

// Multiplicity of moment component d (T_dm row order: 1; x y z; xx xy xz yy
// yz zz; xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz).
__device__ constexpr float kMult[20] = {1, 1, 1, 1, 1, 2, 2, 1, 2, 1, 1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
__device__ constexpr int kOrderStart[5] = {0, 1, 4, 10, 20};

template <int M>
__device__ __forceinline__ void monomials(float x, float y, float z, float* Mv) {
    Mv[0] = 1.0f;
    if constexpr (M >= 1) {
        Mv[1] = x;
        Mv[2] = y;
        Mv[3] = z;
    }
    if constexpr (M >= 2) {
        Mv[4] = x * x;
        Mv[5] = x * y;
        Mv[6] = x * z;
        Mv[7] = y * y;
        Mv[8] = y * z;
        Mv[9] = z * z;
    }
    if constexpr (M >= 3) {
        Mv[10] = Mv[4] * x;
        Mv[11] = Mv[4] * y;
        Mv[12] = Mv[4] * z;
        Mv[13] = x * Mv[7];
        Mv[14] = x * Mv[8];
        Mv[15] = x * Mv[9];
        Mv[16] = Mv[7] * y;
        Mv[17] = Mv[7] * z;
        Mv[18] = y * Mv[9];
        Mv[19] = Mv[9] * z;
    }
}

// Reduced moment basis.  For a unit vector u, zz = 1 - xx - yy, so
//   zz = 1 - xx - yy,  xzz = x - xxx - xyy,  yzz = y - xxy - yyy,  zzz = z - xxz - yyz,
// and any linear form in the 20 monomials equals, on the unit sphere, a form in
// the other 16: 1; x y z; xx xy xz yy yz; xxx xxy xxz xyy xyz yyy yyz (M = 3;
// for M = 2 the 9 without zz).  This holds for each neighbour's monomials, so
// for their sums P too (expand_P recovers the dropped components), and for
// the adjoint's polynomial sum_d P'_d M_d(u) (fold_Pbar moves the dropped
// coefficients onto the kept ones).  Index of a kept component in the full
// T_dm row order:
template <int M>
__device__ __forceinline__ constexpr int full_index(int r) {
    if constexpr (M < 2) return r;
    else if constexpr (M == 2) return r;  // 0..8 (zz = 9 dropped)
    else return r < 9 ? r : (r < 14 ? r + 1 : r + 2);  // xxx..xyz -> 10..14, yyy yyz -> 16 17
}

template <int M>
__device__ __forceinline__ void reduced_monomials(float x, float y, float z, float* Mv) {
    Mv[0] = 1.0f;
    if constexpr (M >= 1) {
        Mv[1] = x;
        Mv[2] = y;
        Mv[3] = z;
    }
    if constexpr (M >= 2) {
        Mv[4] = x * x;
        Mv[5] = x * y;
        Mv[6] = x * z;
        Mv[7] = y * y;
        Mv[8] = y * z;
    }
    if constexpr (M >= 3) {
        Mv[9] = Mv[4] * x;
        Mv[10] = Mv[4] * y;
        Mv[11] = Mv[4] * z;
        Mv[12] = x * Mv[7];
        Mv[13] = x * Mv[8];
        Mv[14] = Mv[7] * y;
        Mv[15] = Mv[7] * z;
    }
}

// The full 20 (or 10) components of P from its kept ones: the unit-norm
// identity applied to each neighbour's monomials, summed.
template <int M, int KC>
__device__ __forceinline__ void expand_P(const float (&Pr)[KC][Moments<M>::DR], float (&P)[KC][Moments<M>::D]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
        for (int r = 0; r < Moments<M>::DR; ++r) P[kk][full_index<M>(r)] = Pr[kk][r];
        if constexpr (M >= 2) P[kk][9] = Pr[kk][0] - Pr[kk][4] - Pr[kk][7];
        if constexpr (M >= 3) {
            P[kk][15] = Pr[kk][1] - Pr[kk][9] - Pr[kk][12];
            P[kk][18] = Pr[kk][2] - Pr[kk][10] - Pr[kk][14];
            P[kk][19] = Pr[kk][3] - Pr[kk][11] - Pr[kk][15];
        }
    }
}

// Coefficients of sum_d Pb_d M_d(u) in the kept basis (equal on the unit sphere).
template <int M, int KC>
__device__ __forceinline__ void fold_Pbar(const float (&P)[KC][Moments<M>::D], float (&Pr)[KC][Moments<M>::DR]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
#pragma unroll
        for (int r = 0; r < Moments<M>::DR; ++r) Pr[kk][r] = P[kk][full_index<M>(r)];
        if constexpr (M >= 2) {
            Pr[kk][0] += P[kk][9];
            Pr[kk][4] -= P[kk][9];
            Pr[kk][7] -= P[kk][9];
        }
        if constexpr (M >= 3) {
            Pr[kk][1] += P[kk][15];
            Pr[kk][9] -= P[kk][15];
            Pr[kk][12] -= P[kk][15];
            Pr[kk][2] += P[kk][18];
            Pr[kk][10] -= P[kk][18];
            Pr[kk][14] -= P[kk][18];
            Pr[kk][3] += P[kk][19];
            Pr[kk][11] -= P[kk][19];
            Pr[kk][15] -= P[kk][19];
        }
    }
}

// A = sum_r V_r grad_u M_r over the kept basis (the ambient gradient; only its
// part tangent to the sphere enters a force, and that part is the same for
// every form equal on the sphere) and B = u . A.
template <int M>
__device__ __forceinline__ void reduced_moment_adjoint(float x, float y, float z, const float* V, const float* Mv,
                                                       float& Ax, float& Ay, float& Az, float& B) {
    Ax = Ay = Az = 0.0f;
    if constexpr (M >= 1) {
        Ax = V[1];
        Ay = V[2];
        Az = V[3];
    }
    if constexpr (M >= 2) {
        Ax += 2.0f * x * V[4] + y * V[5] + z * V[6];
        Ay += x * V[5] + 2.0f * y * V[7] + z * V[8];
        Az += x * V[6] + y * V[8];
    }
    if constexpr (M >= 3) {
        const float xx = Mv[4], xy = Mv[5], xz = Mv[6], yy = Mv[7], yz = Mv[8];
        Ax += 3.0f * xx * V[9] + 2.0f * xy * V[10] + 2.0f * xz * V[11] + yy * V[12] + yz * V[13];
        Ay += xx * V[10] + 2.0f * xy * V[12] + xz * V[13] + 3.0f * yy * V[14] + 2.0f * yz * V[15];
        Az += xx * V[11] + xy * V[13] + yy * V[15];
    }
    B = x * Ax + y * Ay + z * Az;
}

// A = sum_d V_d grad_u M_d and B = sum_d ord(d) V_d M_d.
template <int M>
__device__ __forceinline__ void moment_adjoint(float x, float y, float z, const float* V, const float* Mv,
                                               float& Ax, float& Ay, float& Az, float& B) {
    Ax = Ay = Az = 0.0f;
    if constexpr (M >= 1) {
        Ax = V[1];
        Ay = V[2];
        Az = V[3];
    }
    if constexpr (M >= 2) {
        Ax += 2.0f * x * V[4] + y * V[5] + z * V[6];
        Ay += x * V[5] + 2.0f * y * V[7] + z * V[8];
        Az += x * V[6] + y * V[8] + 2.0f * z * V[9];
    }
    if constexpr (M >= 3) {
        const float xx = Mv[4], xy = Mv[5], xz = Mv[6], yy = Mv[7], yz = Mv[8], zz = Mv[9];
        Ax += 3.0f * xx * V[10] + 2.0f * xy * V[11] + 2.0f * xz * V[12] + yy * V[13] + yz * V[14] + zz * V[15];
        Ay += xx * V[11] + 2.0f * xy * V[13] + xz * V[14] + 3.0f * yy * V[16] + 2.0f * yz * V[17] + zz * V[18];
        Az += xx * V[12] + xy * V[14] + 2.0f * xz * V[15] + yy * V[17] + 2.0f * yz * V[18] + 3.0f * zz * V[19];
    }
    // sum_d ord(d) V_d M_d = u . A: the monomials of order m are homogeneous of
    // degree m, so u . grad M_d = m M_d (Euler)
    B = x * Ax + y * Ay + z * Az;
}

// Directional derivative of the monomials along t: Mt_d = grad_u M_d . t.
template <int M>
__device__ __forceinline__ void monomial_tangent(const float* Mv, float x, float y, float z, float tx, float ty,
                                                 float tz, float* Mt) {
    Mt[0] = 0.0f;
    if constexpr (M >= 1) {
        Mt[1] = tx;
        Mt[2] = ty;
        Mt[3] = tz;
    }
    if constexpr (M >= 2) {
        Mt[4] = 2.0f * x * tx;
        Mt[5] = tx * y + x * ty;
        Mt[6] = tx * z + x * tz;
        Mt[7] = 2.0f * y * ty;
        Mt[8] = ty * z + y * tz;
        Mt[9] = 2.0f * z * tz;
    }
    if constexpr (M >= 3) {
        const float xx = Mv[4], xy = Mv[5], xz = Mv[6], yy = Mv[7], yz = Mv[8], zz = Mv[9];
        Mt[10] = 3.0f * xx * tx;
        Mt[11] = 2.0f * xy * tx + xx * ty;
        Mt[12] = 2.0f * xz * tx + xx * tz;
        Mt[13] = yy * tx + 2.0f * xy * ty;
        Mt[14] = yz * tx + xz * ty + xy * tz;
        Mt[15] = zz * tx + 2.0f * xz * tz;
        Mt[16] = 3.0f * yy * ty;
        Mt[17] = 2.0f * yz * ty + yy * tz;
        Mt[18] = zz * ty + 2.0f * yz * tz;
        Mt[19] = 3.0f * zz * tz;
    }
}

}  // namespace ops
}  // namespace tmd
