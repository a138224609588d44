// gfx950 kernels of the pseudo-potential D2Q9 lattice Boltzmann step (arXiv:1412.5170).
//
// State: FP32 populations, population q of node (x, y) at y * frow + q * fq + x (nine planes
// either one after the other, fq = pitch * ny, frow = pitch, or interleaved by rows,
// fq = pitch, frow = 9 * pitch), double-buffered; one FP32 psi plane (y * pitch + x).
//
// A time step is either
//   psi_kernel + fused_kernel (two passes): the first pass forms rho = sum_q f_q (Eq. 3) and
//     psi from the K-rescaled Carnahan-Starling EOS (Eq. 29-30) through p0 = rho/3 + G psi^2/2
//     (Eq. 7) and writes psi; the second stages psi of a tile and its one-node halo in LDS,
//     forms the interaction force (Eq. 6; Eq. 4 for A = 0), the velocities (Sec. 3.2), the
//     forcing scheme (EDM Eq. 22, Guo Eq. 23, Guo + Li Eq. 31), the BGK (Eq. 1) or MRT
//     (Eq. 34-35) collision, and pushes f* to the neighbours (Eq. 36, periodic);
// or
//   sweep_kernel (one pass): the same per-node arithmetic, with psi computed from the
//     populations as each row is loaded and kept in an LDS ring, so each population is read
//     once per step.
//
// Arithmetic: D is the type of every quantity of the size of a population (rho, momentum,
// the force and the velocities, f^eq - f and its moments, the update, the mass closure, the
// EOS), whose rounding decides the accuracy of the FP32 state; R is the type of the small
// relative terms (equilibrium shape, Guo's bracket and source, Li's term).
// (R, D) = (float, float), (double, double) or (float, double).
//
// Velocity order: 0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1),
// 7 (-1,-1), 8 (1,-1).  All formulas below are unrolled by hand for this order.

#include <cmath>
#include <cstdint>
#include <mutex>

#include "lbm_internal.h"

namespace pplbm {
namespace {

template <typename T>
__device__ __forceinline__ T qnan();
template <>
__device__ __forceinline__ float qnan<float>() { return __builtin_nanf(""); }
template <>
__device__ __forceinline__ double qnan<double>() { return __builtin_nan(""); }

__device__ __forceinline__ int wrap_any(int g, int n) {
    g %= n;
    return g < 0 ? g + n : g;
}

// rho = sum_q f_q in one fixed order, shared by every kernel that needs it.
template <typename T>
__device__ __forceinline__ T density(T f0, T f1, T f2, T f3, T f4, T f5, T f6, T f7, T f8) {
    return ((f0 + (f1 + f3)) + (f2 + f4)) + ((f5 + f7) + (f6 + f8));
}

template <typename T>
__device__ __forceinline__ T density9(const float f[9]) {
    return density<T>(f[0], f[1], f[2], f[3], f[4], f[5], f[6], f[7], f[8]);
}

// 1 / x for x > 0 from the hardware reciprocal: in FP32 as it is (1 ulp); in FP64 refined by
// one Newton step, which squares the estimate's relative error (an estimate good to single
// precision comes out good to about 2^-46, far below the FP32 rounding of the stored state).
template <typename T>
__device__ __forceinline__ T recip(T x) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_amdgcn_rcpf(x);
    } else {
        const T r = __builtin_amdgcn_rcp(x);
        return fma(r, fma(-x, r, T(1)), r);
    }
}

// Effective density of Eq. 7 with the rescaled Carnahan-Starling pressure of Eq. 29-30,
// p0 = K rho (R T Z - a rho), Z = (1 + eta + eta^2 - eta^3) / (1 - eta)^3, eta = b rho / 4.
// The radicand 2 (p0 - rho/3) / G is formed as rho (e1 Z - (e2 rho + e3)) with the constants
// e1 = 2 K R T / G, e2 = 2 K a / G, e3 = 2 / (3 G) folded on the host.  NaN when the node is
// outside the EOS (b rho/4 >= 1, rho <= 0) or 2 U / G <= 0.
template <typename T>
__device__ __forceinline__ T eos_psi(T rho, T bq, T e1, T e2, T e3) {
    const T eta = bq * rho;
    const T om = T(1) - eta;
    const T Z = (T(1) + eta * (T(1) + eta * om)) * recip<T>(om * om * om);
    const T r = rho * (e1 * Z - (e2 * rho + e3));
    // psi is stored in FP32, so its square root is the hardware FP32 one (1 ulp) of the
    // radicand rounded once.
    const bool ok = eta < T(1) && rho > T(0) && r > T(0);
    return ok ? T(__builtin_amdgcn_sqrtf((float)r)) : qnan<T>();
}

// Effective density of Eq. 33 (Sbragaglia-Shan): exp(-1/rho) for eps = 0 (inv_eps = 0 flags
// it), (rho / (1 + rho))^(1/eps) otherwise.  The EOS is then the one Eq. 7 implies.
template <typename T>
__device__ __forceinline__ T ss_psi(T rho, T inv_eps) {
    if (!(rho > T(0))) return qnan<T>();
    if (inv_eps == T(0)) return exp(-T(1) / rho);
    return exp(inv_eps * log(rho / (T(1) + rho)));
}

// ---------------------------------------------------------------------------------------
// Constants of a step, converted once on the host.
// ---------------------------------------------------------------------------------------
template <typename R, typename D>
struct StepConst {
    int nx, ny;
    size_t pitch;      // psi row stride (floats)
    size_t frow, fq;   // population row and velocity strides (floats)
    unsigned fbytes;   // bytes of one population buffer when below 4 GiB (whole-buffer resource)
    size_t ffloats;    // floats of one population buffer (per-row resources beyond 4 GiB)
    int flags;         // kFlagNT | kFlagXCD
    D bq, e1, e2, e3;  // EOS (Eq. 29-30) through Eq. 7: b/4 and the constants of eos_psi
    int psi_kind;     // 0: psi from the C-S EOS through Eq. 7; 1: psi of Eq. 33
    D inv_eps;        // Eq. 33 exponent 1/eps (0: the exp(-1/rho) branch)
    D tau;            // relaxation time (Shan-Chen velocity shift, Eq. 21)
    D gA;     // -G A / 2        coefficient of sum w psi^2 e    (Eq. 6, U = G psi^2 / 2)
    D gB;     // -G (1 - A)      coefficient of psi(x) sum w psi e
    D omega;  // 1 / tau
    R li2;    // 2 sigma: Li's extra stress X = li2 F F / psi^2 (Eq. 31 in moment space)
    D sd[9];  // rates in moment order (all 1/tau for BGK) over the squared norms of M's rows
              // (M^-1 = M^T D^-1)
    D hd[9];  // (1 - s/2) over the same norms
    R lim[9]; // 1 / (1/s_k - 1/2) for the moments that carry Li's stress

    __device__ __forceinline__ float psi_of_rho(D rho) const {
        if (psi_kind == 0) return (float)eos_psi<D>(rho, bq, e1, e2, e3);
        // Eq. 33 in the shape precision R (FP32 in the mixed path): psi is stored in FP32.
        return (float)ss_psi<R>((R)rho, (R)inv_eps);
    }
    // psi of a node from its populations.  psi is a relative quantity stored in FP32, so the
    // density it is evaluated at is summed in R (FP32 in the mixed path); the collision forms
    // its own density in D.
    __device__ __forceinline__ float psi_of(const float f[9]) const {
        return psi_of_rho((D)density9<R>(f));
    }
};

// psi of the node and of its eight neighbours.
template <typename R>
struct Nb {
    R c, E, W, N, S, NE, NW, SW, SE;
};

// Equilibrium of Eq. 2 (c_s^2 = 1/3) written as f^eq_q = w_q rho (1 + s_q),
// s_q = 3 e.u + 9/2 (e.u)^2 - 3/2 u.u; returns s_q.
template <typename R>
__device__ __forceinline__ void eq_shape(R ux, R uy, R s[9]) {
    const R usq = R(1.5) * (ux * ux + uy * uy);
    s[0] = -usq;
    const R e[8] = {ux, uy, -ux, -uy, ux + uy, uy - ux, -ux - uy, ux - uy};
#pragma unroll
    for (int q = 0; q < 8; ++q) s[1 + q] = R(3) * e[q] + R(4.5) * e[q] * e[q] - usq;
}

template <typename T>
__device__ __forceinline__ T wgt(int q) {
    return q == 0 ? T(4) / T(9) : (q < 5 ? T(1) / T(9) : T(1) / T(36));
}

// f^eq_q(rho, u) - f_q in D: the non-equilibrium part can be as large as f itself (in the
// light phase next to an interface u and v differ by F/(2 rho)), so it is formed in D; only the
// shape term s_q (relative accuracy suffices) comes from R.
template <typename R, typename D>
__device__ __forceinline__ void eq_minus_f(D rho_d, R ux, R uy, const float f[9], D out[9]) {
    R s[9];
    eq_shape<R>(ux, uy, s);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const D wr = wgt<D>(q) * rho_d;
        out[q] = (wr - (D)f[q]) + wr * (D)s[q];
    }
}

// 1 / psi^2 for Li's term (Eq. 31): a small correction, so FP32 takes the hardware
// reciprocal (1 ulp) instead of a correctly rounded division.
template <typename R>
__device__ __forceinline__ R inv_sq(float pc) {
    if constexpr (sizeof(R) == 4)
        return __builtin_amdgcn_rcpf(pc * pc);
    else
        return R(1) / (R(pc) * R(pc));
}

// One node of the time step once psi is known around it: interaction force (Eq. 6), moments
// and velocities (Sec. 3.2), forcing scheme and collision.  f holds the post-streaming
// populations of the node; fs receives the post-collision ones (FP32, ready to store).
template <typename R, typename D, int SCHEME, int COLL>
__device__ __forceinline__ void collide(const float f[9], const Nb<float> &p,
                                        const StepConst<R, D> &c, float fs[9]) {
    // Eq. 6 with w(1) = 1/3, w(2) = 1/12: link sums as differences of opposite pairs.  In D:
    // in the light phase u and F/(2 rho) nearly cancel in v, so F and u must be accurate.
    const D third = D(1) / D(3), twelfth = D(1) / D(12);
    const D pE = p.E, pW = p.W, pN = p.N, pS = p.S, pNE = p.NE, pNW = p.NW, pSW = p.SW,
            pSE = p.SE;
    const D dA = pNE - pSW, dB = pSE - pNW;
    const D s1x = third * (pE - pW) + twelfth * (dA + dB);
    const D s1y = third * (pN - pS) + twelfth * (dA - dB);
    D Fxd = c.gB * (D)p.c * s1x;
    D Fyd = c.gB * (D)p.c * s1y;
    if (c.gA != D(0)) {
        // sum w psi^2 e with psi_a^2 - psi_b^2 = (psi_a - psi_b)(psi_a + psi_b)
        const D qA = dA * (pNE + pSW), qB = dB * (pSE + pNW);
        const D s2x = third * ((pE - pW) * (pE + pW)) + twelfth * (qA + qB);
        const D s2y = third * ((pN - pS) * (pN + pS)) + twelfth * (qA - qB);
        Fxd += c.gA * s2x;
        Fyd += c.gA * s2y;
    }

    // Eq. 3 in D from the sums of opposite pairs, in density()'s order (sums of FP32 values
    // in FP64 are exact, so any grouping gives the same density); u = sum f e / rho,
    // v = u + F / (2 rho).  Momentum from opposite-pair differences.
    const D f0 = f[0];
    const D p13 = (D)f[1] + (D)f[3], p24 = (D)f[2] + (D)f[4];
    const D p57 = (D)f[5] + (D)f[7], p68 = (D)f[6] + (D)f[8];
    const D rho_d = ((f0 + p13) + p24) + (p57 + p68);
    const D jx = (((D)f[1] - (D)f[3]) + ((D)f[5] - (D)f[7])) + ((D)f[8] - (D)f[6]);
    const D jy = (((D)f[2] - (D)f[4]) + ((D)f[5] - (D)f[7])) + ((D)f[6] - (D)f[8]);
    const D inv = recip<D>(rho_d), hinv = D(0.5) * inv;
    const D uxd = jx * inv, uyd = jy * inv;
    const D vxd = uxd + Fxd * hinv, vyd = uyd + Fyd * hinv;
    const R ux = (R)uxd, uy = (R)uyd;
    const R vx = (R)vxd, vy = (R)vyd;
    const R Fx = (R)Fxd, Fy = (R)Fyd;
    const R pc = p.c;

    D upd[9];  // f*_q - f_q
    if constexpr (SCHEME == EDM || SCHEME == SC) {  // BGK only (lbm_create rejects MRT)
        D neq[9];
        if constexpr (SCHEME == EDM) {
            // Eq. 22 with f^eq(rho, u + D) - f^eq(rho, u) written out exactly:
            // w rho [3 e.D + 9/2 (e.D)(e.(2u + D)) - 3/2 D.(2u + D)],  D = F / rho.
            eq_minus_f<R, D>(rho_d, ux, uy, f, neq);
            const R Dx = (R)(Fxd * inv), Dy = (R)(Fyd * inv);
            const R Sx = R(2) * ux + Dx, Sy = R(2) * uy + Dy;
            const R DS = R(1.5) * (Dx * Sx + Dy * Sy);
            const R eD[9] = {R(0), Dx, Dy, -Dx, -Dy, Dx + Dy, Dy - Dx, -Dx - Dy, Dx - Dy};
            const R eS[9] = {R(0), Sx, Sy, -Sx, -Sy, Sx + Sy, Sy - Sx, -Sx - Sy, Sx - Sy};
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const R shape = R(3) * eD[q] + R(4.5) * eD[q] * eS[q] - DS;
                upd[q] = c.omega * neq[q] + wgt<D>(q) * rho_d * (D)shape;
            }
        } else if constexpr (SCHEME == SC) {
            // Eq. 20-21: BGK towards f^eq(rho, u + tau F / rho), no source term.
            const R ex = (R)(uxd + c.tau * Fxd * inv), ey = (R)(uyd + c.tau * Fyd * inv);
            eq_minus_f<R, D>(rho_d, ex, ey, f, neq);
#pragma unroll
            for (int q = 0; q < 9; ++q) upd[q] = c.omega * neq[q];
        }
    } else {
        // Guo's forcing (Eq. 23; Eq. 31 with Li's term) with the BGK collision (Eq. 1) or the
        // MRT collision (Eq. 34), both in moment space: BGK is the MRT collision with every rate
        // 1/tau (the rates lbm_create sets for BGK), which reproduces Eq. 1 with Eq. 23 or Eq. 31
        // exactly and costs fewer instructions than the nine populations' equilibria.
        // MRT, Eq. 34: m* = m - Lambda (m - m_eq) + (I - Lambda/2) S with m_eq = M f^eq(rho, v).
        // Evaluated as f* = f + M^-1 [Lambda (m_eq - m) + (I - Lambda/2) S] so that only
        // non-equilibrium quantities go through the inverse transform.  m_eq has the closed form
        // rho (1, -2 + 3 v.v, 1 - 3 v.v, v_x, -v_x, v_y, -v_y, v_x^2 - v_y^2, v_x v_y) of the
        // moments of Eq. 2; each difference is written on the populations' deviation from the
        // rest state, and rho v = j + F/2 fixes the momentum rows exactly.
        const D ax = p13 + p24, dg = p57 + p68;
        const D d13 = (D)f[1] - (D)f[3], d24 = (D)f[2] - (D)f[4];
        const D rv2 = rho_d * (vxd * vxd + vyd * vyd);
        const D hFx = D(0.5) * Fxd, hFy = D(0.5) * Fyd;
        D n[9];  // m_eq - m
        n[0] = D(0);                                           // mass is conserved
        n[1] = (D(3) * rv2 + D(2) * f0) - (ax + D(4) * dg);    // e
        n[2] = D(3) * ((ax - f0) - rv2);                       // epsilon
        n[3] = hFx;                                            // j_x
        n[4] = (D(3) * d13 - D(2) * jx) - hFx;                 // q_x
        n[5] = hFy;                                            // j_y
        n[6] = (D(3) * d24 - D(2) * jy) - hFy;                 // q_y
        n[7] = rho_d * ((vxd - vyd) * (vxd + vyd)) - (p13 - p24);
        n[8] = rho_d * (vxd * vyd) - (p57 - p68);
        // Guo's source in moment space, S = M B(v).
        const R vF = vx * Fx + vy * Fy;
        R S[9] = {R(0), R(6) * vF, -R(6) * vF, Fx, -Fx, Fy, -Fy,
                  R(2) * (vx * Fx - vy * Fy), vx * Fy + vy * Fx};
        if constexpr (SCHEME == GUO_LI) {
            const R cl = c.li2 * inv_sq<R>(pc);
            const R Xxx = cl * Fx * Fx, Xyy = cl * Fy * Fy, Xxy = cl * Fx * Fy;
            const R tr3 = R(3) * (Xxx + Xyy);
            S[1] += tr3 * c.lim[1];
            S[2] -= tr3 * c.lim[2];
            S[7] += (Xxx - Xyy) * c.lim[7];
            S[8] += Xxy * c.lim[8];
        }
        // a = D^-1 [Lambda (m_eq - m) + (I - Lambda/2) S]; row 0 vanishes (n_0 = S_0 = 0).  The
        // momentum rows are exactly F / 6 whatever s_j is (j* = j + F), and the other F-sized
        // sources are taken in D, where F already is.
        D a[9];
        a[1] = c.sd[1] * n[1] + c.hd[1] * (D)S[1];
        a[2] = c.sd[2] * n[2] + c.hd[2] * (D)S[2];
        a[3] = Fxd * (D(1) / D(6));
        a[4] = c.sd[4] * n[4] - c.hd[4] * Fxd;
        a[5] = Fyd * (D(1) / D(6));
        a[6] = c.sd[6] * n[6] - c.hd[6] * Fyd;
        a[7] = c.sd[7] * n[7] + c.hd[7] * (D)S[7];
        a[8] = c.sd[8] * n[8] + c.hd[8] * (D)S[8];
        // M^-1 = M^T D^-1, the pairs of opposite velocities formed once
        const D c0 = -a[1] - D(2) * a[2];
        const D c5 = D(2) * a[1] + a[2];
        const D gx = a[3] - D(2) * a[4], gy = a[5] - D(2) * a[6];
        const D hx = a[3] + a[4], hy = a[5] + a[6];
        const D ap = c0 + a[7], am = c0 - a[7];
        const D bp = c5 + a[8], bm = c5 - a[8];
        const D hsum = hx + hy, hdif = hx - hy;
        upd[1] = ap + gx;
        upd[3] = ap - gx;
        upd[2] = am + gy;
        upd[4] = am - gy;
        upd[5] = bp + hsum;
        upd[7] = bp - hsum;
        upd[8] = bm + hdif;
        upd[6] = bm - hdif;
    }
#pragma unroll
    for (int q = 1; q < 9; ++q) fs[q] = (float)((D)f[q] + upd[q]);
    // Every scheme conserves mass exactly (sum_q f*_q = rho); closing the rest population on
    // it keeps the binary rounding of the weights 4/9, 1/9, 1/36 from drifting the mass.
    // (density()'s order without its first term)
    const D moving = (((D)fs[1] + (D)fs[3]) + ((D)fs[2] + (D)fs[4])) +
                     (((D)fs[5] + (D)fs[7]) + ((D)fs[6] + (D)fs[8]));
    fs[0] = (float)(rho_d - moving);
}

__device__ __forceinline__ void put(float *p, float v, bool nt) {
    if (nt)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Push streaming, Eq. 36: f_q(x + e_q, t + 1) = f*_q(x, t), periodic.
template <typename R, typename D>
__device__ __forceinline__ void stream_out(float *__restrict__ fout, const StepConst<R, D> &c,
                                           int x, int y, const float fs[9], bool nt) {
    const int xe = x + 1 == c.nx ? 0 : x + 1, xw = x == 0 ? c.nx - 1 : x - 1;
    const int yn = y + 1 == c.ny ? 0 : y + 1, ys = y == 0 ? c.ny - 1 : y - 1;
    const size_t q = c.fq;
    const size_t rc = (size_t)y * c.frow, rn = (size_t)yn * c.frow, rs = (size_t)ys * c.frow;
    put(fout + rc + x, fs[0], nt);
    put(fout + q + rc + xe, fs[1], nt);
    put(fout + 2 * q + rn + x, fs[2], nt);
    put(fout + 3 * q + rc + xw, fs[3], nt);
    put(fout + 4 * q + rs + x, fs[4], nt);
    put(fout + 5 * q + rn + xe, fs[5], nt);
    put(fout + 6 * q + rn + xw, fs[6], nt);
    put(fout + 7 * q + rs + xw, fs[7], nt);
    put(fout + 8 * q + rs + xe, fs[8], nt);
}

__device__ __forceinline__ void load9(const float *__restrict__ f, size_t i, size_t fq, float v[9]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = f[i + q * fq];
}

// Buffer-resource access for the one-pass sweep: the population buffer is one 128-bit
// resource in scalar registers; a node's address is a 32-bit per-lane byte offset (its column)
// plus a wave-uniform scalar offset (row and velocity plane), so the nine loads and nine
// stores of a node share three per-lane offsets (x, x + 1, x - 1) instead of eighteen 64-bit
// pointers.  The resource also bounds every access by the buffer size.
constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit access on CDNA

__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const float *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, (int)bytes,
                                             kBufferWord3);
}

// Lattices whose population buffer exceeds 4 GiB (32-bit offsets) get one resource per row,
// based at the row's first float by 64-bit scalar arithmetic and bounded by the end of the
// buffer: the velocity plane stays in the scalar offset and the column in the per-lane offset
// (row-interleaved layout only, where a whole row spans 9 x pitch floats).  About 3 % slower
// than the whole-buffer resource (more scalar registers), so it is kept for those lattices.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float *p, size_t frow,
                                                           size_t total, int row) {
    const size_t off = (size_t)row * frow;
    const size_t rem = (total - off) * sizeof(float);
    const unsigned bytes = rem > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned)rem;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p + off), (short)0, (int)bytes,
                                             kBufferWord3);
}

__device__ __forceinline__ void bload9(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                       unsigned qstride, float v[9]) {
#pragma unroll
    for (int q = 0; q < 9; ++q)
        v[q] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff + q * qstride, 0));
}

__device__ __forceinline__ void bput(__amdgpu_buffer_rsrc_t r, float v, unsigned voff,
                                     unsigned soff, bool nt) {
    if (nt)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 2);  // nt
    else
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}

// Push streaming (Eq. 36) through the per-row resources of rows y, y + 1 and y - 1.
template <typename R, typename D>
__device__ __forceinline__ void bstream_out_rows(float *fout, const StepConst<R, D> &c, int x,
                                                 int y, const float fs[9], bool nt) {
    const unsigned vx = 4u * x, ve = 4u * (x + 1 == c.nx ? 0 : x + 1),
                   vw = 4u * (x == 0 ? c.nx - 1 : x - 1);
    const int yn = y + 1 == c.ny ? 0 : y + 1, ys = y == 0 ? c.ny - 1 : y - 1;
    const unsigned q = 4u * (unsigned)c.fq;
    const __amdgpu_buffer_rsrc_t rc = row_rsrc(fout, c.frow, c.ffloats, y),
                                 rn = row_rsrc(fout, c.frow, c.ffloats, yn),
                                 rs = row_rsrc(fout, c.frow, c.ffloats, ys);
    auto all = [&](auto put1) {
        put1(rc, fs[0], vx, 0);
        put1(rc, fs[1], ve, q);
        put1(rn, fs[2], vx, 2 * q);
        put1(rc, fs[3], vw, 3 * q);
        put1(rs, fs[4], vx, 4 * q);
        put1(rn, fs[5], ve, 5 * q);
        put1(rn, fs[6], vw, 6 * q);
        put1(rs, fs[7], vw, 7 * q);
        put1(rs, fs[8], ve, 8 * q);
    };
    if (nt)
        all([&](__amdgpu_buffer_rsrc_t r, float v, unsigned vo, unsigned so) { bput(r, v, vo, so, true); });
    else
        all([&](__amdgpu_buffer_rsrc_t r, float v, unsigned vo, unsigned so) { bput(r, v, vo, so, false); });
}

// Push streaming (Eq. 36) through the buffer resource.
template <typename R, typename D>
__device__ __forceinline__ void bstream_out(__amdgpu_buffer_rsrc_t r, const StepConst<R, D> &c,
                                            int x, int y, const float fs[9], bool nt) {
    const unsigned vx = 4u * x, ve = 4u * (x + 1 == c.nx ? 0 : x + 1),
                   vw = 4u * (x == 0 ? c.nx - 1 : x - 1);
    const int yn = y + 1 == c.ny ? 0 : y + 1, ys = y == 0 ? c.ny - 1 : y - 1;
    const unsigned q = 4u * (unsigned)c.fq, fr = 4u * (unsigned)c.frow;
    const unsigned rc = fr * y, rn = fr * yn, rs = fr * ys;
    auto all = [&](auto put1) {
        put1(fs[0], vx, rc);
        put1(fs[1], ve, q + rc);
        put1(fs[2], vx, 2 * q + rn);
        put1(fs[3], vw, 3 * q + rc);
        put1(fs[4], vx, 4 * q + rs);
        put1(fs[5], ve, 5 * q + rn);
        put1(fs[6], vw, 6 * q + rn);
        put1(fs[7], vw, 7 * q + rs);
        put1(fs[8], ve, 8 * q + rs);
    };
    if (nt)
        all([&](float v, unsigned vo, unsigned so) { bput(r, v, vo, so, true); });
    else
        all([&](float v, unsigned vo, unsigned so) { bput(r, v, vo, so, false); });
}

// Block index remapped so that consecutive tiles land on the same XCD (workgroups are dealt
// round-robin to the eight XCDs, each with its own L2): neighbouring tiles then share the
// psi halo rows and the partially written cache lines of the shifted planes in one L2.
__device__ __forceinline__ int tile_id(int b, int nb, bool xcd) {
    if (!xcd) return b;
    const int full = nb & ~7;
    if (b >= full) return b;
    const int per = full >> 3;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------------------
// Two-pass step, pass 1: density and psi (Eq. 3, Eq. 29-30, Eq. 7), four nodes per thread
// with 16-byte loads along x (rows are padded to 64 floats).
// ---------------------------------------------------------------------------------------
template <typename R, typename D>
__global__ void __launch_bounds__(256) psi_kernel(const float *__restrict__ f,
                                                  float *__restrict__ psi, StepConst<R, D> c) {
    const int x4 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
    if (x4 >= c.nx) return;
    for (int y = blockIdx.y; y < c.ny; y += gridDim.y) {
        const size_t i = (size_t)y * c.frow + x4;
        float4 v[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = *reinterpret_cast<const float4 *>(f + i + q * c.fq);
        float4 out;
        {
            const float a[9] = {v[0].x, v[1].x, v[2].x, v[3].x, v[4].x, v[5].x, v[6].x, v[7].x, v[8].x};
            out.x = c.psi_of(a);
        }
        {
            const float a[9] = {v[0].y, v[1].y, v[2].y, v[3].y, v[4].y, v[5].y, v[6].y, v[7].y, v[8].y};
            out.y = c.psi_of(a);
        }
        {
            const float a[9] = {v[0].z, v[1].z, v[2].z, v[3].z, v[4].z, v[5].z, v[6].z, v[7].z, v[8].z};
            out.z = c.psi_of(a);
        }
        {
            const float a[9] = {v[0].w, v[1].w, v[2].w, v[3].w, v[4].w, v[5].w, v[6].w, v[7].w, v[8].w};
            out.w = c.psi_of(a);
        }
        *reinterpret_cast<float4 *>(psi + (size_t)y * c.pitch + x4) = out;
    }
}

// ---------------------------------------------------------------------------------------
// Two-pass step, pass 2: fused force + collision + streaming on a TX x TY tile, psi of the
// tile and a one-node halo staged in LDS.
// ---------------------------------------------------------------------------------------
template <typename R, typename D, int SCHEME, int COLL>
__global__ void __launch_bounds__(1024) fused_kernel(const float *__restrict__ fin,
                                                     const float *__restrict__ psi,
                                                     float *__restrict__ fout,
                                                     StepConst<R, D> c) {
    extern __shared__ float tile[];
    const int TX = blockDim.x, TY = blockDim.y;
    const int W = TX + 2;
    const int nx = c.nx, ny = c.ny;
    const int b = tile_id(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y,
                          c.flags & kFlagXCD);
    const int x0 = (b % gridDim.x) * TX, y0 = (b / gridDim.x) * TY;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < nx && y < ny;

    // Populations first, so their latency overlaps the psi staging below.
    float f[9];
    if (active) load9(fin, (size_t)y * c.frow + x, c.fq, f);

    // Stage psi of the tile and its one-node halo (periodic) in LDS.
    const bool inner = x0 >= 1 && x0 + TX < nx && y0 >= 1 && y0 + TY < ny;
    for (int ly = ty; ly < TY + 2; ly += TY) {
        int gy = y0 + ly - 1;
        if (!inner) gy = wrap_any(gy, ny);
        const float *row = psi + (size_t)gy * c.pitch;
        for (int lx = tx; lx < W; lx += TX) {
            int gx = x0 + lx - 1;
            if (!inner) gx = wrap_any(gx, nx);
            tile[ly * W + lx] = row[gx];
        }
    }
    __syncthreads();
    if (!active) return;

    const int lc = (ty + 1) * W + tx + 1;
    const Nb<float> nb = {tile[lc],         tile[lc + 1],     tile[lc - 1],
                      tile[lc + W],     tile[lc - W],     tile[lc + W + 1],
                      tile[lc + W - 1], tile[lc - W - 1], tile[lc - W + 1]};
    float fs[9];
    collide<R, D, SCHEME, COLL>(f, nb, c, fs);
    stream_out<R, D>(fout, c, x, y, fs, c.flags & kFlagNT);
}

// ---------------------------------------------------------------------------------------
// One-pass step: a workgroup of TX threads owns a strip of TX columns and sweeps a segment of
// H rows (upwards or downwards).  psi is computed from the populations as each row is loaded and kept in a
// four-row LDS ring (plus the two halo columns, computed by lanes 0 and 1), so every
// population is read from memory once per step; only the halo columns and the row below and
// above the segment are read twice (neighbouring segments sweep in opposite directions, so
// that second read comes from L2).  Rows are software-pipelined two deep: while row y is
// collided, row y+1 (loaded one iteration earlier) becomes psi and the loads of row y+2 are
// in flight.  Same per-node arithmetic as the two-pass step, bit for bit.
// ---------------------------------------------------------------------------------------
// One tile of the sweep: columns [x0, x0 + blockDim.x) (clipped at nx) and rows [y0, y0 + H)
// (clipped at ny) of the lattice described by c; ring is the workgroup's LDS (4 x (TX + 2)).
template <typename R, typename D, int SCHEME, int COLL, int PF, bool BIG = false>
__device__ __forceinline__ void sweep_tile(const float *__restrict__ fin, float *__restrict__ fout,
                                           const StepConst<R, D> &c, int x0, int y0, int H,
                                           float *ring) {
    const int TX = blockDim.x, W = TX + 2;
    const int nx = c.nx, ny = c.ny;
    const int tx = threadIdx.x;
    const int na = nx - x0 < TX ? nx - x0 : TX;  // active columns of this strip
    const bool active = tx < na;
    const bool halo = tx < 2;                    // lanes 0 and 1 also own the halo columns
    const int x = x0 + tx;
    const int y1 = y0 + H < ny ? y0 + H : ny;
    const int hcol = tx == 0 ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + na == nx ? 0 : x0 + na);
    const int hslot = tx == 0 ? 0 : na + 1;
    const bool nt = c.flags & kFlagNT;
    const __amdgpu_buffer_rsrc_t rbuf = pop_rsrc(fin, c.fbytes), rout = pop_rsrc(fout, c.fbytes);
    const unsigned qs = 4u * (unsigned)c.fq, fr = 4u * (unsigned)c.frow;
    // Loads of row r: resource and scalar offset (whole buffer, or the row's own resource).
    auto rin = [&](int r) { return BIG ? row_rsrc(fin, c.frow, c.ffloats, r) : rbuf; };
    auto roff = [&](int r) { return BIG ? 0u : fr * (unsigned)r; };
    const unsigned vx = 4u * x, vh = 4u * hcol;
    auto wrapy = [&](int yy) { return yy >= ny ? yy - ny : (yy < 0 ? yy + ny : yy); };
    auto slot = [&](int yy_rel) { return ring + ((yy_rel + 1) & 3) * W; };

    // PF = 2: rows y (fa), y+1 (fb) and y+2 (fc, loads in flight) in registers; halo lanes
    // issue the loads of halo row y+2 at the top of iteration y and turn them into psi at its
    // bottom, straight into the ring slot of row y+2 (that slot held row y-2, which no thread
    // reads in iteration y; iteration y+1 reads it after its barrier).
    // PF = 1: row y+1 is loaded and turned into psi at the top of iteration y.
    // Segments alternate direction (even ones sweep up, odd ones down), so the two segments
    // that share a boundary read the boundary rows at the same time -- both at their start or
    // both at their end -- and the second read of those rows hits in L2.  Row k of the sweep
    // is ys + dir k; the ring keeps rows k-1 ("behind"), k and k+1 ("ahead").
    const int nrow = y1 - y0;
    const int dir = ((y0 / H) & 1) ? -1 : 1;
    const int ys = dir > 0 ? y0 : y1 - 1;
    auto row = [&](int k) { return wrapy(ys + dir * k); };
    float fa[9], fb[9], fc[9], hc[9];
    {
        const int rm = row(-1), r0 = row(0), rp = row(1);
        if (active) bload9(rin(rm), vx, roff(rm), qs, fc);
        if (active) bload9(rin(r0), vx, roff(r0), qs, fa);
        if (active) slot(-1)[tx + 1] = c.psi_of(fc);
        if (active) slot(0)[tx + 1] = c.psi_of(fa);
        if (PF == 2 && active) bload9(rin(rp), vx, roff(rp), qs, fb);
        if (halo) {
            bload9(rin(rm), vh, roff(rm), qs, hc);
            slot(-1)[hslot] = c.psi_of(hc);
            bload9(rin(r0), vh, roff(r0), qs, hc);
            slot(0)[hslot] = c.psi_of(hc);
            if (PF == 2) {
                bload9(rin(rp), vh, roff(rp), qs, hc);
                slot(1)[hslot] = c.psi_of(hc);
            }
        }
    }
    for (int k = 0; k < nrow; ++k) {
        float *ahead = slot(k + 1);
        bool more = false;
        if constexpr (PF == 2) {
            // Row k+2 is needed only while row k+1 is still inside the segment.
            more = k + 2 <= nrow;
            if (more) {
                const int r2 = row(k + 2);
                const __amdgpu_buffer_rsrc_t rr = rin(r2);
                if (active) bload9(rr, vx, roff(r2), qs, fc);
                if (halo) bload9(rr, vh, roff(r2), qs, hc);
            }
        } else {
            const int r1 = row(k + 1);
            const __amdgpu_buffer_rsrc_t rr = rin(r1);
            if (active) bload9(rr, vx, roff(r1), qs, fb);
            if (halo) {
                bload9(rr, vh, roff(r1), qs, hc);
                ahead[hslot] = c.psi_of(hc);
            }
        }
        if (active) ahead[tx + 1] = c.psi_of(fb);
        __syncthreads();
        if (active) {
            const float *behind = slot(k - 1), *rc = slot(k);
            const float *rn = dir > 0 ? ahead : behind, *rs = dir > 0 ? behind : ahead;
            const int l = tx + 1;
            const Nb<float> nb = {rc[l], rc[l + 1], rc[l - 1], rn[l], rs[l],
                                  rn[l + 1], rn[l - 1], rs[l - 1], rs[l + 1]};
            float fs[9];
            collide<R, D, SCHEME, COLL>(fa, nb, c, fs);
            if constexpr (BIG)
                bstream_out_rows<R, D>(fout, c, x, row(k), fs, nt);
            else
                bstream_out<R, D>(rout, c, x, row(k), fs, nt);
        }
        if (PF == 2 && halo && more) slot(k + 2)[hslot] = c.psi_of(hc);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            fa[q] = fb[q];
            if (PF == 2) fb[q] = fc[q];
        }
    }
}

template <typename R, typename D, int SCHEME, int COLL, int PF, bool BIG>
__device__ __forceinline__ void sweep_entry(const float *__restrict__ fin, float *__restrict__ fout,
                                            const StepConst<R, D> &c, int H) {
    extern __shared__ float ring[];  // 4 rows x (TX + 2)
    const int b = tile_id(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y,
                          c.flags & kFlagXCD);
    sweep_tile<R, D, SCHEME, COLL, PF, BIG>(fin, fout, c, (b % gridDim.x) * blockDim.x,
                                            (b / gridDim.x) * H, H, ring);
}

template <typename R, typename D, int SCHEME, int COLL, int PF, bool BIG = false>
__global__ void __launch_bounds__(512) sweep_kernel(const float *__restrict__ fin,
                                                    float *__restrict__ fout,
                                                    StepConst<R, D> c, int H) {
    sweep_entry<R, D, SCHEME, COLL, PF, BIG>(fin, fout, c, H);
}

// The same kernel asking the register allocator for five waves per SIMD: the mixed-precision
// and FP32 variants fit without spilling (the FP64 ones would spill, so they use the plain one).
template <typename R, typename D, int SCHEME, int COLL, int PF, bool BIG = false>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(5, 8)))
sweep_kernel_w5(const float *__restrict__ fin, float *__restrict__ fout, StepConst<R, D> c, int H) {
    sweep_entry<R, D, SCHEME, COLL, PF, BIG>(fin, fout, c, H);
}

// ---------------------------------------------------------------------------------------
// Two steps per pass (temporal blocking).  Each wave owns a strip of 64 columns and sweeps a
// segment of rows, computing step t on every lane and step t + 1 two rows behind.  x-neighbours
// -- psi of either step, and the populations of step t that stream along x -- move between
// lanes by whole-wave DPP shifts; y-neighbours stay in registers; so a wave needs no LDS and no
// barrier, and only step t + 1 goes back to memory: half the HBM traffic per step.  Each step
// loses one lane of validity on either side (step t is right on lanes 1..62, the streamed
// populations of step t + 1 on 2..61, step t + 1 on 3..60), so a strip outputs its inner 58
// columns and neighbouring strips overlap by 6.  Same per-node arithmetic as the one-step
// sweep, so the same bits.
// ---------------------------------------------------------------------------------------
// Whole-wave shifts by one lane.  The end lane with no source reads 0 through the bound
// control bit, so no old value has to be written into the destination first (one move less
// per shift); that lane lies outside the valid range either way.
__device__ __forceinline__ float lane_below(float v) {  // lane i receives lane i - 1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_above(float v) {  // lane i receives lane i + 1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

constexpr int kSweep2Out = 58;  // output columns of a 64-lane strip (lanes 3..60)

// One wave's tile: the strip whose first output column is xw (on lane 3), rows [y0, y0 + H)
// (clipped at ny); xw, y0 and H are wave-uniform.  DIR = +1 sweeps the rows upwards in y,
// DIR = -1 downwards (the same per-node arithmetic on the same neighbours, so the same bits):
// the tiles of a strip alternate, so that two neighbouring segments read the six rows they
// share at the same end of their sweeps, at about the same time, and one of the two reads is
// served by L2.
template <typename R, typename D, int SCHEME, int COLL, bool BIG, int DIR>
__device__ __forceinline__ void sweep2_tile(const float *__restrict__ fin,
                                            float *__restrict__ fout, const StepConst<R, D> &c,
                                            int xw, int y0, int H) {
    static_assert(DIR == 1 || DIR == -1, "sweep direction");
    const int lane = threadIdx.x & 63;
    const int nx = c.nx, ny = c.ny;
    const int y1 = y0 + H < ny ? y0 + H : ny;
    auto wrapx = [&](int xx) { xx %= nx; return xx < 0 ? xx + nx : xx; };
    // row r of the sweep (r = 0 is the first row of the segment in the sweep's order; wrapped)
    const int base = DIR > 0 ? y0 : y1 - 1;
    auto row = [&](int r) { int yy = (base + DIR * r) % ny; return yy < 0 ? yy + ny : yy; };
    const int x = wrapx(xw - 3 + lane);
    const bool out = lane >= 3 && lane < 3 + kSweep2Out && xw + lane - 3 < nx;
    const bool nt = c.flags & kFlagNT;
    const __amdgpu_buffer_rsrc_t rbuf = pop_rsrc(fin, c.fbytes), rout = pop_rsrc(fout, c.fbytes);
    const unsigned qs = 4u * (unsigned)c.fq, fr = 4u * (unsigned)c.frow;
    const unsigned vx = 4u * x;
    // loads of sweep row r: the whole-buffer resource, or beyond 4 GiB the row's own
    auto load_row = [&](int r, float v[9]) {
        const int rr = row(r);
        if constexpr (BIG)
            bload9(row_rsrc(fin, c.frow, c.ffloats, rr), vx, 0u, qs, v);
        else
            bload9(rbuf, vx, fr * rr, qs, v);
    };
    // psi of a node's eight neighbours from the rows behind (pb), at (pc) and ahead of (pa) it
    // in the sweep's order; lane i + 1 is the neighbour in +x
    auto stencil = [&](float pc, float pa, float pb) {
        const float pn = DIR > 0 ? pa : pb, ps = DIR > 0 ? pb : pa;
        return Nb<float>{pc, lane_above(pc), lane_below(pc), pn, ps,
                         lane_above(pn), lane_below(pn), lane_below(ps), lane_above(ps)};
    };

    // step t: populations of sweep rows s (fa), s+1 (fb), s+2 (fc, loads in flight); psi of
    // rows s-1, s, s+1 (pm, pc, pn)
    const int s0 = -2;
    float fa[9], fb[9], fc[9];
    load_row(s0 - 1, fc);
    float pm = c.psi_of(fc);
    load_row(s0, fa);
    float pc = c.psi_of(fa);
    load_row(s0 + 1, fb);
    // step t+1: the populations of row s-1 streamed so far -- planes 0, 1, 3 from row s-1; the
    // three planes that move along the sweep (2, 5, 6 upwards, 4, 7, 8 downwards) from row s-2
    // (b*) and, for row s, from row s-1 (c*) --, row s-2 complete (g), and psi of rows s-3 and
    // s-2
    float a0 = 0.f, a1 = 0.f, a3 = 0.f, b2 = 0.f, b5 = 0.f, b6 = 0.f, c2 = 0.f, c5 = 0.f,
          c6 = 0.f;
    float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float qm = 0.f, qc = 0.f;
    const int nrow = y1 - y0 + 4;
    for (int k = 0; k < nrow; ++k) {
        const int s = s0 + k;
        if (k + 1 < nrow) load_row(s + 2, fc);
        const float pn = c.psi_of(fb);
        // step t, row s (right on lanes 1..62)
        float fs[9];
        collide<R, D, SCHEME, COLL>(fa, stencil(pc, pn, pm), c, fs);
        // stream along x between lanes; along y into the rows held in registers
        const float e1 = lane_below(fs[1]), e5 = lane_below(fs[5]), e8 = lane_below(fs[8]);
        const float w3 = lane_above(fs[3]), w6 = lane_above(fs[6]), w7 = lane_above(fs[7]);
        float f1[9];  // row s-1 of step t+1
        if constexpr (DIR > 0) {
            const float r[9] = {a0, a1, b2, a3, fs[4], b5, b6, w7, e8};
#pragma unroll
            for (int q = 0; q < 9; ++q) f1[q] = r[q];
        } else {
            const float r[9] = {a0, a1, fs[2], a3, b2, e5, w6, b5, b6};
#pragma unroll
            for (int q = 0; q < 9; ++q) f1[q] = r[q];
        }
        b2 = c2;
        b5 = c5;
        b6 = c6;
        c2 = DIR > 0 ? fs[2] : fs[4];
        c5 = DIR > 0 ? e5 : w7;
        c6 = DIR > 0 ? w6 : e8;
        a0 = fs[0];
        a1 = e1;
        a3 = w3;
        const float qn = c.psi_of(f1);
        // step t+1, row s-2 (right on lanes 3..60)
        if (k >= 4) {
            float fo[9];
            collide<R, D, SCHEME, COLL>(g, stencil(qc, qn, qm), c, fo);
            if (out) {
                if constexpr (BIG)
                    bstream_out_rows<R, D>(fout, c, x, row(s - 2), fo, nt);
                else
                    bstream_out<R, D>(rout, c, x, row(s - 2), fo, nt);
            }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] = f1[q];
        qm = qc;
        qc = qn;
        pm = pc;
        pc = pn;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            fa[q] = fb[q];
            fb[q] = fc[q];
        }
    }
}

// The tile in the direction of its segment's parity (even segments upwards).
template <typename R, typename D, int SCHEME, int COLL, bool BIG>
__device__ __forceinline__ void sweep2_tile_alt(const float *__restrict__ fin,
                                                float *__restrict__ fout,
                                                const StepConst<R, D> &c, int xw, int y0, int H,
                                                bool down) {
    if (down)
        sweep2_tile<R, D, SCHEME, COLL, BIG, -1>(fin, fout, c, xw, y0, H);
    else
        sweep2_tile<R, D, SCHEME, COLL, BIG, 1>(fin, fout, c, xw, y0, H);
}

template <typename R, typename D, int SCHEME, int COLL, bool BIG = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
sweep2_kernel(const float *__restrict__ fin, float *__restrict__ fout, StepConst<R, D> c, int H,
              int nstrips, int ntiles) {
    // the wave's tile: uniform across the wave (a scalar), so that row offsets stay scalar
    // operands of the buffer accesses; with LBM_LAUNCH_XCD_ORDER consecutive workgroups (rows
    // of strips, and the segments above and below them) share one XCD's L2
    const int b = tile_id(blockIdx.x, gridDim.x, c.flags & kFlagXCD);
    const int t = b * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= ntiles) return;  // whole waves
    const int seg = t / nstrips;
    sweep2_tile_alt<R, D, SCHEME, COLL, BIG>(fin, fout, c, (t % nstrips) * kSweep2Out, seg * H, H,
                                             seg & 1);
}

// ---------------------------------------------------------------------------------------
// Batched sweep: many independent lattices (own size, physics and relaxation) advanced by one
// launch per kind of lattice and step.  Each workgroup walks its kind's slice of the shared
// tile list (lattice, x0, y0, rows); the list and the slices live in device memory, so the
// host can drop converged lattices between replays of a captured graph.  Mixed precision.
// ---------------------------------------------------------------------------------------
struct BatchLattice {
    StepConst<float, double> c;
    float *f[2];
    float *vprev;            // velocity at the previous convergence check (2 floats per node)
    int scheme, coll;
    int xa, ya, xb, yb;      // probe nodes
};

// One kind of the batch (forcing scheme and collision): its tiles are the slice meta[kind] =
// (offset, count) of the shared tile list, both read from device memory so that the host can
// drop lattices between replays of a captured graph.  One specialised kernel per kind keeps the
// register allocation of the single-lattice sweep (five waves per SIMD with one row of loads in
// flight; the two-row variants of some kinds would spill at five, so they ask for four).
template <int SCHEME, int COLL, int PF>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(PF == 1 ? 5 : 4, 8)))
batch_kind_kernel(const BatchLattice *__restrict__ lats, const int4 *__restrict__ tiles,
                  const int2 *__restrict__ meta, int kind, int parity) {
    extern __shared__ float ring[];
    const int2 m = meta[kind];
    // Workgroups are dealt round-robin to the eight XCDs (the grid is a multiple of 8): XCD k
    // walks the k-th contiguous eighth of the slice, so neighbouring tiles -- which share halo
    // rows and columns -- meet in one L2.
    const int per = gridDim.x >> 3, xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int begin = (int)((long long)m.y * xcd / 8), end = (int)((long long)m.y * (xcd + 1) / 8);
    for (int t = begin + local; t < end; t += per) {
        const int4 tl = tiles[m.x + t];
        const BatchLattice &L = lats[tl.x];
        const StepConst<float, double> c = L.c;
        sweep_tile<float, double, SCHEME, COLL, PF>(L.f[parity], L.f[parity ^ 1], c, tl.y, tl.z,
                                                    tl.w, ring);
        __syncthreads();  // the ring is reused by the next tile
    }
}

// Two steps per launch for one kind of the batch: one wave per tile of the kind's slice
// meta2[kind] of the two-step tile list (lattice, first output column, first row, rows), each a
// 64-lane strip of 58 output columns (the single lattice's two-step sweep, tile by tile).  The
// grid holds at least one wave per tile (waves past the slice's count, read from device memory,
// return at once); workgroups are remapped so that each XCD takes a contiguous run of tiles,
// and tiles that overlap (neighbouring strips and segments of one lattice) are read through the
// same L2.
template <int SCHEME, int COLL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
batch2_kind_kernel(const BatchLattice *__restrict__ lats, const int4 *__restrict__ tiles,
                   const int2 *__restrict__ meta, int kind, int parity) {
    const int2 m = meta[kind];
    const int b = tile_id(blockIdx.x, gridDim.x, true);
    const int t = b * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= m.y) return;  // whole waves
    const int4 tl = tiles[m.x + t];
    const BatchLattice &L = lats[tl.x];
    const StepConst<float, double> c = L.c;
    sweep2_tile_alt<float, double, SCHEME, COLL, false>(L.f[parity], L.f[parity ^ 1], c, tl.y,
                                                        tl.z, tl.w, (tl.z / tl.w) & 1);
}

// FP64 observables of one node of a batch lattice; psi of the stencil recomputed from f.
__device__ __forceinline__ void batch_node(const BatchLattice &L, const float *__restrict__ f,
                                           int x, int y, double acc[6], size_t k, bool track) {
    const StepConst<float, double> &c = L.c;
    const int xe = x + 1 == c.nx ? 0 : x + 1, xw = x == 0 ? c.nx - 1 : x - 1;
    const int yn = y + 1 == c.ny ? 0 : y + 1, ys = y == 0 ? c.ny - 1 : y - 1;
    float v[9];
    auto P = [&](int xx, int yy) {
        float w[9];
        load9(f, (size_t)yy * c.frow + xx, c.fq, w);
        return (double)c.psi_of(w);
    };
    load9(f, (size_t)y * c.frow + x, c.fq, v);
    const double rho = density9<double>(v);
    const double jx = (((double)v[1] - v[3]) + ((double)v[5] - v[7])) + ((double)v[8] - v[6]);
    const double jy = (((double)v[2] - v[4]) + ((double)v[5] - v[7])) + ((double)v[6] - v[8]);
    const double pc = c.psi_of(v), pE = P(xe, y), pW = P(xw, y), pN = P(x, yn), pS = P(x, ys);
    const double pNE = P(xe, yn), pNW = P(xw, yn), pSW = P(xw, ys), pSE = P(xe, ys);
    const double dA = pNE - pSW, dB = pSE - pNW;
    const double s1x = (pE - pW) / 3.0 + (dA + dB) / 12.0;
    const double s1y = (pN - pS) / 3.0 + (dA - dB) / 12.0;
    const double qA = dA * (pNE + pSW), qB = dB * (pSE + pNW);
    const double s2x = (pE - pW) * (pE + pW) / 3.0 + (qA + qB) / 12.0;
    const double s2y = (pN - pS) * (pN + pS) / 3.0 + (qA - qB) / 12.0;
    const double Fx = c.gB * pc * s1x + c.gA * s2x, Fy = c.gB * pc * s1y + c.gA * s2y;
    const double vx = jx / rho + Fx / (2.0 * rho), vy = jy / rho + Fy / (2.0 * rho);
    if (!(isfinite(rho) && isfinite(vx) && isfinite(vy) && isfinite(pc))) {
        acc[5] += 1.0;
        return;
    }
    acc[0] += rho;
    acc[1] = fmin(acc[1], rho);
    acc[2] = fmax(acc[2], rho);
    acc[3] = fmax(acc[3], sqrt(vx * vx + vy * vy));
    if (track) {
        acc[4] = fmax(acc[4], fmax(fabs(vx - (double)L.vprev[2 * k]), fabs(vy - (double)L.vprev[2 * k + 1])));
        L.vprev[2 * k] = (float)vx;
        L.vprev[2 * k + 1] = (float)vy;
    }
}

// ---------------------------------------------------------------------------------------
// Initial state, read-out and observables (FP64 arithmetic on the FP32 state).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) init_kernel(Physics p, const double *__restrict__ rho0,
                                                   const double *__restrict__ u0,
                                                   float *__restrict__ f) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= p.nx) return;
    for (int y = blockIdx.y; y < p.ny; y += gridDim.y) {
        const size_t k = (size_t)y * p.nx + x;
        const double ux = u0 ? u0[2 * k] : 0.0, uy = u0 ? u0[2 * k + 1] : 0.0;
        double s[9];
        eq_shape<double>(ux, uy, s);
        const size_t i = (size_t)y * p.frow + x;
#pragma unroll
        for (int q = 0; q < 9; ++q) f[i + q * p.fq] = (float)(wgt<double>(q) * rho0[k] * (1.0 + s[q]));
    }
}

// Radial-profile initial state (warm start): rho(x, y) = exp(L(r - shift)), r the distance
// from the lattice centre (nx/2, ny/2), L the piecewise-linear interpolant of 64 values of
// log rho at r_k = r0 + k dr (k = 0..63), held at the first value below r0 and at the last
// beyond r0 + 63 dr; f = f^eq(rho, 0).
constexpr int kProfilePoints = 64;

struct Profile {
    double v[kProfilePoints];  // log rho at r_k
    double r0, inv_dr;         // first radius, 1 / spacing
    double shift;              // radial shift of the whole profile
};

__device__ __forceinline__ double profile_rho(const Profile &P, int nx, int ny, int x, int y) {
    const double dx = x - 0.5 * nx, dy = y - 0.5 * ny;
    const double t = (sqrt(dx * dx + dy * dy) - P.shift - P.r0) * P.inv_dr;
    double l;
    if (!(t > 0)) {
        l = P.v[0];
    } else if (t >= kProfilePoints - 1) {
        l = P.v[kProfilePoints - 1];
    } else {
        const int k = (int)t;
        const double w = t - k;
        l = P.v[k] + w * (P.v[k + 1] - P.v[k]);
    }
    return exp(l);
}

__global__ void __launch_bounds__(256) profile_init_kernel(Physics p, Profile P,
                                                           float *__restrict__ f) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= p.nx) return;
    for (int y = blockIdx.y; y < p.ny; y += gridDim.y) {
        const double rho = profile_rho(P, p.nx, p.ny, x, y);
        const size_t i = (size_t)y * p.frow + x;
#pragma unroll
        for (int q = 0; q < 9; ++q) f[i + q * p.fq] = (float)(wgt<double>(q) * rho);
    }
}

// Sum, min and max of the profile density over the lattice: one partial triple per block in a
// fixed pattern; the host adds the partials in block order.
__global__ void __launch_bounds__(256) profile_mass_kernel(int nx, int ny, Profile P,
                                                           double *__restrict__ partial) {
    __shared__ double sh[3][256];
    double s = 0.0, lo = INFINITY, hi = -INFINITY;
    const size_t N = (size_t)nx * ny;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < N; k += (size_t)gridDim.x * 256) {
        const int y = (int)(k / nx), x = (int)(k - (size_t)y * nx);
        const double r = profile_rho(P, nx, ny, x, y);
        s += r;
        lo = fmin(lo, r);
        hi = fmax(hi, r);
    }
    const int t = threadIdx.x;
    sh[0][t] = s;
    sh[1][t] = lo;
    sh[2][t] = hi;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sh[0][t] += sh[0][t + h];
            sh[1][t] = fmin(sh[1][t], sh[1][t + h]);
            sh[2][t] = fmax(sh[2][t], sh[2][t + h]);
        }
        __syncthreads();
    }
    if (t < 3) partial[3 * (size_t)blockIdx.x + t] = sh[t][0];
}

struct NodeMacro {
    double rho, vx, vy;
    bool finite;
};

// rho and v = u + F/(2 rho) of node (x, y) from the populations and the psi plane, FP64.
__device__ __forceinline__ NodeMacro node_macro(const Physics &p, const float *__restrict__ f,
                                                const float *__restrict__ psi, int x, int y) {
    float v[9];
    load9(f, (size_t)y * p.frow + x, p.fq, v);
    const double rho = density9<double>(v);
    const double jx = (((double)v[1] - v[3]) + ((double)v[5] - v[7])) + ((double)v[8] - v[6]);
    const double jy = (((double)v[2] - v[4]) + ((double)v[5] - v[7])) + ((double)v[6] - v[8]);
    const int xe = x + 1 == p.nx ? 0 : x + 1, xw = x == 0 ? p.nx - 1 : x - 1;
    const int yn = y + 1 == p.ny ? 0 : y + 1, ys = y == 0 ? p.ny - 1 : y - 1;
    auto P = [&](int xx, int yy) { return (double)psi[(size_t)yy * p.pitch + xx]; };
    const double pc = P(x, y), pE = P(xe, y), pW = P(xw, y), pN = P(x, yn), pS = P(x, ys);
    const double pNE = P(xe, yn), pNW = P(xw, yn), pSW = P(xw, ys), pSE = P(xe, ys);
    const double dA = pNE - pSW, dB = pSE - pNW;
    const double s1x = (pE - pW) / 3.0 + (dA + dB) / 12.0;
    const double s1y = (pN - pS) / 3.0 + (dA - dB) / 12.0;
    const double qA = dA * (pNE + pSW), qB = dB * (pSE + pNW);
    const double s2x = (pE - pW) * (pE + pW) / 3.0 + (qA + qB) / 12.0;
    const double s2y = (pN - pS) * (pN + pS) / 3.0 + (qA - qB) / 12.0;
    const double gA = -p.G * p.A / 2.0, gB = -p.G * (1.0 - p.A);
    const double Fx = gB * pc * s1x + gA * s2x, Fy = gB * pc * s1y + gA * s2y;
    NodeMacro m;
    m.rho = rho;
    m.vx = jx / rho + Fx / (2.0 * rho);
    m.vy = jy / rho + Fy / (2.0 * rho);
    m.finite = isfinite(rho) && isfinite(m.vx) && isfinite(m.vy) && isfinite(pc);
    return m;
}

// Rest state consistent with the force: f holds f^eq(rho, 0) and psi the plane of that state;
// each node is rewritten in place as f^eq(rho, u) with u = -F / (2 rho), so that the physical
// velocity v = u + F / (2 rho) (Sec. 3) starts at zero.  A bare f^eq(rho, 0) start carries
// v = F / (2 rho) at every interface, an impulse that rings for thousands of steps.
__global__ void __launch_bounds__(256) rest_kernel(Physics p, float *__restrict__ f,
                                                   const float *__restrict__ psi) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= p.nx) return;
    for (int y = blockIdx.y; y < p.ny; y += gridDim.y) {
        const NodeMacro m = node_macro(p, f, psi, x, y);  // j = 0, so v = F / (2 rho)
        double s[9];
        eq_shape<double>(-m.vx, -m.vy, s);
        const size_t i = (size_t)y * p.frow + x;
#pragma unroll
        for (int q = 0; q < 9; ++q) f[i + q * p.fq] = (float)(wgt<double>(q) * m.rho * (1.0 + s[q]));
    }
}

__global__ void __launch_bounds__(256) macro_kernel(Physics p, const float *__restrict__ f,
                                                    const float *__restrict__ psi,
                                                    double *__restrict__ rho,
                                                    double *__restrict__ u) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= p.nx) return;
    for (int y = blockIdx.y; y < p.ny; y += gridDim.y) {
        const NodeMacro m = node_macro(p, f, psi, x, y);
        const size_t k = (size_t)y * p.nx + x;
        if (rho) rho[k] = m.rho;
        if (u) {
            u[2 * k] = m.vx;
            u[2 * k + 1] = m.vy;
        }
    }
}

constexpr int kStatsBlock = 256;
constexpr int kStatsMaxBlocks = 2048;

// Block-level reduction in a fixed pattern (deterministic for a fixed block size).
__device__ void block_reduce(double v[kStatsFields], double (*sh)[kStatsBlock]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kStatsFields; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int s = kStatsBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] += sh[0][t + s];
            sh[1][t] = fmin(sh[1][t], sh[1][t + s]);
            sh[2][t] = fmax(sh[2][t], sh[2][t + s]);
            sh[3][t] = fmax(sh[3][t], sh[3][t + s]);
            sh[4][t] = fmax(sh[4][t], sh[4][t + s]);
            sh[5][t] += sh[5][t + s];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kStatsBlock) stats_kernel(Physics p, const float *__restrict__ f,
                                                            const float *__restrict__ psi,
                                                            float *__restrict__ vprev,
                                                            double *__restrict__ partial) {
    __shared__ double sh[kStatsFields][kStatsBlock];
    double acc[kStatsFields] = {0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
    const size_t N = (size_t)p.nx * p.ny;
    const size_t stride = (size_t)gridDim.x * kStatsBlock;
    for (size_t k = (size_t)blockIdx.x * kStatsBlock + threadIdx.x; k < N; k += stride) {
        const int y = (int)(k / p.nx), x = (int)(k - (size_t)y * p.nx);
        const NodeMacro m = node_macro(p, f, psi, x, y);
        if (!m.finite) {
            acc[5] += 1.0;
            continue;
        }
        acc[0] += m.rho;
        acc[1] = fmin(acc[1], m.rho);
        acc[2] = fmax(acc[2], m.rho);
        acc[3] = fmax(acc[3], sqrt(m.vx * m.vx + m.vy * m.vy));
        if (vprev) {
            const double dvx = m.vx - (double)vprev[2 * k], dvy = m.vy - (double)vprev[2 * k + 1];
            acc[4] = fmax(acc[4], fmax(fabs(dvx), fabs(dvy)));
            vprev[2 * k] = (float)m.vx;
            vprev[2 * k + 1] = (float)m.vy;
        }
    }
    block_reduce(acc, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < kStatsFields; ++q) partial[(size_t)blockIdx.x * kStatsFields + q] = sh[q][0];
}

__global__ void __launch_bounds__(kStatsBlock) stats_final_kernel(Physics p, const float *__restrict__ f,
                                                                  const double *__restrict__ partial,
                                                                  int nblocks, double *__restrict__ out,
                                                                  int xa, int ya, int xb, int yb) {
    __shared__ double sh[kStatsFields][kStatsBlock];
    double acc[kStatsFields] = {0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kStatsBlock) {
        const double *q = partial + (size_t)b * kStatsFields;
        acc[0] += q[0];
        acc[1] = fmin(acc[1], q[1]);
        acc[2] = fmax(acc[2], q[2]);
        acc[3] = fmax(acc[3], q[3]);
        acc[4] = fmax(acc[4], q[4]);
        acc[5] += q[5];
    }
    block_reduce(acc, sh);
    if (threadIdx.x < kStatsFields) out[threadIdx.x] = sh[threadIdx.x][0];
    if (threadIdx.x == 0 || threadIdx.x == 1) {
        const int x = threadIdx.x == 0 ? xa : xb, y = threadIdx.x == 0 ? ya : yb;
        float v[9];
        load9(f, (size_t)y * p.frow + x, p.fq, v);
        out[kStatsFields + threadIdx.x] = density9<double>(v);
    }
}

// Batch observables.  Block b covers chunk sb[b].y of sb[b].z chunks of lattice sb[b].x and
// writes its partial at sb[b].w; one final block per lattice reduces its chunks in order.
__global__ void __launch_bounds__(kStatsBlock) batch_stats_kernel(const BatchLattice *__restrict__ lats,
                                                                  const int4 *__restrict__ sb, int parity,
                                                                  int track, double *__restrict__ partial) {
    __shared__ double sh[kStatsFields][kStatsBlock];
    double acc[kStatsFields] = {0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
    const int4 d = sb[blockIdx.x];
    const BatchLattice &L = lats[d.x];
    const float *f = L.f[parity];
    const size_t N = (size_t)L.c.nx * L.c.ny;
    const size_t stride = (size_t)d.z * kStatsBlock;
    for (size_t k = (size_t)d.y * kStatsBlock + threadIdx.x; k < N; k += stride) {
        const int y = (int)(k / L.c.nx), x = (int)(k - (size_t)y * L.c.nx);
        batch_node(L, f, x, y, acc, k, track != 0);
    }
    block_reduce(acc, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < kStatsFields; ++q) partial[(size_t)d.w * kStatsFields + q] = sh[q][0];
}

__global__ void __launch_bounds__(kStatsBlock) batch_stats_final_kernel(const BatchLattice *__restrict__ lats,
                                                                        const int2 *__restrict__ ranges,
                                                                        const int *__restrict__ ids,
                                                                        int parity, const double *__restrict__ partial,
                                                                        double *__restrict__ out) {
    __shared__ double sh[kStatsFields][kStatsBlock];
    double acc[kStatsFields] = {0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
    const int2 r = ranges[blockIdx.x];  // first partial, count
    for (int b = threadIdx.x; b < r.y; b += kStatsBlock) {
        const double *q = partial + (size_t)(r.x + b) * kStatsFields;
        acc[0] += q[0];
        acc[1] = fmin(acc[1], q[1]);
        acc[2] = fmax(acc[2], q[2]);
        acc[3] = fmax(acc[3], q[3]);
        acc[4] = fmax(acc[4], q[4]);
        acc[5] += q[5];
    }
    block_reduce(acc, sh);
    const int id = ids[blockIdx.x];
    double *o = out + (size_t)id * kStatsOut;
    if (threadIdx.x < kStatsFields) o[threadIdx.x] = sh[threadIdx.x][0];
    if (threadIdx.x == 0 || threadIdx.x == 1) {
        const BatchLattice &L = lats[id];
        const int x = threadIdx.x == 0 ? L.xa : L.xb, y = threadIdx.x == 0 ? L.ya : L.yb;
        float v[9];
        load9(L.f[parity], (size_t)y * L.c.frow + x, L.c.fq, v);
        o[kStatsFields + threadIdx.x] = density9<double>(v);
    }
}

__global__ void __launch_bounds__(256) copy_kernel(float4 *__restrict__ dst,
                                                   const float4 *__restrict__ src, size_t n4) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void copy_tail_kernel(float *__restrict__ dst, const float *__restrict__ src,
                                 size_t from, size_t n) {
    const size_t i = from + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------------
// Squared norms of the rows of the D2Q9 moment matrix (rho, e, epsilon, j_x, q_x, j_y, q_y,
// p_xx, p_xy): its rows are orthogonal, so M^-1 = M^T diag(1 / norm).
constexpr double kRowNorm[9] = {9.0, 36.0, 36.0, 6.0, 12.0, 6.0, 12.0, 4.0, 4.0};

template <typename R, typename D>
StepConst<R, D> make_const(const Physics &p, int flags) {
    StepConst<R, D> c{};
    c.nx = p.nx;
    c.ny = p.ny;
    c.pitch = p.pitch;
    c.frow = p.frow;
    c.fq = p.fq;
    c.fbytes = (unsigned)(pop_bytes(p) > kSweepMaxBytes ? kSweepMaxBytes : pop_bytes(p));
    c.ffloats = pop_bytes(p) / sizeof(float);
    c.flags = flags;
    c.bq = (D)p.b_quarter;
    c.e1 = (D)(2.0 * p.K * p.RT / p.G);
    c.e2 = (D)(2.0 * p.K * p.a / p.G);
    c.e3 = (D)(2.0 / (3.0 * p.G));
    c.psi_kind = p.psi_kind;
    c.inv_eps = (D)p.inv_eps;
    c.tau = (D)p.tau;
    c.gA = (D)(-p.G * p.A / 2.0);
    c.gB = (D)(-p.G * (1.0 - p.A));
    c.omega = (D)(1.0 / p.tau);
    c.li2 = (R)(2.0 * p.sigma);
    for (int k = 0; k < 9; ++k) {
        c.sd[k] = (D)(p.s[k] / kRowNorm[k]);
        c.hd[k] = (D)((1.0 - p.s[k] / 2.0) / kRowNorm[k]);
        c.lim[k] = (R)(1.0 / (1.0 / p.s[k] - 0.5));
    }
    return c;
}

dim3 row_grid(int nx, int ny, int block) {
    return dim3((unsigned)((nx + block - 1) / block), (unsigned)(ny < 65535 ? ny : 65535));
}

// Instantiates KERNEL<R, D, scheme, collision EXTRA> for the run-time scheme; EXTRA is empty or
// a further template argument list starting with a comma.  The exact-difference and Shan-Chen
// schemes are BGK only; Guo's schemes (with or without Li's term) run one kernel for both
// collisions -- their collision is computed in moment space, BGK being every rate 1/tau -- which
// is instantiated with COLL = MRT (kernel_kind in lbm_internal.h names the same grouping).
#define PPLBM_DISPATCH_X(KERNEL, R, D, EXTRA, p, grid, block, lds, s, ...)                        \
    do {                                                                                        \
        if ((p).scheme == EDM)                                                                  \
            hipLaunchKernelGGL((KERNEL<R, D, EDM, BGK EXTRA>), grid, block, lds, s, __VA_ARGS__);        \
        else if ((p).scheme == SC)                                                              \
            hipLaunchKernelGGL((KERNEL<R, D, SC, BGK EXTRA>), grid, block, lds, s, __VA_ARGS__);         \
        else if ((p).scheme == GUO)                                                             \
            hipLaunchKernelGGL((KERNEL<R, D, GUO, MRT EXTRA>), grid, block, lds, s, __VA_ARGS__);        \
        else                                                                                    \
            hipLaunchKernelGGL((KERNEL<R, D, GUO_LI, MRT EXTRA>), grid, block, lds, s, __VA_ARGS__);     \
    } while (0)
#define PPLBM_NOEXTRA
#define PPLBM_PF1 , 1
#define PPLBM_PF2 , 2
#define PPLBM_PF1_BIG , 1, true
#define PPLBM_BIG , true
#define PPLBM_PF2_BIG , 2, true
#define PPLBM_DISPATCH(KERNEL, R, D, p, grid, block, lds, s, ...) \
    PPLBM_DISPATCH_X(KERNEL, R, D, PPLBM_NOEXTRA, p, grid, block, lds, s, __VA_ARGS__)

template <typename R, typename D>
hipError_t psi_dispatch(const Physics &p, int flags, const float *fin, float *psi, hipStream_t s) {
    const StepConst<R, D> c = make_const<R, D>(p, flags);
    const dim3 grid((unsigned)((p.nx + 4 * 256 - 1) / (4 * 256)),
                    (unsigned)(p.ny < 65535 ? p.ny : 65535));
    hipLaunchKernelGGL((psi_kernel<R, D>), grid, dim3(256), 0, s, fin, psi, c);
    return hipGetLastError();
}

template <typename R, typename D>
hipError_t fused_dispatch(const Physics &p, const Launch &L, const float *fin, const float *psi,
                          float *fout, hipStream_t s) {
    const StepConst<R, D> c = make_const<R, D>(p, L.flags);
    const dim3 grid((unsigned)((p.nx + L.tx - 1) / L.tx), (unsigned)((p.ny + L.ty - 1) / L.ty));
    const size_t lds = (size_t)(L.tx + 2) * (L.ty + 2) * sizeof(float);
    PPLBM_DISPATCH(fused_kernel, R, D, p, grid, dim3(L.tx, L.ty), lds, s, fin, psi, fout, c);
    return hipGetLastError();
}

template <typename R, typename D>
hipError_t sweep_dispatch(const Physics &p, const Launch &L, const float *fin, float *fout,
                          hipStream_t s) {
    const StepConst<R, D> c = make_const<R, D>(p, L.flags);
    const dim3 grid((unsigned)((p.nx + L.tx - 1) / L.tx), (unsigned)((p.ny + L.ty - 1) / L.ty));
    const size_t lds = 4 * (size_t)(L.tx + 2) * sizeof(float);
    if (pop_bytes(p) > kSweepMaxBytes) {  // per-row resources (row-interleaved layout only)
        if (p.fq != p.pitch) return hipErrorInvalidValue;
        if constexpr (sizeof(R) == 8) {
            if (L.flags & kFlagShallow)
                PPLBM_DISPATCH_X(sweep_kernel, R, D, PPLBM_PF1_BIG, p, grid, dim3(L.tx), lds, s, fin, fout, c, L.ty);
            else
                PPLBM_DISPATCH_X(sweep_kernel, R, D, PPLBM_PF2_BIG, p, grid, dim3(L.tx), lds, s, fin, fout, c, L.ty);
        } else {
            if (L.flags & kFlagShallow)
                PPLBM_DISPATCH_X(sweep_kernel_w5, R, D, PPLBM_PF1_BIG, p, grid, dim3(L.tx), lds, s, fin, fout, c, L.ty);
            else
                PPLBM_DISPATCH_X(sweep_kernel_w5, R, D, PPLBM_PF2_BIG, p, grid, dim3(L.tx), lds, s, fin, fout, c, L.ty);
        }
        return hipGetLastError();
    }
    if constexpr (sizeof(R) == 8) {
        if (L.flags & kFlagShallow)
            PPLBM_DISPATCH_X(sweep_kernel, R, D, PPLBM_PF1, p, grid, dim3(L.tx), lds, s, fin, fout, c, L.ty);
        else
            PPLBM_DISPATCH_X(sweep_kernel, R, D, PPLBM_PF2, p, grid, dim3(L.tx), lds, s, fin, fout, c, L.ty);
    } else {
        if (L.flags & kFlagShallow)
            PPLBM_DISPATCH_X(sweep_kernel_w5, R, D, PPLBM_PF1, p, grid, dim3(L.tx), lds, s, fin, fout, c, L.ty);
        else
            PPLBM_DISPATCH_X(sweep_kernel_w5, R, D, PPLBM_PF2, p, grid, dim3(L.tx), lds, s, fin, fout, c, L.ty);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_psi(const Physics &p, int prec, int flags, const float *f, float *psi,
                      hipStream_t s) {
    switch (prec) {
    case kPrecF64: return psi_dispatch<double, double>(p, flags, f, psi, s);
    default: return psi_dispatch<float, double>(p, flags, f, psi, s);
    }
}

hipError_t launch_fused(const Physics &p, int prec, const Launch &L, const float *fin,
                        const float *psi, float *fout, hipStream_t s) {
    switch (prec) {
    case kPrecF64: return fused_dispatch<double, double>(p, L, fin, psi, fout, s);
    default: return fused_dispatch<float, double>(p, L, fin, psi, fout, s);
    }
}

namespace {
template <typename R, typename D>
hipError_t sweep2_dispatch(const Physics &p, const Launch &L, const float *fin, float *fout,
                           hipStream_t s) {
    const StepConst<R, D> c = make_const<R, D>(p, L.flags);
    const int nstrips = (p.nx + kSweep2Out - 1) / kSweep2Out;
    const int nseg = (p.ny + L.ty - 1) / L.ty;
    const int ntiles = nstrips * nseg, wpg = L.tx / 64;
    const dim3 grid((unsigned)((ntiles + wpg - 1) / wpg));
    if (pop_bytes(p) > kSweepMaxBytes) {  // per-row resources (row-interleaved layout only)
        if (p.fq != p.pitch) return hipErrorInvalidValue;
        PPLBM_DISPATCH_X(sweep2_kernel, R, D, PPLBM_BIG, p, grid, dim3(L.tx), 0, s, fin, fout, c,
                         L.ty, nstrips, ntiles);
    } else {
        PPLBM_DISPATCH(sweep2_kernel, R, D, p, grid, dim3(L.tx), 0, s, fin, fout, c, L.ty,
                       nstrips, ntiles);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_sweep2(const Physics &p, int prec, const Launch &L, const float *fin,
                         float *fout, hipStream_t s) {
    switch (prec) {
    case kPrecF64: return sweep2_dispatch<double, double>(p, L, fin, fout, s);
    default: return sweep2_dispatch<float, double>(p, L, fin, fout, s);
    }
}

hipError_t launch_sweep(const Physics &p, int prec, const Launch &L, const float *fin,
                        float *fout, hipStream_t s) {
    switch (prec) {
    case kPrecF64: return sweep_dispatch<double, double>(p, L, fin, fout, s);
    default: return sweep_dispatch<float, double>(p, L, fin, fout, s);
    }
}

hipError_t launch_init(const Physics &p, const double *rho0, const double *u0, float *f,
                       hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, row_grid(p.nx, p.ny, 256), dim3(256), 0, s, p, rho0, u0, f);
    return hipGetLastError();
}

hipError_t launch_rest(const Physics &p, float *f, float *psi, hipStream_t s) {
    hipError_t e = launch_psi(p, kPrecF64, 0, f, psi, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rest_kernel, row_grid(p.nx, p.ny, 256), dim3(256), 0, s, p, f, psi);
    return hipGetLastError();
}

hipError_t launch_macro(const Physics &p, const float *f, const float *psi, double *rho,
                        double *u, hipStream_t s) {
    hipLaunchKernelGGL(macro_kernel, row_grid(p.nx, p.ny, 256), dim3(256), 0, s, p, f, psi, rho,
                       u);
    return hipGetLastError();
}

namespace {
Profile make_profile(const double *log_rho, double r0, double dr, double shift) {
    Profile P;
    for (int k = 0; k < kProfilePoints; ++k) P.v[k] = log_rho[k];
    P.r0 = r0;
    P.inv_dr = 1.0 / dr;
    P.shift = shift;
    return P;
}
}  // namespace

int profile_mass_blocks(const Physics &p) {
    const size_t N = (size_t)p.nx * p.ny, b = (N + 255) / 256;
    return (int)(b < 1024 ? b : 1024);
}

hipError_t launch_profile_mass(const Physics &p, const double *log_rho, double r0, double dr,
                               double shift, double *partial, hipStream_t s) {
    hipLaunchKernelGGL(profile_mass_kernel, dim3(profile_mass_blocks(p)), dim3(256), 0, s, p.nx,
                       p.ny, make_profile(log_rho, r0, dr, shift), partial);
    return hipGetLastError();
}

hipError_t launch_profile_init(const Physics &p, const double *log_rho, double r0, double dr,
                               double shift, float *f, hipStream_t s) {
    hipLaunchKernelGGL(profile_init_kernel, row_grid(p.nx, p.ny, 256), dim3(256), 0, s, p,
                       make_profile(log_rho, r0, dr, shift), f);
    return hipGetLastError();
}

size_t stats_partial_count(const Physics &p) {
    const size_t N = (size_t)p.nx * p.ny;
    size_t b = (N + kStatsBlock - 1) / kStatsBlock;
    return b < (size_t)kStatsMaxBlocks ? b : (size_t)kStatsMaxBlocks;
}

hipError_t launch_stats(const Physics &p, const float *f, const float *psi, float *vprev,
                        double *partial, double *out, int xa, int ya, int xb, int yb,
                        hipStream_t s) {
    const int nb = (int)stats_partial_count(p);
    hipLaunchKernelGGL(stats_kernel, dim3(nb), dim3(kStatsBlock), 0, s, p, f, psi, vprev, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(kStatsBlock), 0, s, p, f, partial, nb, out,
                       xa, ya, xb, yb);
    return hipGetLastError();
}

size_t batch_lattice_bytes() { return sizeof(BatchLattice); }

void batch_lattice_fill(const Physics &p, float *f0, float *f1, float *vprev, int xa, int ya,
                        int xb, int yb, int flags, void *out) {
    BatchLattice L{};
    L.c = make_const<float, double>(p, flags);
    L.f[0] = f0;
    L.f[1] = f1;
    L.vprev = vprev;
    L.scheme = p.scheme;
    L.coll = p.coll;
    L.xa = xa;
    L.ya = ya;
    L.xb = xb;
    L.yb = yb;
    *reinterpret_cast<BatchLattice *>(out) = L;
}

hipError_t launch_batch_kind(const void *lats, const int4 *tiles, const int2 *meta, int kind,
                             int scheme, int coll, int parity, int tx, int groups, bool shallow,
                             hipStream_t s) {
    const size_t lds = 4 * (size_t)(tx + 2) * sizeof(float);
    const BatchLattice *L = reinterpret_cast<const BatchLattice *>(lats);
    const dim3 g(groups), blk(tx);
#define PPLBM_KIND(S, C)                                                                         \
    if (shallow)                                                                                 \
        hipLaunchKernelGGL((batch_kind_kernel<S, C, 1>), g, blk, lds, s, L, tiles, meta, kind, parity); \
    else                                                                                         \
        hipLaunchKernelGGL((batch_kind_kernel<S, C, 2>), g, blk, lds, s, L, tiles, meta, kind, parity)
    switch (scheme * 2 + coll) {
    case EDM * 2 + BGK: PPLBM_KIND(EDM, BGK); break;
    case SC * 2 + BGK: PPLBM_KIND(SC, BGK); break;
    case GUO * 2 + MRT: PPLBM_KIND(GUO, MRT); break;
    case GUO_LI * 2 + MRT: PPLBM_KIND(GUO_LI, MRT); break;
    default: return hipErrorInvalidValue;
    }
#undef PPLBM_KIND
    return hipGetLastError();
}

hipError_t launch_batch2_kind(const void *lats, const int4 *tiles, const int2 *meta, int kind,
                              int scheme, int coll, int parity, int groups, hipStream_t s) {
    const BatchLattice *L = reinterpret_cast<const BatchLattice *>(lats);
    const dim3 g(groups), blk(256);
#define PPLBM_KIND2(S, C) \
    hipLaunchKernelGGL((batch2_kind_kernel<S, C>), g, blk, 0, s, L, tiles, meta, kind, parity)
    switch (scheme * 2 + coll) {
    case EDM * 2 + BGK: PPLBM_KIND2(EDM, BGK); break;
    case SC * 2 + BGK: PPLBM_KIND2(SC, BGK); break;
    case GUO * 2 + MRT: PPLBM_KIND2(GUO, MRT); break;
    case GUO_LI * 2 + MRT: PPLBM_KIND2(GUO_LI, MRT); break;
    default: return hipErrorInvalidValue;
    }
#undef PPLBM_KIND2
    return hipGetLastError();
}

int sweep2_out_columns() { return kSweep2Out; }

hipError_t launch_batch_stats(const void *lats, const int4 *sblocks, int nsblocks,
                              const int2 *ranges, const int *ids, int nlat, int parity, int track,
                              double *partial, double *out, hipStream_t s) {
    const BatchLattice *L = reinterpret_cast<const BatchLattice *>(lats);
    hipLaunchKernelGGL(batch_stats_kernel, dim3(nsblocks), dim3(kStatsBlock), 0, s, L, sblocks, parity,
                       track, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_stats_final_kernel, dim3(nlat), dim3(kStatsBlock), 0, s, L, ranges, ids,
                       parity, partial, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Allocation-free observables (lbm_stats_noalloc): the reduction's block partials and its
// result vector live in one fixed device array, one copy per GPU, held until the process ends.
// Every reduction writes all the partials and results it reads, so nothing is cleared between
// calls; calls that overlap on one GPU race on it.  Host code never passes the array's name to
// a kernel or a copy (in host code it is a stand-in, not a device address): it takes the
// address hipGetSymbolAddress reports for the current device, looked up once per device.
// ---------------------------------------------------------------------------------------
constexpr size_t kScratchDoubles = (size_t)kStatsMaxBlocks * kStatsFields + kStatsOut;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kScratchMaxDevices = 64;
std::mutex scratch_mutex;
double *scratch_dev[kScratchMaxDevices];  // address of `scratch` on each device, once known
}  // namespace

hipError_t stats_scratch(double **ptr, size_t *doubles) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_dev[dev] = static_cast<double *>(p);
    }
    *ptr = scratch_dev[dev];
    if (doubles) *doubles = kScratchDoubles;
    return hipSuccess;
}

hipError_t launch_copy(float *dst, const float *src, size_t n, hipStream_t s) {
    const size_t n4 = n / 4;
    if (n4) {
        size_t blocks = (n4 + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<float4 *>(dst), reinterpret_cast<const float4 *>(src), n4);
    }
    if (n4 * 4 < n)
        hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(4), 0, s, dst, src, n4 * 4, n);
    return hipGetLastError();
}

}  // namespace pplbm
