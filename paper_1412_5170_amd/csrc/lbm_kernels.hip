// gfx950 kernels of the pseudo-potential D2Q9 lattice Boltzmann step (arXiv:1412.5170).
//
// State: FP32 populations in nine SoA planes (plane q at q * plane, node at y * pitch + x),
// double-buffered; one FP32 psi plane.  A time step is two launches:
//   psi_kernel    rho = sum_q f_q (Eq. 3), psi from the K-rescaled Carnahan-Starling EOS
//                 (Eq. 29-30) through p0 = rho/3 + G psi^2/2 (Eq. 7).  Reads 36 B, writes 4 B
//                 per node.
//   fused_kernel  stages the psi tile plus a one-node halo in LDS, forms the hybrid
//                 interaction force (Eq. 6; Eq. 4 for A = 0), the moments and velocities
//                 (Sec. 3.2), the forcing scheme (EDM Eq. 22, Guo Eq. 23, Guo + Li Eq. 31),
//                 the BGK (Eq. 1) or MRT (Eq. 34-35) collision, and pushes f* to the
//                 neighbours (Eq. 36, periodic).  Reads 36 B + psi, writes 36 B per node.
// The arithmetic type R is float or double; storage is FP32 either way.
//
// Velocity order: 0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1),
// 7 (-1,-1), 8 (1,-1).  All formulas below are unrolled by hand for this order.

#include <cmath>
#include <cstdint>

#include "lbm_internal.h"

namespace pplbm {
namespace {

template <typename R>
__device__ __forceinline__ R qnan();
template <>
__device__ __forceinline__ float qnan<float>() { return __builtin_nanf(""); }
template <>
__device__ __forceinline__ double qnan<double>() { return __builtin_nan(""); }

__device__ __forceinline__ int wrap_any(int g, int n) {
    g %= n;
    return g < 0 ? g + n : g;
}

// rho = sum_q f_q in one fixed order, shared by every kernel that needs it.
template <typename R>
__device__ __forceinline__ R density(R f0, R f1, R f2, R f3, R f4, R f5, R f6, R f7, R f8) {
    return ((f0 + (f1 + f3)) + (f2 + f4)) + ((f5 + f7) + (f6 + f8));
}

// Effective density of Eq. 7 with the rescaled Carnahan-Starling pressure of Eq. 29-30.
// NaN when the node is outside the EOS (b rho/4 >= 1) or 2 U / G <= 0.
template <typename R>
__device__ __forceinline__ R eos_psi(R rho, R bq, R RT, R a, R K, R two_over_G) {
    const R eta = bq * rho;
    if (!(eta < R(1)) || !(rho > R(0))) return qnan<R>();
    const R om = R(1) - eta;
    const R Z = (R(1) + eta * (R(1) + eta * (R(1) - eta))) / (om * om * om);
    const R p0 = K * (rho * (RT * Z - a * rho));
    const R r = two_over_G * (p0 - rho / R(3));
    return r > R(0) ? sqrt(r) : qnan<R>();
}

// ---------------------------------------------------------------------------------------
// Density / psi pass.
// ---------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) psi_kernel(const float *__restrict__ f,
                                                  float *__restrict__ psi, int nx, int ny,
                                                  size_t pitch, size_t plane, R bq, R RT, R a,
                                                  R K, R two_over_G) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    for (int y = blockIdx.y; y < ny; y += gridDim.y) {
        const size_t i = (size_t)y * pitch + x;
        const R rho = density<R>(f[i], f[i + plane], f[i + 2 * plane], f[i + 3 * plane],
                                 f[i + 4 * plane], f[i + 5 * plane], f[i + 6 * plane],
                                 f[i + 7 * plane], f[i + 8 * plane]);
        psi[i] = (float)eos_psi<R>(rho, bq, RT, a, K, two_over_G);
    }
}

// ---------------------------------------------------------------------------------------
// Fused force + collision + streaming pass.
// ---------------------------------------------------------------------------------------
template <typename R>
struct StepConst {
    int nx, ny;
    size_t pitch, plane;
    R gA;     // -G A / 2        coefficient of sum w psi^2 e    (Eq. 6, U = G psi^2 / 2)
    R gB;     // -G (1 - A)      coefficient of psi(x) sum w psi e
    R omega;  // 1 / tau
    R kguo;   // 1 - 1/(2 tau)   (Eq. 23)
    R li;     // sigma / (tau - 1/2): v' = v + li F / psi^2 (Eq. 31)
    R li2;    // 2 sigma: Li's extra stress X = li2 F F / psi^2 (MRT form)
    R s[9];   // MRT rates in moment order
    R hs[9];  // 1 - s/2
    R lim[9]; // 1 / (1/s_k - 1/2) for the moments that carry Li's stress
};

template <typename R>
__device__ __forceinline__ void equilibrium(R rho, R ux, R uy, R fe[9]) {
    // Eq. 2 with c_s^2 = 1/3: w rho (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u)
    const R w0 = R(4) / R(9), w1 = R(1) / R(9), w2 = R(1) / R(36);
    const R usq = R(1.5) * (ux * ux + uy * uy);
    const R r0 = w0 * rho, r1 = w1 * rho, r2 = w2 * rho;
    fe[0] = r0 * (R(1) - usq);
    const R ea[4] = {ux, uy, -ux, -uy};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const R e = ea[q];
        fe[1 + q] = r1 * (R(1) + R(3) * e + R(4.5) * e * e - usq);
    }
    const R ed[4] = {ux + uy, uy - ux, -ux - uy, ux - uy};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const R e = ed[q];
        fe[5 + q] = r2 * (R(1) + R(3) * e + R(4.5) * e * e - usq);
    }
}

// Guo's bracket B_q = w_q [3 e.F + 9 (e.F)(e.V) - 3 F.V] (Eq. 23 with c_s^2 = 1/3).
template <typename R>
__device__ __forceinline__ void guo_bracket(R Fx, R Fy, R Vx, R Vy, R B[9]) {
    const R w0 = R(4) / R(9), w1 = R(1) / R(9), w2 = R(1) / R(36);
    const R FV = R(3) * (Fx * Vx + Fy * Vy);
    B[0] = -w0 * FV;
    const R eF[8] = {Fx, Fy, -Fx, -Fy, Fx + Fy, Fy - Fx, -Fx - Fy, Fx - Fy};
    const R eV[8] = {Vx, Vy, -Vx, -Vy, Vx + Vy, Vy - Vx, -Vx - Vy, Vx - Vy};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const R w = q < 4 ? w1 : w2;
        B[1 + q] = w * (R(3) * eF[q] + R(9) * eF[q] * eV[q] - FV);
    }
}

template <typename R, int SCHEME, int COLL>
__global__ void __launch_bounds__(1024) fused_kernel(const float *__restrict__ fin,
                                                     const float *__restrict__ psi,
                                                     float *__restrict__ fout,
                                                     StepConst<R> c) {
    extern __shared__ float tile[];
    const int TX = blockDim.x, TY = blockDim.y;
    const int W = TX + 2;
    const int nx = c.nx, ny = c.ny;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tx = threadIdx.x, ty = threadIdx.y;

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

    const int x = x0 + tx, y = y0 + ty;
    if (x >= nx || y >= ny) return;

    const size_t pl = c.plane;
    const size_t i = (size_t)y * c.pitch + x;
    const R f0 = fin[i], f1 = fin[i + pl], f2 = fin[i + 2 * pl], f3 = fin[i + 3 * pl],
            f4 = fin[i + 4 * pl], f5 = fin[i + 5 * pl], f6 = fin[i + 6 * pl],
            f7 = fin[i + 7 * pl], f8 = fin[i + 8 * pl];

    // Interaction force, Eq. 6: sums over the eight links as differences of opposite pairs.
    const int lc = (ty + 1) * W + tx + 1;
    const R pc = tile[lc];
    const R pE = tile[lc + 1], pW = tile[lc - 1], pN = tile[lc + W], pS = tile[lc - W];
    const R pNE = tile[lc + W + 1], pNW = tile[lc + W - 1], pSW = tile[lc - W - 1],
            pSE = tile[lc - W + 1];
    const R third = R(1) / R(3), twelfth = R(1) / R(12);
    const R dA = pNE - pSW, dB = pSE - pNW;  // diagonal pair differences
    const R s1x = third * (pE - pW) + twelfth * (dA + dB);
    const R s1y = third * (pN - pS) + twelfth * (dA - dB);
    R Fx = c.gB * pc * s1x;
    R Fy = c.gB * pc * s1y;
    if (c.gA != R(0)) {
        // sum w psi^2 e with psi_a^2 - psi_b^2 = (psi_a - psi_b)(psi_a + psi_b)
        const R qA = dA * (pNE + pSW), qB = dB * (pSE + pNW);
        const R s2x = third * ((pE - pW) * (pE + pW)) + twelfth * (qA + qB);
        const R s2y = third * ((pN - pS) * (pN + pS)) + twelfth * (qA - qB);
        Fx += c.gA * s2x;
        Fy += c.gA * s2y;
    }

    // Moments (Eq. 3), u = sum f e / rho, v = u + F / (2 rho) (Sec. 3.2).
    const R rho = density<R>(f0, f1, f2, f3, f4, f5, f6, f7, f8);
    const R jx = ((f1 - f3) + (f5 - f7)) + (f8 - f6);
    const R jy = ((f2 - f4) + (f5 - f7)) + (f6 - f8);
    const R ux = jx / rho, uy = jy / rho;
    const R vx = ux + Fx / (R(2) * rho), vy = uy + Fy / (R(2) * rho);

    const R fin9[9] = {f0, f1, f2, f3, f4, f5, f6, f7, f8};
    R fs[9];
    R fe[9];
    if constexpr (COLL == BGK) {
        if constexpr (SCHEME == EDM) {
            // Eq. 22 with f^eq(rho, u + D) - f^eq(rho, u) written out exactly:
            // w rho [3 e.D + 9/2 (e.D)(e.(2u + D)) - 3/2 D.(2u + D)],  D = F / rho.
            equilibrium<R>(rho, ux, uy, fe);
            const R Dx = Fx / rho, Dy = Fy / rho;
            const R Sx = R(2) * ux + Dx, Sy = R(2) * uy + Dy;
            const R DS = R(1.5) * (Dx * Sx + Dy * Sy);
            const R eD[9] = {R(0), Dx, Dy, -Dx, -Dy, Dx + Dy, Dy - Dx, -Dx - Dy, Dx - Dy};
            const R eS[9] = {R(0), Sx, Sy, -Sx, -Sy, Sx + Sy, Sy - Sx, -Sx - Sy, Sx - Sy};
            const R wr[3] = {R(4) / R(9) * rho, R(1) / R(9) * rho, R(1) / R(36) * rho};
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const R w = q == 0 ? wr[0] : (q < 5 ? wr[1] : wr[2]);
                const R df = w * (R(3) * eD[q] + R(4.5) * eD[q] * eS[q] - DS);
                fs[q] = fin9[q] + c.omega * (fe[q] - fin9[q]) + df;
            }
        } else {
            // Eq. 23 (Guo) or Eq. 31 (Li): equilibrium at v, bracket at v or v'.
            equilibrium<R>(rho, vx, vy, fe);
            R bx = vx, by = vy;
            if constexpr (SCHEME == GUO_LI) {
                const R cl = c.li / (pc * pc);
                bx = vx + cl * Fx;
                by = vy + cl * Fy;
            }
            R B[9];
            guo_bracket<R>(Fx, Fy, bx, by, B);
#pragma unroll
            for (int q = 0; q < 9; ++q) fs[q] = fin9[q] + c.omega * (fe[q] - fin9[q]) + c.kguo * B[q];
        }
    } else {
        // MRT, Eq. 34: m* = m - Lambda (m - m_eq) + (I - Lambda/2) S with m_eq = M f^eq(rho, v).
        // Evaluated as f* = f - M^-1 [Lambda M (f - f^eq) - (I - Lambda/2) S] so that only
        // non-equilibrium quantities go through the transform (FP32 accuracy).
        equilibrium<R>(rho, vx, vy, fe);
        R d[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) d[q] = fin9[q] - fe[q];
        const R ax = d[1] + d[2] + d[3] + d[4], dg = d[5] + d[6] + d[7] + d[8];
        const R d13 = d[1] - d[3], d24 = d[2] - d[4], d57 = d[5] - d[7], d86 = d[8] - d[6],
                d68 = d[6] - d[8];
        R n[9];
        n[0] = (d[0] + ax) + dg;
        n[1] = -R(4) * d[0] - ax + R(2) * dg;
        n[2] = R(4) * d[0] - R(2) * ax + dg;
        n[3] = d13 + d57 + d86;
        n[4] = -R(2) * d13 + d57 + d86;
        n[5] = d24 + d57 + d68;
        n[6] = -R(2) * d24 + d57 + d68;
        n[7] = (d[1] + d[3]) - (d[2] + d[4]);
        n[8] = (d[5] + d[7]) - (d[6] + d[8]);
        // Guo's source in moment space, S = M B(v).
        const R vF = vx * Fx + vy * Fy;
        R S[9] = {R(0), R(6) * vF, -R(6) * vF, Fx, -Fx, Fy, -Fy,
                  R(2) * (vx * Fx - vy * Fy), vx * Fy + vy * Fx};
        if constexpr (SCHEME == GUO_LI) {
            const R cl = c.li2 / (pc * pc);
            const R Xxx = cl * Fx * Fx, Xyy = cl * Fy * Fy, Xxy = cl * Fx * Fy;
            const R tr3 = R(3) * (Xxx + Xyy);
            S[1] += tr3 * c.lim[1];
            S[2] -= tr3 * c.lim[2];
            S[7] += (Xxx - Xyy) * c.lim[7];
            S[8] += Xxy * c.lim[8];
        }
        R a[9];
        const R Dinv[9] = {R(1) / R(9), R(1) / R(36), R(1) / R(36), R(1) / R(6), R(1) / R(12),
                           R(1) / R(6), R(1) / R(12), R(1) / R(4), R(1) / R(4)};
#pragma unroll
        for (int k = 0; k < 9; ++k) a[k] = (c.s[k] * n[k] - c.hs[k] * S[k]) * Dinv[k];
        // M^-1 = M^T D^-1
        const R c0 = a[0] - a[1] - R(2) * a[2];
        const R c5 = a[0] + R(2) * a[1] + a[2];
        const R gx = a[3] - R(2) * a[4], gy = a[5] - R(2) * a[6];
        const R hx = a[3] + a[4], hy = a[5] + a[6];
        fs[0] = fin9[0] - (a[0] - R(4) * a[1] + R(4) * a[2]);
        fs[1] = fin9[1] - (c0 + gx + a[7]);
        fs[2] = fin9[2] - (c0 + gy - a[7]);
        fs[3] = fin9[3] - (c0 - gx + a[7]);
        fs[4] = fin9[4] - (c0 - gy - a[7]);
        fs[5] = fin9[5] - (c5 + hx + hy + a[8]);
        fs[6] = fin9[6] - (c5 - hx + hy - a[8]);
        fs[7] = fin9[7] - (c5 - hx - hy + a[8]);
        fs[8] = fin9[8] - (c5 + hx - hy - a[8]);
    }

    // Every scheme conserves mass exactly (sum_q f*_q = rho); closing the rest population on
    // it keeps the binary rounding of the weights 4/9, 1/9, 1/36 from drifting the mass.
    fs[0] = rho - (((fs[1] + fs[3]) + (fs[2] + fs[4])) + ((fs[5] + fs[7]) + (fs[6] + fs[8])));

    // Push streaming, Eq. 36: f_q(x + e_q, t + 1) = f*_q(x, t), periodic.
    const int xe = x + 1 == nx ? 0 : x + 1, xw = x == 0 ? nx - 1 : x - 1;
    const int yn = y + 1 == ny ? 0 : y + 1, ys = y == 0 ? ny - 1 : y - 1;
    const size_t rc = (size_t)y * c.pitch, rn = (size_t)yn * c.pitch, rs = (size_t)ys * c.pitch;
    fout[rc + x] = (float)fs[0];
    fout[pl + rc + xe] = (float)fs[1];
    fout[2 * pl + rn + x] = (float)fs[2];
    fout[3 * pl + rc + xw] = (float)fs[3];
    fout[4 * pl + rs + x] = (float)fs[4];
    fout[5 * pl + rn + xe] = (float)fs[5];
    fout[6 * pl + rn + xw] = (float)fs[6];
    fout[7 * pl + rs + xw] = (float)fs[7];
    fout[8 * pl + rs + xe] = (float)fs[8];
}

// ---------------------------------------------------------------------------------------
// Initial state, read-out and observables (FP64 arithmetic on the FP32 state).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) init_kernel(const double *__restrict__ rho0,
                                                   const double *__restrict__ u0,
                                                   float *__restrict__ f, int nx, int ny,
                                                   size_t pitch, size_t plane) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    for (int y = blockIdx.y; y < ny; y += gridDim.y) {
        const size_t k = (size_t)y * nx + x;
        const double ux = u0 ? u0[2 * k] : 0.0, uy = u0 ? u0[2 * k + 1] : 0.0;
        double fe[9];
        equilibrium<double>(rho0[k], ux, uy, fe);
        const size_t i = (size_t)y * pitch + x;
#pragma unroll
        for (int q = 0; q < 9; ++q) f[i + q * plane] = (float)fe[q];
    }
}

struct NodeMacro {
    double rho, vx, vy;
    bool finite;
};

// rho and v = u + F/(2 rho) of node (x, y) from the populations and the psi plane, FP64.
__device__ __forceinline__ NodeMacro node_macro(const Physics &p, const float *__restrict__ f,
                                                const float *__restrict__ psi, int x, int y) {
    const size_t pl = p.plane;
    const size_t i = (size_t)y * p.pitch + x;
    const double f0 = f[i], f1 = f[i + pl], f2 = f[i + 2 * pl], f3 = f[i + 3 * pl],
                 f4 = f[i + 4 * pl], f5 = f[i + 5 * pl], f6 = f[i + 6 * pl], f7 = f[i + 7 * pl],
                 f8 = f[i + 8 * pl];
    const double rho = density<double>(f0, f1, f2, f3, f4, f5, f6, f7, f8);
    const double jx = ((f1 - f3) + (f5 - f7)) + (f8 - f6);
    const double jy = ((f2 - f4) + (f5 - f7)) + (f6 - f8);
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
        const size_t i = (size_t)y * p.pitch + x, pl = p.plane;
        out[kStatsFields + threadIdx.x] =
            density<double>(f[i], f[i + pl], f[i + 2 * pl], f[i + 3 * pl], f[i + 4 * pl],
                            f[i + 5 * pl], f[i + 6 * pl], f[i + 7 * pl], f[i + 8 * pl]);
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

template <typename R>
StepConst<R> make_const(const Physics &p) {
    StepConst<R> c{};
    c.nx = p.nx;
    c.ny = p.ny;
    c.pitch = p.pitch;
    c.plane = p.plane;
    c.gA = (R)(-p.G * p.A / 2.0);
    c.gB = (R)(-p.G * (1.0 - p.A));
    c.omega = (R)(1.0 / p.tau);
    c.kguo = (R)(1.0 - 1.0 / (2.0 * p.tau));
    c.li = (R)(p.sigma / (p.tau - 0.5));
    c.li2 = (R)(2.0 * p.sigma);
    for (int k = 0; k < 9; ++k) {
        c.s[k] = (R)p.s[k];
        c.hs[k] = (R)(1.0 - p.s[k] / 2.0);
        c.lim[k] = (R)(1.0 / (1.0 / p.s[k] - 0.5));
    }
    return c;
}

dim3 row_grid(int nx, int ny, int block) {
    return dim3((unsigned)((nx + block - 1) / block), (unsigned)(ny < 65535 ? ny : 65535));
}

template <typename R>
hipError_t fused_dispatch(const Physics &p, int tx, int ty, const float *fin, const float *psi,
                          float *fout, hipStream_t s) {
    const StepConst<R> c = make_const<R>(p);
    const dim3 block(tx, ty);
    const dim3 grid((unsigned)((p.nx + tx - 1) / tx), (unsigned)((p.ny + ty - 1) / ty));
    const size_t lds = (size_t)(tx + 2) * (ty + 2) * sizeof(float);
    if (p.coll == BGK) {
        if (p.scheme == EDM)
            hipLaunchKernelGGL((fused_kernel<R, EDM, BGK>), grid, block, lds, s, fin, psi, fout, c);
        else if (p.scheme == GUO)
            hipLaunchKernelGGL((fused_kernel<R, GUO, BGK>), grid, block, lds, s, fin, psi, fout, c);
        else
            hipLaunchKernelGGL((fused_kernel<R, GUO_LI, BGK>), grid, block, lds, s, fin, psi, fout, c);
    } else {
        if (p.scheme == GUO)
            hipLaunchKernelGGL((fused_kernel<R, GUO, MRT>), grid, block, lds, s, fin, psi, fout, c);
        else
            hipLaunchKernelGGL((fused_kernel<R, GUO_LI, MRT>), grid, block, lds, s, fin, psi, fout, c);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_psi(const Physics &p, bool fp64, const float *f, float *psi, hipStream_t s) {
    const dim3 grid = row_grid(p.nx, p.ny, 256);
    const double two_over_G = 2.0 / p.G;
    if (fp64)
        hipLaunchKernelGGL(psi_kernel<double>, grid, dim3(256), 0, s, f, psi, p.nx, p.ny, p.pitch,
                           p.plane, p.b_quarter, p.RT, p.a, p.K, two_over_G);
    else
        hipLaunchKernelGGL(psi_kernel<float>, grid, dim3(256), 0, s, f, psi, p.nx, p.ny, p.pitch,
                           p.plane, (float)p.b_quarter, (float)p.RT, (float)p.a, (float)p.K,
                           (float)two_over_G);
    return hipGetLastError();
}

hipError_t launch_fused(const Physics &p, bool fp64, int tx, int ty, const float *fin,
                        const float *psi, float *fout, hipStream_t s) {
    return fp64 ? fused_dispatch<double>(p, tx, ty, fin, psi, fout, s)
                : fused_dispatch<float>(p, tx, ty, fin, psi, fout, s);
}

hipError_t launch_init(const Physics &p, const double *rho0, const double *u0, float *f,
                       hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, row_grid(p.nx, p.ny, 256), dim3(256), 0, s, rho0, u0, f,
                       p.nx, p.ny, p.pitch, p.plane);
    return hipGetLastError();
}

hipError_t launch_macro(const Physics &p, const float *f, const float *psi, double *rho,
                        double *u, hipStream_t s) {
    hipLaunchKernelGGL(macro_kernel, row_grid(p.nx, p.ny, 256), dim3(256), 0, s, p, f, psi, rho,
                       u);
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
