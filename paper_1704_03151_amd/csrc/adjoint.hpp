// Transposed linearisation of the steady residual, the preconditioner of the
// adjoint iteration and the wall-temperature sensitivities.  The state f,
// the records and every sum are double; the vectors of the Krylov iteration
// (its basis, the preconditioner's input and output) have the storage type
// VT, double or float, and are read into and formed in double.
//
// The steady state solves the microscopic residual of Steps 3-4 with the
// equilibrium of the state itself (Sec. II A):
//   r_ik(f) = (g_ik(W_i(f), q_i(f)) - f_ik) tau_i^-1(W_i(f)) - div_ik(f),
// div the transport term of Step 1 (UGKS interface flux, van Leer slopes,
// micro-slopes from the cell moments, time slope from the compatibility
// condition; first-order kinetic boundary fluxes, Sec. III B).  The kernels
// below form out = (dr/df)^T v by reverse accumulation through exactly that
// arithmetic, in four stages:
//   k_adj_cell   per cell: the collision term (reductions over k),
//   k_adj_face   per interior face: the interface flux (two passes over k,
//                reusing the forward interface records),
//   k_adj_wall   per wall side: the diffuse-wall density,
//   k_adj_gather / k_adj_assemble   per (k, cell): the per-velocity terms,
//                gathered from the faces of the cell and of its neighbours
//                (the limited slope of a cell reads both neighbours), so
//                nothing is scattered and no atomics are needed.
#pragma once

#include "kernels.hpp"

namespace miugks {

constexpr int NFA = 14;   // per face: W0bar[4], q0bar[2], Wbar of L[4], Wbar of R[4]
constexpr int NCA = 9;    // per cell: Wbar[4], qbar[2], U, V, 1/tau

// d(q1..q5)/dtau of time_coeffs on the same branches (x = dt/tau)
__device__ inline void time_coeffs_dtau(double dt, double tau, double* d) {
    double x = dt / tau;
    double em1 = -expm1(-x);
    double E = exp(-x);
    d[3] = em1 - E * x;
    if (x < 0.5) {
        double s1 = 0, s2 = 0, s3 = 0, s5 = 0, fact = 1.0, p2 = 1.0, p3 = 1.0;   // x^(m-2), x^(m-3)
        for (int m = 1; m <= 25; ++m) {
            fact *= m;
            double sg = (m & 1) ? -1.0 : 1.0;
            if (m >= 2) {
                s1 += sg * (m - 1) * p2 / fact;
                if (m >= 3) {
                    s2 += sg * (m - 2) * (m - 2) * p3 / fact;
                    s3 -= sg * (m - 2) * p3 / fact;
                    s5 += sg * (1 - m) * (m - 2) * p3 / fact;
                    p3 *= x;
                }
                p2 *= x;
            }
        }
        double dx = -x / tau;
        d[0] = dt * s1 * dx;
        d[1] = dt * dt * s2 * dx;
        d[2] = dt * dt * s3 * dx;
        d[4] = dt * dt * s5 * dx;
    } else {
        d[0] = -em1 + E * x;
        d[1] = 4.0 * tau * em1 - 2.0 * tau * E * x - dt - dt * E - dt * E * x;
        d[2] = -dt + 2.0 * tau * em1 - tau * E * x;
        d[4] = dt * E + dt * E * x - 2.0 * tau * em1 + tau * E * x;
    }
}

// reverse of micro_slope: adds the adjoints of b (bb), U, V, lam for the
// output adjoint ab
__device__ inline void micro_slope_rev(const double* b, double U, double V, double lam, double K, const double* ab,
                                       double* bb, double& Ub, double& Vb, double& lb) {
    double e = U * U + V * V + K / (2.0 * lam);
    double R2 = b[1] - U * b[0], R3 = b[2] - V * b[0], R4 = 2.0 * b[3] - e * b[0];
    double c4 = 4.0 * lam * lam / K;
    double X = R4 - 2.0 * U * R2 - 2.0 * V * R3;
    double a4 = c4 * X, a3 = 2.0 * lam * R3 - V * a4, a2 = 2.0 * lam * R2 - U * a4;
    double a1b = ab[0], a2b = ab[1], a3b = ab[2], a4b = ab[3], eb = 0.0;
    // a1 = b0 - U a2 - V a3 - a4 e / 2
    bb[0] += a1b;
    Ub -= a1b * a2;
    a2b -= a1b * U;
    Vb -= a1b * a3;
    a3b -= a1b * V;
    a4b -= 0.5 * a1b * e;
    eb -= 0.5 * a1b * a4;
    // a2 = 2 lam R2 - U a4, a3 = 2 lam R3 - V a4
    lb += 2.0 * (a2b * R2 + a3b * R3);
    double R2b = 2.0 * lam * a2b, R3b = 2.0 * lam * a3b;
    Ub -= a2b * a4;
    Vb -= a3b * a4;
    a4b -= a2b * U + a3b * V;
    // a4 = c4 X
    lb += a4b * (8.0 * lam / K) * X;
    double Xb = a4b * c4;
    Ub -= 2.0 * R2 * Xb;
    Vb -= 2.0 * R3 * Xb;
    R2b -= 2.0 * U * Xb;
    R3b -= 2.0 * V * Xb;
    double R4b = Xb;
    bb[3] += 2.0 * R4b;
    eb -= b[0] * R4b;
    bb[0] -= e * R4b + V * R3b + U * R2b;
    bb[2] += R3b;
    bb[1] += R2b;
    Vb -= b[0] * R3b;
    Ub -= b[0] * R2b;
    Ub += 2.0 * U * eb;
    Vb += 2.0 * V * eb;
    lb -= K / (2.0 * lam * lam) * eb;
}

// reverse of (rho, U, V, lam) = prim_of(W): W bar for the primitive adjoints
__device__ inline void prim_rev(const double* W, double K, double rb, double Ub, double Vb, double lb, double* Wb) {
    double rho = W[0], U = W[1] / rho, V = W[2] / rho;
    double e = W[3] - 0.5 * rho * (U * U + V * V);
    double lam = K * rho / (4.0 * e);
    Wb[0] += rb - (Ub * U + Vb * V) / rho + lb * (K / (4.0 * e) - lam / e * 0.5 * (U * U + V * V));
    Wb[1] += Ub / rho + lb * lam * U / e;
    Wb[2] += Vb / rho + lb * lam * V / e;
    Wb[3] -= lb * lam / e;
}

// one velocity's share of the reverse of the Shakhov pair (G, H) with output
// adjoints gb, hb: adds to acc = (rho, U, V, lam, qx, qy) bar; G0 is the
// Maxwellian rho (lam/pi) exp(-lam |c|^2) of this velocity
__device__ inline void shakhov_rev_k(double rho, double U, double V, double lam, double qx, double qy, double u,
                                     double v, int Ki, double s, double G0, double gb, double hb, double* acc) {
    double cx = u - U, cy = v - V, c2 = cx * cx + cy * cy;
    double H0 = (Ki / (2.0 * lam)) * G0;
    double F = s * lam * lam * (cx * qx + cy * qy) / rho;
    double PG = 1.0 + F * (2.0 * lam * c2 - 4.0), PH = 1.0 + F * (2.0 * lam * c2 - 2.0);
    double G0b = gb * PG + hb * PH * Ki / (2.0 * lam);
    double Fb = gb * G0 * (2.0 * lam * c2 - 4.0) + hb * H0 * (2.0 * lam * c2 - 2.0);
    double t = gb * G0 + hb * H0;
    double lb = t * F * 2.0 * c2 - hb * PH * G0 * Ki / (2.0 * lam * lam);
    double c2b = t * F * 2.0 * lam;
    double f1 = s * lam * lam / rho;
    double rb = -Fb * F / rho + G0b * G0 / rho;
    lb += Fb * 2.0 * F / lam + G0b * G0 * (1.0 / lam - c2);
    double cxb = Fb * f1 * qx + c2b * 2.0 * cx - G0b * G0 * 2.0 * lam * cx;
    double cyb = Fb * f1 * qy + c2b * 2.0 * cy - G0b * G0 * 2.0 * lam * cy;
    acc[0] += rb;
    acc[1] -= cxb;
    acc[2] -= cyb;
    acc[3] += lb;
    acc[4] += Fb * f1 * cx;
    acc[5] += Fb * f1 * cy;
}

// one velocity's share of the reverse of (Ga, Ha) = slope_poly(a) (G0, H0)
// with output adjoints Gb, Hb: adds to ab[4] and lb; returns the adjoints of
// G0 and H0 in g0b, h0b
__device__ inline void slope_rev_k(const double* a, double u, double v, double lam, int Ki, double G0, double H0,
                                   double Gb, double Hb, double* ab, double& lb, double& g0b, double& h0b) {
    double pG, pH;
    slope_poly<double>(a, u, v, lam, Ki, pG, pH);
    double tG = Gb * G0, tH = Hb * H0, t = tG + tH;
    ab[0] += t;
    ab[1] += t * u;
    ab[2] += t * v;
    ab[3] += 0.5 * t * (u * u + v * v) + (0.5 * Ki * tG + 0.5 * (Ki + 2.0) * tH) / (2.0 * lam);
    lb -= 0.5 * a[3] * (Ki * tG + (Ki + 2.0) * tH) / (2.0 * lam * lam);
    g0b = Gb * pG;
    h0b = Hb * pH;
}

// adjoints of (G0, H0) of one velocity folded into (rho, U, V, lam) bar,
// G0 = rho (lam/pi) exp(-lam |c|^2), H0 = K_int/(2 lam) G0
__device__ inline void g0_fold(double G0, double cx, double cy, double rho, double lam, int Ki, double g0b, double h0b,
                               double* acc) {
    double tot = (g0b + h0b * Ki / (2.0 * lam)) * G0;
    acc[0] += tot / rho;
    acc[1] += tot * 2.0 * lam * cx;
    acc[2] += tot * 2.0 * lam * cy;
    acc[3] += tot * (1.0 / lam - (cx * cx + cy * cy)) - h0b * G0 * Ki / (2.0 * lam * lam);
}

template <int M>
__device__ __forceinline__ void wave_allsum(double* a) {
#pragma unroll
    for (int m = 0; m < M; ++m)
        for (int off = 32; off > 0; off >>= 1) a[m] += __shfl_xor(a[m], off, 64);
}

// Collision term, one wavefront per cell: the adjoint moments Wbar (through
// g and tau), the heat-flux adjoint, U, V and 1/tau into rec[m nc + c]
template <typename VT>
__global__ void __launch_bounds__(256) k_adj_cell(Geo g, Vel vel, Gas gas, const double* __restrict__ f,
                                                   const double* __restrict__ W, const double* __restrict__ q,
                                                   const VT* __restrict__ v, double* __restrict__ rec) {
    int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= g.nc) return;
    const int nc = g.nc;
    if (g.solid[c]) {
        if (lane < NCA) rec[(size_t)lane * nc + c] = 0.0;
        return;
    }
    const size_t ho = (size_t)vel.nk * nc;
    double Wc[4] = {W[c], W[nc + c], W[2 * nc + c], W[3 * nc + c]};
    double rho, U, V, lam;
    prim_of(Wc, gas.K, rho, U, V, lam);
    const double qx = q[c], qy = q[nc + c];
    const double tinv = (rho / (2.0 * lam)) / mu_of(gas, 1.0 / lam);
    const double s = shakhov_prefactor(gas);
    const int Ki = gas.K_int;
    double acc[11] = {0};   // 0-5 shakhov (rho U V lam qx qy), 6 tau^-1 bar, 7 S0, 8 Sxx, 9 Syy, 10 Sxy
    for (int k = lane; k < vel.nk; k += 64) {
        double u = vel.u[k], vv = vel.v[k], w = vel.w[k];
        size_t i = (size_t)k * nc + c;
        double G = f[i], H = f[ho + i], vG = v[i], vH = v[ho + i];
        double cx = u - U, cy = vv - V, c2 = cx * cx + cy * cy;
        double G0 = rho * (lam / M_PI) * exp(-lam * c2), H0 = (Ki / (2.0 * lam)) * G0;
        double Fs = s * lam * lam * (cx * qx + cy * qy) / rho;
        double Gt = G0 * (1.0 + Fs * (2.0 * lam * c2 - 4.0)), Ht = H0 * (1.0 + Fs * (2.0 * lam * c2 - 2.0));
        acc[6] += vG * (Gt - G) + vH * (Ht - H);
        shakhov_rev_k(rho, U, V, lam, qx, qy, u, vv, Ki, s, G0, vG * tinv, vH * tinv, acc);
        acc[7] += w * (c2 * G + H);
        acc[8] += w * cx * cx * G;
        acc[9] += w * cy * cy * G;
        acc[10] += w * cx * cy * G;
    }
    wave_allsum<11>(acc);
    if (lane == 0) {
        double rb = acc[0] + acc[6] * tinv / rho;
        double lb = acc[3] + acc[6] * (gas.omega - 1.0) * tinv / lam;
        double qxb = acc[4], qyb = acc[5];
        double Ub = acc[1] + qxb * (-0.5 * acc[7] - acc[8]) - qyb * acc[10];
        double Vb = acc[2] - qxb * acc[10] + qyb * (-0.5 * acc[7] - acc[9]);
        double Wb[4] = {0, 0, 0, 0};
        prim_rev(Wc, gas.K, rb, Ub, Vb, lb, Wb);
        double out[NCA] = {Wb[0], Wb[1], Wb[2], Wb[3], qxb, qyb, U, V, tinv};
        for (int m = 0; m < NCA; ++m) rec[(size_t)m * nc + c] = out[m];
    }
}

// Interior faces, one wavefront per (direction d, cell c) = the face on side
// 2d of c (c is R, its neighbour L), reading the forward interface record of
// the face (Step 1 of the same f).  Two launches: PART 0 forms the 28 sums
// over the velocities of pass A into fsum[(m * 2 + d) nc + c]; PART 1 runs
// the scalar reverse chain, pass B and the final chain into
// fa[(m * 2 + d) nc + c], m < NFA (the split halves the registers live at once).
constexpr int NFS = 28;
template <int PART, typename VT>
__global__ void __launch_bounds__(256) k_adj_face(Geo g, Vel vel, Gas gas, const double* __restrict__ f,
                                                   const double* __restrict__ W, const double* __restrict__ fp,
                                                   const VT* __restrict__ v, double* __restrict__ fsum,
                                                   double* __restrict__ fa) {
    // the face is the same across the wavefront: its record, geometry and
    // scalars live in scalar registers
    int t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6)), lane = threadIdx.x & 63;
    if (t >= 2 * g.nc) return;
    const int nc = g.nc, d = t / nc, c = t - d * nc;
    const size_t stride = 2 * (size_t)nc;
    const double* rec = fp + (size_t)d * nc + c;
    double* out = fa + (size_t)d * nc + c;
    FaceGeom<double> fg;
    if (g.solid[c] || rec[23 * stride] == 0.0 || !face_geom<double>(g, c, d, fg)) {
        if (PART == 1 && lane < NFA) out[lane * stride] = 0.0;
        return;
    }
    const int L = fg.L, Ki = gas.K_int;
    const double K = gas.K, s = shakhov_prefactor(gas);
    const double rho0 = rec[0], U0 = rec[stride], V0 = rec[2 * stride], lam0 = rec[3 * stride];
    const double shq = s * lam0 * lam0 / rho0;
    const double q0x = shq != 0.0 ? rec[4 * stride] / shq : 0.0, q0y = shq != 0.0 ? rec[5 * stride] / shq : 0.0;
    double aL[4], aR[4], A[4];
    for (int m = 0; m < 4; ++m) {
        aL[m] = rec[(6 + m) * stride];
        aR[m] = rec[(10 + m) * stride];
        A[m] = rec[(14 + m) * stride];
    }
    const double dt = fmin(g.dt[L], g.dt[c]);
    double qc[5];
    for (int m = 0; m < 5; ++m) qc[m] = rec[(18 + m) * stride] * dt;
    const double tau0 = mu_of(gas, 1.0 / lam0) / (rho0 / (2.0 * lam0));
    const double cL = 0.5 / fg.dL, cR = 0.5 / fg.dR;   // S / V of the two cells
    const size_t ho = (size_t)vel.nk * nc;
    // pass A: q1..q5 bar, Shakhov, time slope, G0 folds, compatibility sums,
    // heat-flux sums, in two loops over the velocities (fewer live values)
    double a[NFS] = {0};
    // 0-4 qbar, 5-10 shakhov, 11-14 Abar, 15 lam (A), 16-19 G0 fold, 20-23 Mb, 24 S0 25 Sxx 26 Syy 27 Sxy
    double* sums = fsum + (size_t)d * nc + c;
    if constexpr (PART == 1) {
        for (int m = 0; m < NFS; ++m) a[m] = sums[m * stride];
    } else {
#pragma unroll 1
    for (int k = lane; k < vel.nk; k += 64) {   // A1: needs the interface values
        double u = vel.u[k], vv = vel.v[k], w = vel.w[k], un = d == 0 ? u : vv;
        size_t kc = (size_t)k * nc;
        double Gup, Hup, sGup, sHup;
        face_upwind_k<double, double>(fg, c, f, ho, kc, un, Gup, Hup, sGup, sHup);
        double phG = (-v[kc + L] * cL + v[kc + c] * cR) * un / dt;
        double phH = (-v[ho + kc + L] * cL + v[ho + kc + c] * cR) * un / dt;
        double cx = u - U0, cy = vv - V0, c2 = cx * cx + cy * cy;
        double G0 = rho0 * (lam0 / M_PI) * exp(-lam0 * c2), H0 = (Ki / (2.0 * lam0)) * G0;
        double Fs = s * lam0 * lam0 * (cx * q0x + cy * q0y) / rho0;
        double Geq = G0 * (1.0 + Fs * (2.0 * lam0 * c2 - 4.0)), Heq = H0 * (1.0 + Fs * (2.0 * lam0 * c2 - 2.0));
        double pGL, pHL, pGR, pHR, pGA, pHA;
        slope_poly<double>(aL, u, vv, lam0, Ki, pGL, pHL);
        slope_poly<double>(aR, u, vv, lam0, Ki, pGR, pHR);
        slope_poly<double>(A, u, vv, lam0, Ki, pGA, pHA);
        double hL = un > 0.0 ? 1.0 : (un < 0.0 ? 0.0 : 0.5), hR = 1.0 - hL;
        double Gs = (hL * pGL + hR * pGR) * G0, Hs = (hL * pHL + hR * pHR) * H0;
        a[0] += phG * Geq + phH * Heq;
        a[1] += un * (phG * Gs + phH * Hs);
        a[2] += phG * pGA * G0 + phH * pHA * H0;
        a[3] += phG * Gup + phH * Hup;
        a[4] += un * (phG * sGup + phH * sHup);
        a[20] += w * un * Gs;
        a[21] += w * un * u * Gs;
        a[22] += w * un * vv * Gs;
        a[23] += w * un * 0.5 * ((u * u + vv * vv) * Gs + Hs);
        a[24] += w * (c2 * Gup + Hup);
        a[25] += w * cx * cx * Gup;
        a[26] += w * cy * cy * Gup;
        a[27] += w * cx * cy * Gup;
    }
#pragma unroll 1
    for (int k = lane; k < vel.nk; k += 64) {   // A2: the equilibrium and time-slope reverses
        double u = vel.u[k], vv = vel.v[k], un = d == 0 ? u : vv;
        size_t kc = (size_t)k * nc;
        double phG = (-v[kc + L] * cL + v[kc + c] * cR) * un / dt;
        double phH = (-v[ho + kc + L] * cL + v[ho + kc + c] * cR) * un / dt;
        double cx = u - U0, cy = vv - V0, c2 = cx * cx + cy * cy;
        double G0 = rho0 * (lam0 / M_PI) * exp(-lam0 * c2), H0 = (Ki / (2.0 * lam0)) * G0;
        shakhov_rev_k(rho0, U0, V0, lam0, q0x, q0y, u, vv, Ki, s, G0, qc[0] * phG, qc[0] * phH, a + 5);
        double g0b, h0b;
        slope_rev_k(A, u, vv, lam0, Ki, G0, H0, qc[2] * phG, qc[2] * phH, a + 11, a[15], g0b, h0b);
        g0_fold(G0, cx, cy, rho0, lam0, Ki, g0b, h0b, a + 16);
    }
    wave_allsum<NFS>(a);
    if (lane == 0)
        for (int m = 0; m < NFS; ++m) sums[m * stride] = a[m];
    return;
    }
    double rho0b = a[16], U0b = a[17], V0b = a[18], lam0b = a[15] + a[19];
    rho0b += a[5];
    U0b += a[6];
    V0b += a[7];
    lam0b += a[8];
    const double q0xb = a[9], q0yb = a[10];
    // time slope: A = micro_slope(b), b = -Mb / rho0
    double b[4], bb[4] = {0, 0, 0, 0};
    for (int m = 0; m < 4; ++m) b[m] = -a[20 + m] / rho0;
    micro_slope_rev(b, U0, V0, lam0, K, a + 11, bb, U0b, V0b, lam0b);
    double Mbb[4];
    for (int m = 0; m < 4; ++m) {
        rho0b -= bb[m] * b[m] / rho0;
        Mbb[m] = -bb[m] / rho0;
    }
    // pass B: the spatial micro-slopes through Gs
    double e[13] = {0};   // 0-3 aL bar, 4-7 aR bar, 8 lam, 9-12 G0 fold
#pragma unroll 1
    for (int k = lane; k < vel.nk; k += 64) {
        double u = vel.u[k], vv = vel.v[k], w = vel.w[k], un = d == 0 ? u : vv;
        size_t kc = (size_t)k * nc;
        double phG = (-v[kc + L] * cL + v[kc + c] * cR) * un / dt;
        double phH = (-v[ho + kc + L] * cL + v[ho + kc + c] * cR) * un / dt;
        double cx = u - U0, cy = vv - V0, c2 = cx * cx + cy * cy;
        double G0 = rho0 * (lam0 / M_PI) * exp(-lam0 * c2), H0 = (Ki / (2.0 * lam0)) * G0;
        double Gsb = qc[1] * un * phG + w * un * (Mbb[0] + Mbb[1] * u + Mbb[2] * vv + 0.5 * Mbb[3] * (u * u + vv * vv));
        double Hsb = qc[1] * un * phH + w * un * 0.5 * Mbb[3];
        double hL = un > 0.0 ? 1.0 : (un < 0.0 ? 0.0 : 0.5), hR = 1.0 - hL;
        double g0b, h0b;
        slope_rev_k(aL, u, vv, lam0, Ki, G0, H0, hL * Gsb, hL * Hsb, e, e[8], g0b, h0b);
        g0_fold(G0, cx, cy, rho0, lam0, Ki, g0b, h0b, e + 9);
        slope_rev_k(aR, u, vv, lam0, Ki, G0, H0, hR * Gsb, hR * Hsb, e + 4, e[8], g0b, h0b);
        g0_fold(G0, cx, cy, rho0, lam0, Ki, g0b, h0b, e + 9);
    }
    wave_allsum<13>(e);
    rho0b += e[9];
    U0b += e[10];
    V0b += e[11];
    lam0b += e[8] + e[12];
    // spatial micro-slopes: aL = micro_slope((W0 - W_L)/(dL rho0)), aR = micro_slope((W_R - W0)/(dR rho0))
    double W0[4];
    cons_of(rho0, U0, V0, lam0, K, W0);
    double bL[4], bR[4], bLb[4] = {0, 0, 0, 0}, bRb[4] = {0, 0, 0, 0};
    for (int m = 0; m < 4; ++m) {
        bL[m] = (W0[m] - W[m * nc + L]) / fg.dL / rho0;
        bR[m] = (W[m * nc + c] - W0[m]) / fg.dR / rho0;
    }
    micro_slope_rev(bL, U0, V0, lam0, K, e, bLb, U0b, V0b, lam0b);
    micro_slope_rev(bR, U0, V0, lam0, K, e + 4, bRb, U0b, V0b, lam0b);
    double W0b[4], WLb[4], WRb[4];
    for (int m = 0; m < 4; ++m) {
        rho0b -= (bLb[m] * bL[m] + bRb[m] * bR[m]) / rho0;
        double tL = bLb[m] / (fg.dL * rho0), tR = bRb[m] / (fg.dR * rho0);
        W0b[m] = tL - tR;
        WLb[m] = -tL;
        WRb[m] = tR;
    }
    // time coefficients through tau0
    double dq[5];
    time_coeffs_dtau(dt, tau0, dq);
    double taub = 0.0;
    for (int m = 0; m < 5; ++m) taub += a[m] * dq[m];
    rho0b -= taub * tau0 / rho0;
    lam0b += taub * (1.0 - gas.omega) * tau0 / lam0;
    // heat flux of the interface distribution (about U0, V0)
    U0b += q0xb * (-0.5 * a[24] - a[25]) - q0yb * a[27];
    V0b += -q0xb * a[27] + q0yb * (-0.5 * a[24] - a[26]);
    prim_rev(W0, K, rho0b, U0b, V0b, lam0b, W0b);
    if (lane == 0) {
        double vals[NFA] = {W0b[0], W0b[1], W0b[2], W0b[3], q0xb, q0yb, WLb[0], WLb[1], WLb[2], WLb[3],
                            WRb[0], WRb[1], WRb[2], WRb[3]};
        for (int m = 0; m < NFA; ++m) out[m * stride] = vals[m];
    }
}

// Diffuse walls, one wavefront per wall side: the adjoint of the wall density
// divided by its denominator, rws[j] = (sum_{u_n<0} (Phibar^G u_n C^G +
// Phibar^H u_n C^H)) / den_j with Phibar = -v S/V of the wall's cell
template <typename VT>
__global__ void __launch_bounds__(256) k_adj_wall(Geo g, Vel vel, int K_int, const VT* __restrict__ v,
                                                   double* __restrict__ rws) {
    int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= g.n_wall) return;
    const int c = g.w_cell[j], sd = g.w_side[j], nc = g.nc;
    const size_t ho = (size_t)vel.nk * nc;
    const double sign = (sd & 1) ? 1.0 : -1.0;
    const double cb = 1.0 / (sd < 2 ? g.dx[c % g.nx] : g.dy[c / g.nx]);
    const double lam = 1.0 / g.w_T[j], Uw = g.w_U[j], Vw = g.w_V[j];
    double s = 0.0;
    for (int k = lane; k < vel.nk; k += 64) {
        double u = vel.u[k], vv = vel.v[k];
        double un = sign * (sd < 2 ? u : vv);
        if (un < 0.0) {
            double du = u - Uw, dv = vv - Vw;
            double CG = (lam / M_PI) * exp(-lam * (du * du + dv * dv)), CH = (K_int / (2.0 * lam)) * CG;
            size_t i = (size_t)k * nc + c;
            s += -cb * un * (v[i] * CG + v[ho + i] * CH);
        }
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) rws[j] = s / g.w_den[j];
}

// Per (k, cell), first part: the direct adjoints of the cell's values from
// the interface values of its faces (gbd, 2 planes) and the adjoints of the
// cell's limited slopes (sb[(2 d + plane) Nk nc + k nc + c]).
template <typename VT>
__global__ void __launch_bounds__(256) k_adj_gather(Geo g, Vel vel, const double* __restrict__ fp,
                                                     const double* __restrict__ fa, const VT* __restrict__ v,
                                                     double* __restrict__ gbd, double* __restrict__ sb) {
    const int nc = g.nc;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)vel.nk * nc;
    if (i >= n) return;
    const int k = (int)(i / nc), c = (int)(i - (size_t)k * nc);
    const size_t stride = 2 * (size_t)nc;
    double dG = 0.0, dH = 0.0, s4[4] = {0, 0, 0, 0};
    if (!g.solid[c]) {
        const double u = vel.u[k], vv = vel.v[k], w = vel.w[k];
        for (int d = 0; d < 2; ++d) {
            const double un = d == 0 ? u : vv;
            const double hL = un > 0.0 ? 1.0 : (un < 0.0 ? 0.0 : 0.5), hR = 1.0 - hL;
            for (int side = 0; side < 2; ++side) {
                // side 0: the face on side 2d of c (c is R); side 1: on side 2d+1 (c is L)
                int cr = side == 0 ? c : g.nb[(2 * d + 1) * nc + c];
                if (cr < 0) continue;
                const double* rec = fp + (size_t)d * nc + cr;
                if (rec[23 * stride] == 0.0) continue;
                int cl = g.nb[(2 * d) * nc + cr];
                const double* ad = fa + (size_t)d * nc + cr;
                double dL = 0.5 * (d == 0 ? g.dx[cl % g.nx] : g.dy[cl / g.nx]);
                double dR = 0.5 * (d == 0 ? g.dx[cr % g.nx] : g.dy[cr / g.nx]);
                double dt = fmin(g.dt[cl], g.dt[cr]);
                double q4 = rec[21 * stride] * dt, q5 = rec[22 * stride] * dt;
                double U0 = rec[stride], V0 = rec[2 * stride];
                size_t kc = (size_t)k * nc;
                double phG = (-v[kc + cl] * (0.5 / dL) + v[kc + cr] * (0.5 / dR)) * un / dt;
                double phH = (-v[n + kc + cl] * (0.5 / dL) + v[n + kc + cr] * (0.5 / dR)) * un / dt;
                double cx = u - U0, cy = vv - V0, c2 = cx * cx + cy * cy;
                double qd = ad[4 * stride] * cx + ad[5 * stride] * cy;
                double W3 = ad[3 * stride];
                double Gupb = q4 * phG + w * (ad[0] + ad[stride] * u + ad[2 * stride] * vv + 0.5 * W3 * (u * u + vv * vv)) +
                              0.5 * w * qd * c2;
                double Hupb = q4 * phH + 0.5 * w * W3 + 0.5 * w * qd;
                double sGupb = q5 * un * phG, sHupb = q5 * un * phH;
                if (side == 1) {   // c is L
                    dG += hL * Gupb;
                    dH += hL * Hupb;
                    s4[2 * d] += hL * (dL * Gupb + sGupb);
                    s4[2 * d + 1] += hL * (dL * Hupb + sHupb);
                } else {           // c is R
                    dG += hR * Gupb;
                    dH += hR * Hupb;
                    s4[2 * d] += hR * (-dR * Gupb + sGupb);
                    s4[2 * d + 1] += hR * (-dR * Hupb + sHupb);
                }
            }
        }
    }
    gbd[i] = dG;
    gbd[n + i] = dH;
    for (int m = 0; m < 4; ++m) sb[(size_t)m * n + i] = s4[m];
}

// partial derivatives of the van Leer limiter on the branch the forward
// limiter takes (a b > 0): 2 b^2/(a+b)^2 and 2 a^2/(a+b)^2, written through
// t = a/(a+b) in (0, 1) so that tiny one-sided slopes cannot overflow
__device__ __forceinline__ void vl_partials(double a, double b, double& da, double& db) {
    double s = a * b;
    if (s > 0.0) {
        double t = a / (a + b);
        da = 2.0 * (1.0 - t) * (1.0 - t);
        db = 2.0 * t * t;
    } else {
        da = db = 0.0;
    }
}

// adjoint of F_c (one plane) through the limited slopes along direction d of
// c and of its two neighbours (each slope reads its cell and both neighbours)
__device__ inline double slope_adjoint(const Geo& g, int d, int c, const double* __restrict__ F, size_t kc,
                                       const double* __restrict__ sbp) {
    const int nc = g.nc;
    int lo = g.nb[(2 * d) * nc + c], hi = g.nb[(2 * d + 1) * nc + c];
    double Fc = F[kc + c], r = 0.0;
    double dlo = lo >= 0 ? g.dcent[(2 * d) * nc + c] : 1.0, dhi = hi >= 0 ? g.dcent[(2 * d + 1) * nc + c] : 1.0;
    double am = lo >= 0 ? (Fc - F[kc + lo]) / dlo : 0.0, ap = hi >= 0 ? (F[kc + hi] - Fc) / dhi : 0.0;
    double da, db;
    vl_partials(am, ap, da, db);
    double own = sbp[kc + c];
    if (lo >= 0) r += own * da / dlo;
    if (hi >= 0) r -= own * db / dhi;
    if (lo >= 0) {   // slope of lo: (F_lo - F_lolo)/d, (F_c - F_lo)/dlo
        int ll = g.nb[(2 * d) * nc + lo];
        double dl2 = ll >= 0 ? g.dcent[(2 * d) * nc + lo] : 1.0;
        double a2 = ll >= 0 ? (F[kc + lo] - F[kc + ll]) / dl2 : 0.0;
        vl_partials(a2, am, da, db);
        r += sbp[kc + lo] * db / dlo;
    }
    if (hi >= 0) {   // slope of hi: (F_hi - F_c)/dhi, (F_hihi - F_hi)/d
        int hh = g.nb[(2 * d + 1) * nc + hi];
        double dh2 = hh >= 0 ? g.dcent[(2 * d + 1) * nc + hi] : 1.0;
        double b2 = hh >= 0 ? (F[kc + hh] - F[kc + hi]) / dh2 : 0.0;
        vl_partials(ap, b2, da, db);
        r -= sbp[kc + hi] * da / dhi;
    }
    return r;
}

// Per (k, cell), second part: out = (dr/df)^T v for both planes
template <typename VT>
__global__ void __launch_bounds__(256) k_adj_assemble(Geo g, Vel vel, const double* __restrict__ f,
                                                       const VT* __restrict__ v, const double* __restrict__ crec,
                                                       const double* __restrict__ fa, const double* __restrict__ rws,
                                                       const double* __restrict__ gbd, const double* __restrict__ sb,
                                                       VT* __restrict__ out) {
    const int nc = g.nc;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)vel.nk * nc;
    if (i >= n) return;
    const int k = (int)(i / nc), c = (int)(i - (size_t)k * nc);
    if (g.solid[c]) {
        out[i] = VT(0);
        out[n + i] = VT(0);
        return;
    }
    const size_t stride = 2 * (size_t)nc, kc = (size_t)k * nc;
    const double u = vel.u[k], vv = vel.v[k], w = vel.w[k];
    const double vG = v[i], vH = v[n + i];
    double oG = gbd[i], oH = gbd[n + i];
    for (int d = 0; d < 2; ++d) {
        oG += slope_adjoint(g, d, c, f, kc, sb + (size_t)(2 * d) * n);
        oH += slope_adjoint(g, d, c, f + n, kc, sb + (size_t)(2 * d + 1) * n);
    }
    // collision
    double Wb[4];
    for (int m = 0; m < 4; ++m) Wb[m] = crec[(size_t)m * nc + c];
    double qxb = crec[4 * (size_t)nc + c], qyb = crec[5 * (size_t)nc + c];
    double U = crec[6 * (size_t)nc + c], V = crec[7 * (size_t)nc + c], tinv = crec[8 * (size_t)nc + c];
    double cx = u - U, cy = vv - V, qd = qxb * cx + qyb * cy;
    oG += -vG * tinv + 0.5 * w * qd * (cx * cx + cy * cy);
    oH += -vH * tinv + 0.5 * w * qd;
    // the cell's moments also feed the micro-slopes of its faces
    for (int d = 0; d < 2; ++d) {
        const double* aR = fa + (size_t)d * nc + c;   // c is R of its own face (zero record if none)
        for (int m = 0; m < 4; ++m) Wb[m] += aR[(10 + m) * stride];
        int hi = g.nb[(2 * d + 1) * nc + c];
        if (hi >= 0) {
            const double* aL = fa + (size_t)d * nc + hi;   // c is L of hi's face
            for (int m = 0; m < 4; ++m) Wb[m] += aL[(6 + m) * stride];
        }
    }
    oG += w * (Wb[0] + Wb[1] * u + Wb[2] * vv + 0.5 * Wb[3] * (u * u + vv * vv));
    oH += 0.5 * w * Wb[3];
    // boundary sides
    for (int s = 0; s < 4; ++s) {
        int code = g.nb[s * nc + c];
        if (code >= 0 || code == NB_NONE) continue;
        double sign = (s & 1) ? 1.0 : -1.0;
        double un = sign * (s < 2 ? u : vv);
        double cb = 1.0 / (s < 2 ? g.dx[c % g.nx] : g.dy[c / g.nx]);
        double pG = -vG * cb, pH = -vH * cb;
        if (is_wall(code)) {
            if (un > 0.0) {
                oG += pG * un - w * un * rws[wall_of(code)];
                oH += pH * un;
            }
        } else if (code == NB_FARFIELD) {
            if (un > 0.0) {
                oG += pG * un;
                oH += pH * un;
            }
        } else if (code == NB_OUTFLOW) {
            oG += pG * un;
            oH += pH * un;
        } else if (code == NB_SYMMETRY) {
            // the outgoing value is also the incoming ghost of the mirror velocity
            // (whose normal speed is -u_n)
            if (un > 0.0) {
                size_t im = (size_t)mirror_of(vel, s >> 1, k) * nc + c;
                oG += pG * un + v[im] * cb * un;
                oH += pH * un + v[n + im] * cb * un;
            }
        }
    }
    out[i] = VT(oG);
    out[n + i] = VT(oH);
}

// Preconditioner of the adjoint iteration: y = A^-T r for the velocity-
// diagonal part of the correction operator A of Step 5 (Sec. II A 2: the
// diagonal 1/tau + sum of outgoing u_n S/V, the upwind neighbours off the
// diagonal, outflow ghosts on the diagonal; the wall coupling across
// velocities left out).  A is lower triangular in each velocity's upwind
// order, so A^T is solved by one sweep in the reverse (downwind-first)
// order: y_c = (r_c + sum over downwind neighbours d of u_n y_d / h_d) / D_c.
// One block per velocity, one thread per row, anti-diagonal wavefronts; both
// planes share the operator.  Requires ny <= blockDim.x.
template <typename VT>
__global__ void k_adj_sweep(Geo g, Vel vel, const double* __restrict__ crec, const VT* __restrict__ r,
                            VT* __restrict__ y) {
    extern __shared__ double lds[];   // [2][ny]: the last value of each row
    const int k = blockIdx.x, j = threadIdx.x, nx = g.nx, ny = g.ny, nc = g.nc;
    const size_t n = (size_t)vel.nk * nc, kc = (size_t)k * nc;
    const double u = vel.u[k], v = vel.v[k];
    const bool row = j < ny;
    const int jr = v > 0.0 ? ny - 1 - j : j;   // rank of the row in the processing order
    const int jd = v > 0.0 ? j + 1 : j - 1;    // the row downwind in y
    double xg = 0.0, xh = 0.0;                  // y of the x-downwind neighbour (previous step)
    if (row) {
        lds[j] = 0.0;
        lds[ny + j] = 0.0;
    }
    __syncthreads();
    for (int t = 0; t < nx + ny - 1; ++t) {
        int ir = t - jr;
        bool act = row && ir >= 0 && ir < nx;
        double yg = 0.0, yh = 0.0;
        if (act) {
            int i = u > 0.0 ? nx - 1 - ir : ir;
            int c = j * nx + i;
            if (!g.solid[c]) {
                double D = crec[8 * (size_t)nc + c], sg = r[kc + c], sh = r[n + kc + c];
                for (int s = 0; s < 4; ++s) {
                    double un = ((s & 1) ? 1.0 : -1.0) * (s < 2 ? u : v);
                    double h = s < 2 ? g.dx[i] : g.dy[j];
                    int code = g.nb[s * nc + c];
                    if (un > 0.0) {
                        D += un / h;
                        if (code >= 0) {   // downwind neighbour: the row's previous value in x, the lds row in y
                            if (s < 2) {
                                double hd = g.dx[code % nx];
                                sg += un * xg / hd;
                                sh += un * xh / hd;
                            } else {   // code >= 0 across a y side: the row jd exists (0 <= jd < ny)
                                double hd = g.dy[code / nx];
                                sg += un * lds[jd] / hd;
                                sh += un * lds[ny + jd] / hd;
                            }
                        }
                    } else if (un < 0.0 && code == NB_OUTFLOW) {
                        D += un / h;
                    }
                }
                yg = sg / D;
                yh = sh / D;
            }
            y[kc + c] = VT(yg);
            y[n + kc + c] = VT(yh);
        }
        __syncthreads();
        if (act) {
            lds[j] = yg;
            lds[ny + j] = yh;
            xg = yg;
            xh = yh;
        }
        __syncthreads();
    }
}

// load weights of one velocity at a wall side (wall frame): L^G, L^H
__device__ __forceinline__ void load_weights(int kind, int sd, double cx, double cy, double& LG, double& LH) {
    double cn = ((sd & 1) ? 1.0 : -1.0) * (sd < 2 ? cx : cy), ct = sd < 2 ? cy : cx;
    if (kind == 0) {
        LG = cn * cn;
        LH = 0.0;
    } else if (kind == 1) {
        LG = ct * cn;
        LH = 0.0;
    } else {
        LG = 0.5 * cn * (cx * cx + cy * cy);
        LH = 0.5 * cn;
    }
}

// Per wall side of the objective: Q_j = sum over incoming velocities of
// w (L^G C^G + L^H C^H) (the objective's share of the wall Maxwellian) and
// the wall density rho_w; one wavefront per wall side
__global__ void __launch_bounds__(256) k_adj_objwall(Geo g, Vel vel, int K_int, int kind,
                                                      const double* __restrict__ f, double* __restrict__ Qj,
                                                      double* __restrict__ rhow) {
    int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= g.n_wall) return;
    const int c = g.w_cell[j], sd = g.w_side[j];
    const double sign = (sd & 1) ? 1.0 : -1.0;
    const double lam = 1.0 / g.w_T[j], Uw = g.w_U[j], Vw = g.w_V[j];
    double q = 0.0, m = 0.0;
    for (int k = lane; k < vel.nk; k += 64) {
        double u = vel.u[k], vv = vel.v[k], w = vel.w[k];
        double un = sign * (sd < 2 ? u : vv);
        if (un > 0.0) {
            m += w * un * f[(size_t)k * g.nc + c];
        } else if (un < 0.0) {
            double cx = u - Uw, cy = vv - Vw;
            double CG = (lam / M_PI) * exp(-lam * (cx * cx + cy * cy)), CH = (K_int / (2.0 * lam)) * CG;
            double LG, LH;
            load_weights(kind, sd, cx, cy, LG, LH);
            q += w * (LG * CG + LH * CH);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        q += __shfl_xor(q, off, 64);
        m += __shfl_xor(m, off, 64);
    }
    if (lane == 0) {
        Qj[j] = q;
        rhow[j] = -m / g.w_den[j];
    }
}

// b = dJ/df - mu m per (k, cell): J = sum over weighted wall sides of
// S_j sum_k w (L^G f^G + L^H f^H) on the wall side of the face, whose
// incoming part rho_w C depends on the cell's outgoing G through rho_w;
// m = the mass row (w_k V_c on G)
__global__ void __launch_bounds__(256) k_adj_objgrad(Geo g, Vel vel, int kind, const double* __restrict__ objw,
                                                      const double* __restrict__ Qj, double mu,
                                                      double* __restrict__ b) {
    const int nc = g.nc;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)vel.nk * nc;
    if (i >= n) return;
    const int k = (int)(i / nc), c = (int)(i - (size_t)k * nc);
    double bG = 0.0, bH = 0.0;
    if (!g.solid[c]) {
        const double u = vel.u[k], vv = vel.v[k], w = vel.w[k];
        const double dx = g.dx[c % g.nx], dy = g.dy[c / g.nx];
        for (int s = 0; s < 4; ++s) {
            int code = g.nb[s * nc + c];
            if (!is_wall(code)) continue;
            int j = wall_of(code);
            double wt = objw[j];
            if (wt == 0.0) continue;
            double un = ((s & 1) ? 1.0 : -1.0) * (s < 2 ? u : vv);
            if (!(un > 0.0)) continue;
            double S = s < 2 ? dy : dx;
            double LG, LH;
            load_weights(kind, s, u - g.w_U[j], vv - g.w_V[j], LG, LH);
            bG += wt * S * (w * LG - Qj[j] * w * un / g.w_den[j]);
            bH += wt * S * w * LH;
        }
        bG -= mu * w * dx * dy;
    }
    b[i] = bG;
    b[n + i] = bH;
}

// dJ/dT_w - lam^T dr/dT_w for each listed wall side (one wavefront each):
// the wall temperature enters through the wall Maxwellian of the incoming
// velocities and its density rho_w (zero net mass flux; Sec. III B)
template <typename VT>
__global__ void __launch_bounds__(256) k_adj_paramgrad(Geo g, Vel vel, int K_int, int kind,
                                                        const double* __restrict__ objw,
                                                        const double* __restrict__ Qj,
                                                        const double* __restrict__ rhow,
                                                        const VT* __restrict__ lam_adj,
                                                        const int* __restrict__ sides, int n_sides,
                                                        double* __restrict__ out) {
    int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= n_sides) return;
    const int j = sides[t], c = g.w_cell[j], sd = g.w_side[j], nc = g.nc;
    const size_t n = (size_t)vel.nk * nc;
    const double sign = (sd & 1) ? 1.0 : -1.0;
    const double lam = 1.0 / g.w_T[j], Uw = g.w_U[j], Vw = g.w_V[j];
    const double cb = 1.0 / (sd < 2 ? g.dx[c % g.nx] : g.dy[c / g.nx]);
    const double rw = rhow[j], den = g.w_den[j];
    // pass 1: d(den)/d(lam_w) and dQ/d(lam_w)
    double dden = 0.0, dQ = 0.0;
    for (int k = lane; k < vel.nk; k += 64) {
        double u = vel.u[k], vv = vel.v[k], w = vel.w[k];
        double un = sign * (sd < 2 ? u : vv);
        if (un < 0.0) {
            double cx = u - Uw, cy = vv - Vw, c2 = cx * cx + cy * cy;
            double CG = (lam / M_PI) * exp(-lam * c2), CH = (K_int / (2.0 * lam)) * CG;
            double dCG = CG * (1.0 / lam - c2), dCH = -CH * c2;
            dden += w * un * dCG;
            double LG, LH;
            load_weights(kind, sd, cx, cy, LG, LH);
            dQ += w * (LG * dCG + LH * dCH);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        dden += __shfl_xor(dden, off, 64);
        dQ += __shfl_xor(dQ, off, 64);
    }
    const double drw = -rw / den * dden;
    // pass 2: lam^T dr/d(lam_w), r = ... - cb u_n rho_w C on the incoming velocities
    double s = 0.0;
    for (int k = lane; k < vel.nk; k += 64) {
        double u = vel.u[k], vv = vel.v[k];
        double un = sign * (sd < 2 ? u : vv);
        if (un < 0.0) {
            double cx = u - Uw, cy = vv - Vw, c2 = cx * cx + cy * cy;
            double CG = (lam / M_PI) * exp(-lam * c2), CH = (K_int / (2.0 * lam)) * CG;
            double dCG = CG * (1.0 / lam - c2), dCH = -CH * c2;
            size_t i = (size_t)k * nc + c;
            s += -cb * un * (lam_adj[i] * (drw * CG + rw * dCG) + lam_adj[n + i] * (drw * CH + rw * dCH));
        }
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        double S = sd < 2 ? g.dy[c / g.nx] : g.dx[c % g.nx];
        double dJ = objw[j] != 0.0 ? objw[j] * S * (drw * Qj[j] + rw * dQ) : 0.0;
        // d/dT = -lam^2 d/dlam
        out[t] = -lam * lam * (dJ - s);
    }
}

// x = a - b elementwise; per-block sums of x^2 (fixed order, of the double
// difference) into part
template <typename VT>
__global__ void __launch_bounds__(256) k_adj_residual(const double* __restrict__ a, const double* __restrict__ b,
                                                       VT* __restrict__ x, size_t n, double* __restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        double d = a[i] - b[i];
        x[i] = VT(d);
        s += d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Krylov support: per-block partial dot products of w with the vectors
// V[i ldv ...], i < m, into part[i gridDim.x + block] (fixed order); and
// w += sign sum_i h[i] V[i]
// (eight vectors per pass over w; products and sums in double)
template <typename VT>
__global__ void __launch_bounds__(256) k_adj_dots(const VT* __restrict__ w, const VT* __restrict__ V,
                                                   size_t ldv, int m, size_t n, double* __restrict__ part) {
    __shared__ double sh[8][256];
    for (int i0 = 0; i0 < m; i0 += 8) {
        const int nv = m - i0 < 8 ? m - i0 : 8;
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (size_t)gridDim.x * 256) {
            double x = w[j];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (u < nv) s[u] += x * V[(size_t)(i0 + u) * ldv + j];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) sh[u][threadIdx.x] = s[u];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o)
#pragma unroll
                for (int u = 0; u < 8; ++u) sh[u][threadIdx.x] += sh[u][threadIdx.x + o];
            __syncthreads();
        }
        if ((int)threadIdx.x < nv) part[(size_t)(i0 + threadIdx.x) * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
        __syncthreads();
    }
}

template <typename VT>
__global__ void k_adj_lincomb(VT* __restrict__ w, const VT* __restrict__ V, size_t ldv,
                              const double* __restrict__ h, int m, double sign, size_t n) {
    size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += h[i] * double(V[(size_t)i * ldv + j]);
    w[j] = VT(double(w[j]) + sign * s);
}

template <typename VT>
__global__ void k_adj_scale(VT* __restrict__ y, const VT* __restrict__ x, double a, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = VT(a * double(x[i]));
}

template <typename TX, typename TY>
__global__ void k_adj_axpy(TX* __restrict__ x, const TY* __restrict__ y, double a, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = TX(double(x[i]) + a * double(y[i]));
}

}  // namespace miugks
