// HIP kernels of the MIUGKS hot path for gfx950 (templated on the storage /
// arithmetic type T of the distribution: double, or float for the FP32-f
// form in which moments, macroscopic prediction and norms stay double).
//
// Data layout (HBM): distributions are [2][Nk][nc] (G plane, H plane,
// velocity-major, cells fastest), so a wavefront of 64 lanes covers 64
// consecutive cells of one velocity and every access coalesces.  Per-cell
// macroscopic arrays are [m][nc] doubles.
//
// Most per-(cell, velocity) kernels use one launch shape: a block of 256
// threads = 64 lanes (consecutive cells) x 4 waves, the waves taking
// interleaved velocities of a chunk (KCH = 4 * MK velocities, or a multiple
// of it for the reductions, or 4 * MKF for the flux); reductions over the
// velocities are written as per-chunk partial sums that a finalize kernel
// adds in a fixed order (deterministic, no floating-point atomics).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "setup.hpp"

namespace miugks {

constexpr int TILE = 64;
constexpr int WAVES = 4;
constexpr int MK = 8;                 // velocities per thread per chunk
constexpr int KCH = WAVES * MK;       // velocities per chunk
constexpr int NFP = 24;               // doubles per interface record
constexpr int NCP = 7;                // doubles per cell record of the predicted equilibrium

struct Geo {
    int nx, ny, nc, n_wall;
    const double *xc, *yc, *dx, *dy, *dcent, *dt;
    const int* nb;
    const unsigned char* solid;
    const int *w_cell, *w_side;
    const double *w_T, *w_U, *w_V, *w_den;
    const double *w_invd, *w_vol;   // 1 / width of the wall's cell normal to the wall, its volume
    const int* p_idx;
    const double* p_w;
};

struct Vel {
    int nk;
    const double *u, *v, *w;
    const float *uf, *vf, *wf;
    const int *mx, *my;   // the velocity with u (mx) or v (my) reversed (symmetry faces)
};

// the velocity with the component normal to side direction d reversed
__device__ __forceinline__ int mirror_of(const Vel& vel, int d, int k) { return d == 0 ? vel.mx[k] : vel.my[k]; }

struct Gas {
    int K_int;
    double K, gamma, Pr, omega, mu_ref;
    double W_inf[4];
    double rho_inf, U_inf, V_inf, lam_inf;
};

__device__ __forceinline__ bool is_wall(int code) { return code <= NB_WALL0; }
__device__ __forceinline__ int wall_of(int code) { return NB_WALL0 - code; }

template <typename T> __device__ __forceinline__ T vel_u(const Vel& v, int k);
template <typename T> __device__ __forceinline__ T vel_v(const Vel& v, int k);
template <typename T> __device__ __forceinline__ T vel_w(const Vel& v, int k);
template <> __device__ __forceinline__ double vel_u<double>(const Vel& v, int k) { return v.u[k]; }
template <> __device__ __forceinline__ double vel_v<double>(const Vel& v, int k) { return v.v[k]; }
template <> __device__ __forceinline__ double vel_w<double>(const Vel& v, int k) { return v.w[k]; }
template <> __device__ __forceinline__ float vel_u<float>(const Vel& v, int k) { return v.uf[k]; }
template <> __device__ __forceinline__ float vel_v<float>(const Vel& v, int k) { return v.vf[k]; }
template <> __device__ __forceinline__ float vel_w<float>(const Vel& v, int k) { return v.wf[k]; }

// Shakhov-type correction over the 2 + K_int degrees of freedom of the gas
// (Sec. II A), reduced to the pair (G, H):
//   G+ = s (c.q) (2 lam |c|^2 - 4) G_eq,  H+ = s (c.q) (2 lam |c|^2 - 2) H_eq,
//   s = 4 / (K_int + 4) (1 - Pr) lam^2 / rho,
// which carries no mass, momentum or energy and gives the heat flux (1 - Pr) q
__host__ __device__ inline double shakhov_prefactor(const Gas& gas) {
    return 4.0 / (gas.K_int + 4.0) * (1.0 - gas.Pr);
}

__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }

// Table of 2^(j/64), j < 64, for exp_tab (filled by the block that uses it)
constexpr int EXP_TAB = 64;
__device__ __forceinline__ void exp_tab_fill(double* tab) {
    if (threadIdx.x < EXP_TAB) tab[threadIdx.x] = exp2(double(threadIdx.x) / EXP_TAB);
}

// exp(x) by Tang's table-driven method (ACM TOMS 15(2), 1989): x = (64 m +
// j) ln2/64 + r with |r| <= ln2/128, exp(x) = 2^m 2^(j/64) e^r, e^r - 1 from
// its degree-5 Taylor polynomial (truncation below 4e-17 relative).  The
// reduction subtracts n ln2/64 in two fused steps (ln2/64 split into its
// nearest double and the remainder).  Underflows to zero below about -745;
// a NaN argument gives NaN.
__device__ __forceinline__ double exp_tab(double x, const double* __restrict__ tab) {
    const double n = __builtin_rint(x * 92.33248261689366);   // 64 / ln2
    double r = fma(-n, 0.010830424696249145, x);
    r = fma(-n, 3.623510646634843e-19, r);
    const int ni = int(n);
    double p = fma(r, 1.0 / 120.0, 1.0 / 24.0);
    p = fma(r, p, 1.0 / 6.0);
    p = fma(r, p, 0.5);
    p = fma(r, p, 1.0);
    p *= r;
    const double t = tab[ni & (EXP_TAB - 1)];
    return __builtin_amdgcn_ldexp(fma(t, p, t), ni >> 6);
}

// van Leer limiter: harmonic mean of one-sided slopes of equal sign, else 0
template <typename T> __device__ __forceinline__ T van_leer(T a, T b) {
    T s = a * b;
    return s > T(0) ? T(2) * s / (a + b) : T(0);
}

// ---------------------------------------------------------------------------
// gas-model helpers (double)

__device__ __forceinline__ double mu_of(const Gas& g, double T) { return g.mu_ref * pow(T, g.omega); }

__device__ __forceinline__ void prim_of(const double* W, double K, double& rho, double& U, double& V,
                                        double& lam) {
    rho = W[0];
    U = W[1] / rho;
    V = W[2] / rho;
    double e = W[3] - 0.5 * rho * (U * U + V * V);
    lam = K * rho / (4.0 * e);
}

__device__ __forceinline__ void cons_of(double rho, double U, double V, double lam, double K, double* W) {
    W[0] = rho;
    W[1] = rho * U;
    W[2] = rho * V;
    W[3] = 0.5 * rho * (U * U + V * V) + K * rho / (4.0 * lam);
}

// abar = a1 + a2 u + a3 v + a4 (u^2+v^2+xi^2)/2 with <abar psi g0> = rho0 b for
// a Maxwellian g0 with K total degrees of freedom (closed-form inverse of the
// moment matrix; the standard GKS micro-slope relation).
__device__ __forceinline__ void micro_slope(const double* b, double U, double V, double lam, double K,
                                            double* a) {
    double e = U * U + V * V + K / (2.0 * lam);
    double R2 = b[1] - U * b[0];
    double R3 = b[2] - V * b[0];
    double R4 = 2.0 * b[3] - e * b[0];
    a[3] = 4.0 * lam * lam / K * (R4 - 2.0 * U * R2 - 2.0 * V * R3);
    a[2] = 2.0 * lam * R3 - V * a[3];
    a[1] = 2.0 * lam * R2 - U * a[3];
    a[0] = b[0] - U * a[1] - V * a[2] - 0.5 * a[3] * e;
}

// Exact integrals over [0, dt] of the time factors of the UGKS interface
// distribution (x = dt/tau): (1 - e^{-t/tau}), ((t+tau) e^{-t/tau} - tau),
// (t - tau + tau e^{-t/tau}), e^{-t/tau}, -t e^{-t/tau}.  For x < 1/2 the
// closed forms cancel, so Taylor series (25 terms) are summed instead.
__device__ __forceinline__ void time_coeffs(double dt, double tau, double* q) {
    double x = dt / tau;
    double em1 = -expm1(-x);
    q[3] = tau * em1;
    if (x < 0.5) {
        double s1 = 0, s2 = 0, s3 = 0, s5 = 0, fact = 1.0, xp = 1.0;   // xp = x^(m-2)
        for (int m = 1; m <= 25; ++m) {
            fact *= m;
            double sg = (m & 1) ? -1.0 : 1.0;
            if (m >= 2) {
                s1 += sg * xp * x / fact;
                s5 += sg * (1 - m) * xp / fact;
                if (m >= 3) {
                    s2 += sg * (m - 2) * xp / fact;
                    s3 -= sg * xp / fact;
                }
                xp *= x;
            }
        }
        q[0] = dt * s1;
        q[1] = dt * dt * s2;
        q[2] = dt * dt * s3;
        q[4] = dt * dt * s5;
    } else {
        double e = exp(-x);
        q[0] = dt - tau * em1;
        q[1] = 2.0 * tau * tau * em1 - tau * dt - tau * dt * e;
        q[2] = 0.5 * dt * dt - tau * dt + tau * tau * em1;
        q[4] = tau * dt * e - tau * tau * em1;
    }
}

// ---------------------------------------------------------------------------
// helpers shared by the chunked kernels

struct Chunk {
    int c, lane, wave, k0, k1, chunk;
    bool valid;
};

__device__ __forceinline__ Chunk chunk_of(int nc, int nk, int kch = KCH) {
    Chunk ch;
    ch.lane = threadIdx.x & (TILE - 1);
    ch.wave = threadIdx.x / TILE;
    ch.c = blockIdx.x * TILE + ch.lane;
    ch.valid = ch.c < nc;
    ch.k0 = blockIdx.y * kch;
    ch.k1 = min(nk, ch.k0 + kch);
    ch.chunk = blockIdx.y;
    return ch;
}

// The chip dispatches workgroup b of a launch to XCD b mod 8, each XCD with
// its own L2.  Logical block of workgroup b such that every XCD takes a
// contiguous range of logical blocks (a bijection of [0, nb)).
__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
    constexpr int X = 8;
    int q = nb / X, r = nb % X;
    int x = b % X, i = b / X;
    return x * q + min(x, r) + i;
}

// chunk_of for kernels whose stencil reaches the rows above and below: the
// tiles of one velocity chunk are spread over as few XCDs as possible, so
// the neighbouring rows of a tile are found in the same L2
__device__ __forceinline__ Chunk chunk_of_xcd(int nc, int nk, int kch = KCH) {
    int nt = gridDim.x, nb = gridDim.x * gridDim.y;
    int Lb = xcd_swizzle(blockIdx.x + nt * blockIdx.y, nb);
    int tile = Lb % nt, chunk = Lb / nt;
    Chunk ch;
    ch.lane = threadIdx.x & (TILE - 1);
    ch.wave = threadIdx.x / TILE;
    ch.c = tile * TILE + ch.lane;
    ch.valid = ch.c < nc;
    ch.k0 = chunk * kch;
    ch.k1 = min(nk, ch.k0 + kch);
    ch.chunk = chunk;
    return ch;
}

// sum M partial values across the 4 waves of the block and store them as
// part[(chunk * M + m) * n + i]; sh holds ceil(M / R) * WAVES * TILE doubles
// and the values pass through it in R rounds (less LDS per block)
template <int M, int R = 1>
__device__ __forceinline__ void reduce_store(double* acc, double* sh, double* part, int n, int i,
                                             bool valid, int chunk = -1) {
    if (chunk < 0) chunk = blockIdx.y;
    constexpr int Q = (M + R - 1) / R;
    int lane = threadIdx.x & (TILE - 1), wave = threadIdx.x / TILE;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r > 0) __syncthreads();   // the previous round is read
#pragma unroll
        for (int m = r * Q; m < M && m < (r + 1) * Q; ++m) sh[((m - r * Q) * WAVES + wave) * TILE + lane] = acc[m];
        __syncthreads();
        if (wave == 0 && valid) {
#pragma unroll
            for (int m = r * Q; m < M && m < (r + 1) * Q; ++m) {
                double s = sh[((m - r * Q) * WAVES + 0) * TILE + lane];
                for (int w = 1; w < WAVES; ++w) s += sh[((m - r * Q) * WAVES + w) * TILE + lane];
                part[((size_t)chunk * M + m) * n + i] = s;
            }
        }
    }
}

// raw moments of (G, H): sum w {G, uG, vG, u^2 G, uvG, v^2 G, u|u|^2 G, v|u|^2 G, H, uH, vH}
constexpr int NRAW = 11;

__device__ __forceinline__ void raw_accumulate(double* a, double w, double u, double v, double G,
                                               double H) {
    double wG = w * G, wH = w * H, e2 = u * u + v * v;
    a[0] += wG;
    a[1] += u * wG;
    a[2] += v * wG;
    a[3] += u * u * wG;
    a[4] += u * v * wG;
    a[5] += v * v * wG;
    a[6] += u * e2 * wG;
    a[7] += v * e2 * wG;
    a[8] += wH;
    a[9] += u * wH;
    a[10] += v * wH;
}

// conservative variables and heat flux (about the mean velocity) from raw moments
__device__ __forceinline__ void raw_to_macro(const double* M, double* W, double* q) {
    double rho = M[0], U = M[1] / rho, V = M[2] / rho;
    W[0] = M[0];
    W[1] = M[1];
    W[2] = M[2];
    W[3] = 0.5 * (M[3] + M[5] + M[8]);
    double U2 = U * U + V * V, E2 = M[3] + M[5];
    double cx = M[6] - 2.0 * U * M[3] - 2.0 * V * M[4] + U2 * M[1] - U * E2 + 2.0 * U * U * M[1] +
                2.0 * U * V * M[2] - U * U2 * M[0];
    double cy = M[7] - 2.0 * U * M[4] - 2.0 * V * M[5] + U2 * M[2] - V * E2 + 2.0 * U * V * M[1] +
                2.0 * V * V * M[2] - V * U2 * M[0];
    q[0] = 0.5 * (cx + M[9] - U * M[8]);
    q[1] = 0.5 * (cy + M[10] - V * M[8]);
}

// ---------------------------------------------------------------------------
// initial distribution: reduced Maxwellian of (rho, U, V, T) per cell

template <typename T>
__global__ void __launch_bounds__(256) k_init(Geo g, Vel vel, Gas gas, const double* __restrict__ prim,
                                              T* __restrict__ f) {
    Chunk ch = chunk_of(g.nc, vel.nk);
    if (!ch.valid) return;
    int c = ch.c;
    bool fluid = !g.solid[c];
    double rho = prim[c], U = prim[g.nc + c], V = prim[2 * g.nc + c], lam = 1.0 / prim[3 * g.nc + c];
    for (int k = ch.k0 + ch.wave; k < ch.k1; k += WAVES) {
        double du = vel.u[k] - U, dv = vel.v[k] - V;
        double G = fluid ? rho * (lam / M_PI) * exp(-lam * (du * du + dv * dv)) : 0.0;
        f[(size_t)k * g.nc + c] = T(G);
        f[(size_t)(vel.nk + k) * g.nc + c] = T(gas.K_int / (2.0 * lam) * G);
    }
}

// ---------------------------------------------------------------------------
// cell moments (Step 7 and the compatibility condition): W and q of f.
// With df != nullptr the kernel first applies Step 6, f += df, and stores f.

template <typename T>
__global__ void __launch_bounds__(256) k_moments_partial(Geo g, Vel vel, T* __restrict__ f,
                                                         const T* __restrict__ df,
                                                         double* __restrict__ part, int kch) {
    __shared__ double sh[NRAW * WAVES * TILE];
    Chunk ch = chunk_of(g.nc, vel.nk, kch);
    const int wave = __builtin_amdgcn_readfirstlane(ch.wave);
    const int k0 = __builtin_amdgcn_readfirstlane(ch.k0), k1 = __builtin_amdgcn_readfirstlane(ch.k1);
    double a[NRAW];
    for (int m = 0; m < NRAW; ++m) a[m] = 0.0;
    if (ch.valid) {
        const size_t nc = g.nc, ho = (size_t)vel.nk * nc;
        // UM velocities per step: their loads are issued together (a wave
        // reads 256 bytes per plane and velocity, so one at a time leaves
        // the memory system idle); the sums keep the velocity order
        constexpr int UM = 4;
        int k = k0 + wave;
        for (; k + WAVES * (UM - 1) < k1; k += WAVES * UM) {
            T G[UM], H[UM];
#pragma unroll
            for (int u = 0; u < UM; ++u) {
                const size_t ig = (size_t)(k + WAVES * u) * nc + ch.c;
                G[u] = f[ig];
                H[u] = f[ho + ig];
            }
            if (df) {
                T dG[UM], dH[UM];
#pragma unroll
                for (int u = 0; u < UM; ++u) {
                    const size_t ig = (size_t)(k + WAVES * u) * nc + ch.c;
                    dG[u] = df[ig];
                    dH[u] = df[ho + ig];
                }
#pragma unroll
                for (int u = 0; u < UM; ++u) {
                    const size_t ig = (size_t)(k + WAVES * u) * nc + ch.c;
                    G[u] += dG[u];
                    H[u] += dH[u];
                    f[ig] = G[u];
                    f[ho + ig] = H[u];
                }
            }
#pragma unroll
            for (int u = 0; u < UM; ++u) {
                const int ku = k + WAVES * u;
                raw_accumulate(a, vel.w[ku], vel.u[ku], vel.v[ku], double(G[u]), double(H[u]));
            }
        }
        for (; k < k1; k += WAVES) {
            const size_t ig = (size_t)k * nc + ch.c;
            T G = f[ig], H = f[ho + ig];
            if (df) {
                G += df[ig];
                H += df[ho + ig];
                f[ig] = G;
                f[ho + ig] = H;
            }
            raw_accumulate(a, vel.w[k], vel.u[k], vel.v[k], double(G), double(H));
        }
    }
    reduce_store<NRAW>(a, sh, part, g.nc, ch.c, ch.valid);
}

__global__ void k_moments_finalize(Geo g, const double* __restrict__ part, int nkc,
                                   double* __restrict__ W, double* __restrict__ q) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    if (g.solid[c]) {
        for (int m = 0; m < 4; ++m) W[m * g.nc + c] = 0.0;
        q[c] = q[g.nc + c] = 0.0;
        return;
    }
    double M[NRAW];
    for (int m = 0; m < NRAW; ++m) {
        double s = 0.0;
        for (int j = 0; j < nkc; ++j) s += part[((size_t)j * NRAW + m) * g.nc + c];
        M[m] = s;
    }
    double w4[4], q2[2];
    raw_to_macro(M, w4, q2);
    for (int m = 0; m < 4; ++m) W[m * g.nc + c] = w4[m];
    q[c] = q2[0];
    q[g.nc + c] = q2[1];
}

// W, q of every cell from the summed raw moments Msum[m nc + c] (zero on
// solid cells); one thread per cell
__global__ void k_moments_records(Geo g, const double* __restrict__ Msum, double* __restrict__ W,
                                  double* __restrict__ q) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    if (g.solid[c]) {
        for (int m = 0; m < 4; ++m) W[m * g.nc + c] = 0.0;
        q[c] = q[g.nc + c] = 0.0;
        return;
    }
    double M[NRAW];
    for (int m = 0; m < NRAW; ++m) M[m] = Msum[(size_t)m * g.nc + c];
    double w4[4], q2[2];
    raw_to_macro(M, w4, q2);
    for (int m = 0; m < 4; ++m) W[m * g.nc + c] = w4[m];
    q[c] = q2[0];
    q[g.nc + c] = q2[1];
}

// Loads on the diffuse walls (Sec. IV B: skin friction from the momentum
// the gas hands to the wall): for wall side j the distribution on the wall
// side of the face is the cell's for velocities leaving the gas and the wall
// Maxwellian rho_w C_k for the others (Sec. III B); in the wall's frame,
// c = u - U_w, with c_n along the normal out of the gas and c_t along the
// face, out[j] = sum_k w c_n^2 f^G (pressure), out[nw + j] = sum_k w c_t c_n
// f^G (shear), out[2 nw + j] = 1/2 sum_k w c_n (|c|^2 f^G + f^H) (heat flux),
// out[3 nw + j] = the face area.  One wavefront per wall side, double sums.
template <typename T>
__global__ void k_wall_loads(Geo g, Vel vel, int K_int, const T* __restrict__ f, double* __restrict__ out) {
    int j = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    int lane = threadIdx.x & 63;
    if (j >= g.n_wall) return;
    const int c = g.w_cell[j], sd = g.w_side[j], nw = g.n_wall;
    const size_t ho = (size_t)vel.nk * g.nc;
    const double sign = (sd & 1) ? 1.0 : -1.0;
    const double lam = 1.0 / g.w_T[j], Uw = g.w_U[j], Vw = g.w_V[j];
    double s = 0.0;
    for (int k = lane; k < vel.nk; k += 64) {
        double un = sign * (sd < 2 ? vel.u[k] : vel.v[k]);
        if (un > 0) s += vel.w[k] * un * double(f[(size_t)k * g.nc + c]);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const double rho_w = -s / g.w_den[j];
    double p = 0.0, t = 0.0, q = 0.0;
    for (int k = lane; k < vel.nk; k += 64) {
        double u = vel.u[k], v = vel.v[k], w = vel.w[k];
        double un = sign * (sd < 2 ? u : v);
        double cx = u - Uw, cy = v - Vw, c2 = cx * cx + cy * cy;
        double cn = sign * (sd < 2 ? cx : cy), ct = sd < 2 ? cy : cx;
        double Gf, Hf;
        if (un > 0) {
            Gf = double(f[(size_t)k * g.nc + c]);
            Hf = double(f[ho + (size_t)k * g.nc + c]);
        } else {
            Gf = rho_w * (lam / M_PI) * exp(-lam * c2);
            Hf = (K_int / (2.0 * lam)) * Gf;
        }
        p += w * cn * cn * Gf;
        t += w * ct * cn * Gf;
        q += 0.5 * w * cn * (c2 * Gf + Hf);
    }
    for (int off = 32; off > 0; off >>= 1) {
        p += __shfl_xor(p, off, 64);
        t += __shfl_xor(t, off, 64);
        q += __shfl_xor(q, off, 64);
    }
    if (lane == 0) {
        out[j] = p;
        out[nw + j] = t;
        out[2 * nw + j] = q;
        out[3 * nw + j] = sd < 2 ? g.dy[c / g.nx] : g.dx[c % g.nx];
    }
}

// Diffuse-wall densities from zero mass flux (Sec. III B):
// out[j] = -sum_{u_n > 0} w u_n G / den_j, with G the first (G) plane of f or
// of a correction, or (PRO) the wall densities of df_fine + I_H^h df_coarse
// evaluated at the wall cells only (the prolonged correction is needed
// nowhere else when a sweep follows).  A lane per wall side, the velocities
// in slices of WD_K (blockIdx.y): consecutive sides of a wall lie along
// consecutive cells, so the loads of one velocity coalesce, and
// n_wall / 64 x nk / WD_K wavefronts share the chip.  part[slice][j] = the
// slice's sum; k_wall_density_fin adds the slices in order.
constexpr int WD_K = 32;
inline int wall_density_slices(int nk) { return (nk + WD_K - 1) / WD_K; }
// velocity sets up to this size take k_wall_density_wave (one launch) instead
constexpr int WD_WAVE_MAX_NK = 2048;


template <typename T, bool PRO>
__global__ void __launch_bounds__(64) k_wall_density_part(Geo g, Vel vel, const T* __restrict__ Gf, int ncc,
                                                          const T* __restrict__ Gc, double* __restrict__ part) {
    const int j = blockIdx.x * 64 + threadIdx.x;
    const int k0 = blockIdx.y * WD_K, k1 = min(vel.nk, k0 + WD_K);
    double s = 0.0;
    if (j < g.n_wall) {
        const int c = g.w_cell[j], sd = g.w_side[j];
        const double sign = (sd & 1) ? 1.0 : -1.0;
        int id[4] = {0, 0, 0, 0};
        T pw[4] = {T(0), T(0), T(0), T(0)};
        if constexpr (PRO)
            for (int a = 0; a < 4; ++a) {
                id[a] = g.p_idx[a * g.nc + c];
                pw[a] = T(g.p_w[a * g.nc + c]);
            }
        for (int k = k0; k < k1; ++k) {
            const double un = sign * (sd < 2 ? vel.u[k] : vel.v[k]);
            if (un > 0) {
                T G = Gf[(size_t)k * g.nc + c];
                if constexpr (PRO) {
                    const size_t kc = (size_t)k * ncc;
                    const T add = pw[0] * Gc[kc + id[0]] + pw[1] * Gc[kc + id[1]] + pw[2] * Gc[kc + id[2]] +
                                  pw[3] * Gc[kc + id[3]];
                    G = G + add;
                }
                s += vel.w[k] * un * double(G);
            }
        }
        part[(size_t)blockIdx.y * g.n_wall + j] = s;
    }
}

// The same density in one launch for small velocity sets: one wavefront per
// wall side, lane l taking the velocities l, l + 64, ..., then the lanes in a
// fixed tree; out[j] = rho_w
template <typename T, bool PRO>
__global__ void __launch_bounds__(256) k_wall_density_wave(Geo g, Vel vel, const T* __restrict__ Gf, int ncc,
                                                           const T* __restrict__ Gc, double* __restrict__ out) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    double s = 0.0;
    if (j < g.n_wall) {
        const int c = g.w_cell[j], sd = g.w_side[j];
        const double sign = (sd & 1) ? 1.0 : -1.0;
        int id[4] = {0, 0, 0, 0};
        T pw[4] = {T(0), T(0), T(0), T(0)};
        if constexpr (PRO)
            for (int a = 0; a < 4; ++a) {
                id[a] = g.p_idx[a * g.nc + c];
                pw[a] = T(g.p_w[a * g.nc + c]);
            }
        for (int k = lane; k < vel.nk; k += 64) {
            const double un = sign * (sd < 2 ? vel.u[k] : vel.v[k]);
            if (un > 0) {
                T G = Gf[(size_t)k * g.nc + c];
                if constexpr (PRO) {
                    const size_t kc = (size_t)k * ncc;
                    const T add = pw[0] * Gc[kc + id[0]] + pw[1] * Gc[kc + id[1]] + pw[2] * Gc[kc + id[2]] +
                                  pw[3] * Gc[kc + id[3]];
                    G = G + add;
                }
                s += vel.w[k] * un * double(G);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0 && j < g.n_wall) out[j] = -s / g.w_den[j];
}

// rho_w = -(sum of the slices) / w_den, one wavefront per wall side: lane l
// adds slices l, l + 64, ..., then the lanes in a fixed tree (a fixed order)
__global__ void __launch_bounds__(256) k_wall_density_fin(Geo g, int nslices, const double* __restrict__ part,
                                                          double* __restrict__ out) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    double s = 0.0;
    if (j < g.n_wall)
        for (int b = lane; b < nslices; b += 64) s += part[(size_t)b * g.n_wall + j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0 && j < g.n_wall) out[j] = -s / g.w_den[j];
}


// total mass sum_c V_c rho_c over fluid cells (one block)
__global__ void k_mass(Geo g, const double* __restrict__ W, double* __restrict__ out) {
    __shared__ double sh[1024];
    double s = 0.0;
    for (int c = threadIdx.x; c < g.nc; c += blockDim.x)
        if (!g.solid[c]) s += g.dx[c % g.nx] * g.dy[c / g.nx] * W[c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// closed-domain renormalisation f *= M0 / M (and W, q alike)
template <typename T>
__global__ void k_scale_f(T* __restrict__ f, size_t n, const double* __restrict__ mass, double M0) {
    double s = M0 / mass[0];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        f[i] = T(double(f[i]) * s);
}

__global__ void k_scale_d(double* __restrict__ a, size_t n, const double* __restrict__ mass, double M0) {
    double s = M0 / mass[0];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] *= s;
}

// ---------------------------------------------------------------------------
// Step 1, interface reconstruction (Sec. II A 1; UGKS flux).  Every interior
// face is the -x or -y face of exactly one cell R with neighbour L across it.

// 1/x from the hardware reciprocal refined by Newton steps (two in double,
// one in float): the van Leer limiter below divides once per call
__device__ __forceinline__ double rcp_refined(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp_refined(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
// prim_of with the reciprocals refined instead of divided
__device__ __forceinline__ void prim_of_r(const double* W, double K, double& rho, double& U, double& V,
                                          double& lam) {
    rho = W[0];
    double ir = rcp_refined(rho);
    U = W[1] * ir;
    V = W[2] * ir;
    double e = W[3] - 0.5 * rho * (U * U + V * V);
    lam = K * rho * rcp_refined(4.0 * e);
}

template <typename T> __device__ __forceinline__ T van_leer_fast(T a, T b) {
    T s = a * b;
    return s > T(0) ? T(2) * s * rcp_refined(a + b) : T(0);
}

// Geometry of the face on side 2d of cell c (the cell R = c, neighbour L
// across it), independent of the velocity
template <typename A>
struct FaceGeom {
    int L, LL, RR;        // neighbour across the face, L's neighbour beyond it, c's neighbour beyond (<0: none)
    A idc, idcL, idcR;    // inverse centre distances L-c, LL-L, c-RR
    A dL, dR;             // half widths of L and c normal to the face
};

template <typename A>
__device__ __forceinline__ bool face_geom(const Geo& g, int c, int d, FaceGeom<A>& fg) {
    int nc = g.nc;
    fg.L = g.nb[(2 * d) * nc + c];
    if (fg.L < 0) return false;
    fg.LL = g.nb[(2 * d) * nc + fg.L];
    fg.RR = g.nb[(2 * d + 1) * nc + c];
    fg.idc = A(1.0 / g.dcent[(2 * d) * nc + c]);
    fg.idcL = fg.LL >= 0 ? A(1.0 / g.dcent[(2 * d) * nc + fg.L]) : A(0);
    fg.idcR = fg.RR >= 0 ? A(1.0 / g.dcent[(2 * d + 1) * nc + c]) : A(0);
    fg.dL = A(0.5) * A(d == 0 ? g.dx[fg.L % g.nx] : g.dy[fg.L / g.nx]);
    fg.dR = A(0.5) * A(d == 0 ? g.dx[c % g.nx] : g.dy[c / g.nx]);
    return true;
}

// the stored values a face reconstruction reads for one velocity: L and the
// cell c, L's far neighbour LL and c's far neighbour RR (zero when absent)
template <typename T>
struct FaceVals {
    T GL, GR, HL, HR, GLL, HLL, GRR, HRR;
};

template <typename T, typename A>
__device__ __forceinline__ void face_load(const FaceGeom<A>& fg, int c, const T* __restrict__ F, size_t ho,
                                          size_t kc, FaceVals<T>& q) {
    q.GL = F[kc + fg.L];
    q.GR = F[kc + c];
    q.HL = F[ho + kc + fg.L];
    q.HR = F[ho + kc + c];
    q.GLL = fg.LL >= 0 ? F[kc + fg.LL] : T(0);
    q.HLL = fg.LL >= 0 ? F[ho + kc + fg.LL] : T(0);
    q.GRR = fg.RR >= 0 ? F[kc + fg.RR] : T(0);
    q.HRR = fg.RR >= 0 ? F[ho + kc + fg.RR] : T(0);
}

// face_upwind_k on values already loaded
template <typename T, typename A>
__device__ __forceinline__ void face_upwind_vals(const FaceGeom<A>& fg, const FaceVals<T>& q, A un, A& Gup,
                                                 A& Hup, A& sGup, A& sHup) {
    A GL = A(q.GL), GR = A(q.GR), HL = A(q.HL), HR = A(q.HR);
    A gLR = (GR - GL) * fg.idc, hLR = (HR - HL) * fg.idc;
    A gm = fg.LL >= 0 ? (GL - A(q.GLL)) * fg.idcL : A(0), hm = fg.LL >= 0 ? (HL - A(q.HLL)) * fg.idcL : A(0);
    A gp = fg.RR >= 0 ? (A(q.GRR) - GR) * fg.idcR : A(0), hp = fg.RR >= 0 ? (A(q.HRR) - HR) * fg.idcR : A(0);
    A sGL = un >= A(0) ? van_leer_fast(gm, gLR) : A(0), sHL = un >= A(0) ? van_leer_fast(hm, hLR) : A(0);
    A sGR = un <= A(0) ? van_leer_fast(gLR, gp) : A(0), sHR = un <= A(0) ? van_leer_fast(hLR, hp) : A(0);
    if (un > A(0)) {
        Gup = GL + sGL * fg.dL;
        Hup = HL + sHL * fg.dL;
        sGup = sGL;
        sHup = sHL;
    } else if (un < A(0)) {
        Gup = GR - sGR * fg.dR;
        Hup = HR - sHR * fg.dR;
        sGup = sGR;
        sHup = sHR;
    } else {
        Gup = A(0.5) * (GL + sGL * fg.dL + GR - sGR * fg.dR);
        Hup = A(0.5) * (HL + sHL * fg.dL + HR - sHR * fg.dR);
        sGup = A(0.5) * (sGL + sGR);
        sHup = A(0.5) * (sHL + sHR);
    }
}

// limited slopes and upwind interface values of one velocity (row offset kc
// into the G plane, ho = offset of the H plane) at an interior face
template <typename T, typename A>
__device__ __forceinline__ void face_upwind_k(const FaceGeom<A>& fg, int c, const T* __restrict__ F, size_t ho,
                                              size_t kc, A un, A& Gup, A& Hup, A& sGup, A& sHup) {
    A GL = A(F[kc + fg.L]), GR = A(F[kc + c]), HL = A(F[ho + kc + fg.L]), HR = A(F[ho + kc + c]);
    A gLR = (GR - GL) * fg.idc, hLR = (HR - HL) * fg.idc;
    A sGL = 0, sHL = 0, sGR = 0, sHR = 0;
    if (un >= A(0)) {   // left slope needed (and both for un == 0)
        A gm = 0, hm = 0;
        if (fg.LL >= 0) {
            gm = (GL - A(F[kc + fg.LL])) * fg.idcL;
            hm = (HL - A(F[ho + kc + fg.LL])) * fg.idcL;
        }
        sGL = van_leer_fast(gm, gLR);
        sHL = van_leer_fast(hm, hLR);
    }
    if (un <= A(0)) {
        A gp = 0, hp = 0;
        if (fg.RR >= 0) {
            gp = (A(F[kc + fg.RR]) - GR) * fg.idcR;
            hp = (A(F[ho + kc + fg.RR]) - HR) * fg.idcR;
        }
        sGR = van_leer_fast(gLR, gp);
        sHR = van_leer_fast(hLR, hp);
    }
    if (un > A(0)) {
        Gup = GL + sGL * fg.dL;
        Hup = HL + sHL * fg.dL;
        sGup = sGL;
        sHup = sHL;
    } else if (un < A(0)) {
        Gup = GR - sGR * fg.dR;
        Hup = HR - sHR * fg.dR;
        sGup = sGR;
        sHup = sHR;
    } else {
        Gup = A(0.5) * (GL + sGL * fg.dL + GR - sGR * fg.dR);
        Hup = A(0.5) * (HL + sHL * fg.dL + HR - sHR * fg.dR);
        sGup = A(0.5) * (sGL + sGR);
        sHup = A(0.5) * (sHL + sHR);
    }
}

// limited slopes of the two cells of the face on side (2d) of cell c, and the
// upwind interface values for one velocity.  Returns false if not interior.
template <typename T, typename A>
__device__ __forceinline__ bool face_upwind(const Geo& g, int c, int d, const T* __restrict__ F, int nk,
                                            int k, A un, A& Gup, A& Hup, A& sGup, A& sHup) {
    int nc = g.nc;
    int L = g.nb[(2 * d) * nc + c];
    if (L < 0) return false;
    int LL = g.nb[(2 * d) * nc + L];
    int RR = g.nb[(2 * d + 1) * nc + c];
    size_t ho = (size_t)nk * nc;
    size_t kc = (size_t)k * nc;
    A dcLR = A(g.dcent[(2 * d) * nc + c]);
    A dL = A(0.5) * A(d == 0 ? g.dx[L % g.nx] : g.dy[L / g.nx]);
    A dR = A(0.5) * A(d == 0 ? g.dx[c % g.nx] : g.dy[c / g.nx]);
    A GL = A(F[kc + L]), GR = A(F[kc + c]), HL = A(F[ho + kc + L]), HR = A(F[ho + kc + c]);
    A gLR = (GR - GL) / dcLR, hLR = (HR - HL) / dcLR;
    A sGL = 0, sHL = 0, sGR = 0, sHR = 0;
    if (un >= A(0)) {   // left slope needed (and both for un == 0)
        A gm = 0, hm = 0;
        if (LL >= 0) {
            A dc = A(g.dcent[(2 * d) * nc + L]);
            gm = (GL - A(F[kc + LL])) / dc;
            hm = (HL - A(F[ho + kc + LL])) / dc;
        }
        sGL = van_leer(gm, gLR);
        sHL = van_leer(hm, hLR);
    }
    if (un <= A(0)) {
        A gp = 0, hp = 0;
        if (RR >= 0) {
            A dc = A(g.dcent[(2 * d + 1) * nc + c]);
            gp = (A(F[kc + RR]) - GR) / dc;
            hp = (A(F[ho + kc + RR]) - HR) / dc;
        }
        sGR = van_leer(gLR, gp);
        sHR = van_leer(hLR, hp);
    }
    if (un > A(0)) {
        Gup = GL + sGL * dL;
        Hup = HL + sHL * dL;
        sGup = sGL;
        sHup = sHL;
    } else if (un < A(0)) {
        Gup = GR - sGR * dR;
        Hup = HR - sHR * dR;
        sGup = sGR;
        sHup = sHR;
    } else {
        Gup = A(0.5) * (GL + sGL * dL + GR - sGR * dR);
        Hup = A(0.5) * (HL + sHL * dL + HR - sHR * dR);
        sGup = A(0.5) * (sGL + sGR);
        sHup = A(0.5) * (sHL + sHR);
    }
    return true;
}

// Raw buffer resource over `bytes` bytes from p.  The stencil loads of the
// interface flux go through one per distribution plane and velocity chunk:
// a lane's byte offset (a cell) in a vector register, the velocity's row
// offset in a scalar one, so a load costs no vector address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// A face's reconstruction stencil as byte offsets within a plane row: L and
// the cell R on either side, L's far neighbour LL and R's far neighbour RR
// (an absent far neighbour reads its near one, with its inverse distance
// zero, so that the one-sided difference vanishes)
template <typename T>
struct FaceStencil {
    unsigned oL, oR, oLL, oRR;
    T idc, idcL, idcR, dL, dR;
};

template <typename T, typename A = T>
__device__ __forceinline__ void face_stencil(const Geo& g, int c, int d, FaceStencil<A>& s) {
    FaceGeom<A> fg;
    face_geom<A>(g, c, d, fg);
    s.oL = (unsigned)fg.L * sizeof(T);
    s.oR = (unsigned)c * sizeof(T);
    s.oLL = (unsigned)(fg.LL >= 0 ? fg.LL : fg.L) * sizeof(T);
    s.oRR = (unsigned)(fg.RR >= 0 ? fg.RR : c) * sizeof(T);
    s.idc = fg.idc;
    s.idcL = fg.idcL;
    s.idcR = fg.idcR;
    s.dL = fg.dL;
    s.dR = fg.dR;
}

template <typename T, typename A = T>
__device__ __forceinline__ void stencil_load(const FaceStencil<A>& s, __amdgpu_buffer_rsrc_t RG,
                                             __amdgpu_buffer_rsrc_t RH, unsigned so, FaceVals<T>& q) {
    q.GL = buf_ld<T>(RG, s.oL, so);
    q.GR = buf_ld<T>(RG, s.oR, so);
    q.HL = buf_ld<T>(RH, s.oL, so);
    q.HR = buf_ld<T>(RH, s.oR, so);
    q.GLL = buf_ld<T>(RG, s.oLL, so);
    q.HLL = buf_ld<T>(RH, s.oLL, so);
    q.GRR = buf_ld<T>(RG, s.oRR, so);
    q.HRR = buf_ld<T>(RH, s.oRR, so);
}

// side of a face's upwind cell for a normal velocity un (the same in every
// lane): 0 for un > 0 (L), 1 for un < 0 (R), 2 for un = 0
__device__ __forceinline__ int upwind_side(double un) {
    return __builtin_amdgcn_readfirstlane(un > 0.0 ? 0 : (un < 0.0 ? 1 : 2));
}

// limited slope and interface value on the upwind side (face_upwind_vals
// with the side known for the whole wavefront: only that side's slope is
// formed), in A from the stored values
template <typename T, typename A = T>
__device__ __forceinline__ void upwind_on_side(const FaceStencil<A>& s, const FaceVals<T>& q, int side, A& Gup,
                                               A& Hup, A& sGup, A& sHup) {
    const A GL = A(q.GL), GR = A(q.GR), HL = A(q.HL), HR = A(q.HR);
    A gLR = (GR - GL) * s.idc, hLR = (HR - HL) * s.idc;
    if (side == 0) {
        A gm = (GL - A(q.GLL)) * s.idcL, hm = (HL - A(q.HLL)) * s.idcL;
        sGup = van_leer_fast(gm, gLR);
        sHup = van_leer_fast(hm, hLR);
        Gup = GL + sGup * s.dL;
        Hup = HL + sHup * s.dL;
    } else if (side == 1) {
        A gp = (A(q.GRR) - GR) * s.idcR, hp = (A(q.HRR) - HR) * s.idcR;
        sGup = van_leer_fast(gLR, gp);
        sHup = van_leer_fast(hLR, hp);
        Gup = GR - sGup * s.dR;
        Hup = HR - sHup * s.dR;
    } else {
        A gm = (GL - A(q.GLL)) * s.idcL, hm = (HL - A(q.HLL)) * s.idcL;
        A gp = (A(q.GRR) - GR) * s.idcR, hp = (A(q.HRR) - HR) * s.idcR;
        A sGL = van_leer_fast(gm, gLR), sHL = van_leer_fast(hm, hLR);
        A sGR = van_leer_fast(gLR, gp), sHR = van_leer_fast(hLR, hp);
        Gup = A(0.5) * (GL + sGL * s.dL + GR - sGR * s.dR);
        Hup = A(0.5) * (HL + sHL * s.dL + HR - sHR * s.dR);
        sGup = A(0.5) * (sGL + sGR);
        sHup = A(0.5) * (sHL + sHR);
    }
}

// raw moments of the upwind interface distribution of the -x and -y faces.
// The interface values are formed in T from the stored distribution, with
// the same arithmetic as k_flux_div's (so the equilibrium of a face is built
// from the very values its flux transports); the moments are summed in
// double.  The velocity is the same in every lane: the upwind side is a
// scalar branch and the stencil loads take scalar row offsets.
template <typename T>
__global__ void __launch_bounds__(256) k_face_moments_partial(Geo g, Vel vel, const T* __restrict__ f,
                                                              double* __restrict__ part, int kch) {
    // the 22 sums leave through LDS in two rounds: 22.5 KB per block
    __shared__ double sh[NRAW * WAVES * TILE];
    Chunk ch = chunk_of_xcd(g.nc, vel.nk, kch);
    const int wave = __builtin_amdgcn_readfirstlane(ch.wave);
    const int k0 = __builtin_amdgcn_readfirstlane(ch.k0), k1 = __builtin_amdgcn_readfirstlane(ch.k1);
    const size_t nc = g.nc, ho = (size_t)vel.nk * nc;
    const unsigned rowb = (unsigned)(nc * sizeof(T));
    const unsigned chunkb = (unsigned)(k1 - k0) * rowb;
    const __amdgpu_buffer_rsrc_t RG = buf_rsrc(f + (size_t)k0 * nc, chunkb);
    const __amdgpu_buffer_rsrc_t RH = buf_rsrc(f + ho + (size_t)k0 * nc, chunkb);
    double a[2 * NRAW];
    for (int m = 0; m < 2 * NRAW; ++m) a[m] = 0.0;
    if (ch.valid && !g.solid[ch.c]) {
        for (int d = 0; d < 2; ++d) {
            if (g.nb[(2 * d) * g.nc + ch.c] < 0) continue;   // not an interior face
            FaceStencil<T> st;
            face_stencil<T>(g, ch.c, d, st);
            // the stencil values of the next velocity load while this one computes
            FaceVals<T> cur{}, nxt{};
            int k = k0 + wave;
            if (k < k1) stencil_load<T>(st, RG, RH, (unsigned)(k - k0) * rowb, nxt);
            for (; k < k1; k += WAVES) {
                cur = nxt;
                if (k + WAVES < k1) stencil_load<T>(st, RG, RH, (unsigned)(k + WAVES - k0) * rowb, nxt);
                const double u = vel.u[k], v = vel.v[k], w = vel.w[k];
                const int side = upwind_side(d == 0 ? u : v);
                T Gup, Hup, sG, sH;
                upwind_on_side<T>(st, cur, side, Gup, Hup, sG, sH);
                raw_accumulate(a + d * NRAW, w, u, v, double(Gup), double(Hup));
            }
        }
    }
    reduce_store<2 * NRAW, 2>(a, sh, part, g.nc, ch.c, ch.valid, ch.chunk);
}

// Reductions over all velocities inside one block: 64 lanes (consecutive
// cells) x FW waves, wave w taking velocities w, w + FW, ...; the waves'
// partial sums are added in LDS in a fixed order (deterministic) by wave 0,
// which then owns the totals.
constexpr int FW = 8;

template <int M>
__device__ __forceinline__ void block_sum_waves(double* acc, double* sh) {
    // sh holds at least ceil(M/2) * FW * 64 doubles; two rounds of M/2 moments
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int H = (M + 1) / 2;
    double tot[M];
    for (int half = 0; half < 2; ++half) {
        int m0 = half * H, m1 = M < m0 + H ? M : m0 + H;
        for (int m = m0; m < m1; ++m) sh[((m - m0) * FW + wave) * 64 + lane] = acc[m];
        __syncthreads();
        if (wave == 0)
            for (int m = m0; m < m1; ++m) {
                double t = sh[((m - m0) * FW + 0) * 64 + lane];
                for (int w = 1; w < FW; ++w) t += sh[((m - m0) * FW + w) * 64 + lane];
                tot[m] = t;
            }
        __syncthreads();
    }
    if (wave == 0)
        for (int m = 0; m < M; ++m) acc[m] = tot[m];
}

// Interface record, per (direction d, cell c) = the face on side 2d of c:
//  0 rho0  1 U0  2 V0  3 lam0  4,5 Shakhov coefficients 4/(K_int+4) (1-Pr) lam0^2 q0 / rho0
//  6-9 abar left  10-13 abar right  14-17 Abar  18-22 q1..q5 / dt  23 interior flag
__global__ void k_face_finalize(Geo g, Gas gas, const double* __restrict__ part, int nkc,
                                const double* __restrict__ W, double* __restrict__ fp) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    size_t stride = 2 * (size_t)g.nc;
    for (int d = 0; d < 2; ++d) {
        double* rec = fp + (size_t)d * g.nc + c;
        int L = g.nb[(2 * d) * g.nc + c];
        if (g.solid[c] || L < 0) {
            for (int m = 0; m < NFP; ++m) rec[m * stride] = 0.0;
            continue;
        }
        double M[NRAW];
        for (int m = 0; m < NRAW; ++m) {
            double s = 0.0;
            for (int j = 0; j < nkc; ++j) s += part[((size_t)j * 2 * NRAW + d * NRAW + m) * g.nc + c];
            M[m] = s;
        }
        double W0[4], q0[2];
        raw_to_macro(M, W0, q0);
        double rho, U, V, lam;
        prim_of(W0, gas.K, rho, U, V, lam);
        double tau = mu_of(gas, 1.0 / lam) / (rho / (2.0 * lam));
        double dt = fmin(g.dt[L], g.dt[c]);
        double q[5];
        time_coeffs(dt, tau, q);
        double dL = 0.5 * (d == 0 ? g.dx[L % g.nx] : g.dy[L / g.nx]);
        double dR = 0.5 * (d == 0 ? g.dx[c % g.nx] : g.dy[c / g.nx]);
        double bL[4], bR[4], aL[4], aR[4];
        for (int m = 0; m < 4; ++m) {
            bL[m] = (W0[m] - W[m * g.nc + L]) / dL / rho;
            bR[m] = (W[m * g.nc + c] - W0[m]) / dR / rho;
        }
        micro_slope(bL, U, V, lam, gas.K, aL);
        micro_slope(bR, U, V, lam, gas.K, aR);
        double sh = shakhov_prefactor(gas) * lam * lam / rho;
        double vals[NFP] = {rho, U, V, lam, sh * q0[0], sh * q0[1],
                            aL[0], aL[1], aL[2], aL[3], aR[0], aR[1], aR[2], aR[3],
                            0, 0, 0, 0,
                            q[0] / dt, q[1] / dt, q[2] / dt, q[3] / dt, q[4] / dt, 1.0};
        for (int m = 0; m < NFP; ++m) rec[m * stride] = vals[m];
    }
}

// Interface record of one face from the raw moments of its upwind
// distribution (shared by the face kernels)
__device__ __forceinline__ void face_record(const Geo& g, const Gas& gas, const double* M, int d, int c,
                                            const double* __restrict__ W, double* __restrict__ fp) {
    size_t stride = 2 * (size_t)g.nc;
    double* rec = fp + (size_t)d * g.nc + c;
    int L = g.nb[(2 * d) * g.nc + c];
    if (g.solid[c] || L < 0) {
        for (int m = 0; m < NFP; ++m) rec[m * stride] = 0.0;
        return;
    }
    double W0[4], q0[2];
    raw_to_macro(M, W0, q0);
    double rho, U, V, lam;
    prim_of(W0, gas.K, rho, U, V, lam);
    double tau = mu_of(gas, 1.0 / lam) / (rho / (2.0 * lam));
    double dt = fmin(g.dt[L], g.dt[c]);
    double q[5];
    time_coeffs(dt, tau, q);
    double dL = 0.5 * (d == 0 ? g.dx[L % g.nx] : g.dy[L / g.nx]);
    double dR = 0.5 * (d == 0 ? g.dx[c % g.nx] : g.dy[c / g.nx]);
    double bL[4], bR[4], aL[4], aR[4];
    for (int m = 0; m < 4; ++m) {
        bL[m] = (W0[m] - W[m * g.nc + L]) / dL / rho;
        bR[m] = (W[m * g.nc + c] - W0[m]) / dR / rho;
    }
    micro_slope(bL, U, V, lam, gas.K, aL);
    micro_slope(bR, U, V, lam, gas.K, aR);
    double sh = shakhov_prefactor(gas) * lam * lam / rho;
    double vals[NFP] = {rho, U, V, lam, sh * q0[0], sh * q0[1],
                        aL[0], aL[1], aL[2], aL[3], aR[0], aR[1], aR[2], aR[3],
                        0, 0, 0, 0,
                        q[0] / dt, q[1] / dt, q[2] / dt, q[3] / dt, q[4] / dt, 1.0};
    for (int m = 0; m < NFP; ++m) rec[m * stride] = vals[m];
}

// out[m n + i] = scale * sum_j part[(j M + m) n + i] over the nkc chunks in
// chunk order (zero where mask[i] is set); one thread per (m, i)
__global__ void k_chunk_sum(const double* __restrict__ part, int nkc, int M, int n, double scale,
                            const unsigned char* __restrict__ mask, double* __restrict__ out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * n) return;
    int m = t / n, i = t - m * n;
    double s = 0.0;
#pragma unroll 5
    for (int j = 0; j < nkc; ++j) s += part[((size_t)j * M + m) * n + i];
    out[t] = (mask && mask[i]) ? 0.0 : scale * s;
}

// Step 1: interface records of every face from the summed raw moments
// Msum[(d NRAW + m) nc + c]; one thread per (face direction, cell)
__global__ void k_face_records(Geo g, Gas gas, const double* __restrict__ Msum, const double* __restrict__ W,
                               double* __restrict__ fp) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * g.nc) return;
    int d = t / g.nc, c = t - d * g.nc;
    double M[NRAW];
    for (int m = 0; m < NRAW; ++m) M[m] = Msum[((size_t)d * NRAW + m) * g.nc + c];
    face_record(g, gas, M, d, c, W, fp);
}

// Step 1: time slope Abar of every face from the summed compatibility sums
// Ssum[(4 d + m) nc + c]; one thread per (face direction, cell)
__global__ void k_face_timeslope_records(Geo g, Gas gas, const double* __restrict__ Ssum,
                                         double* __restrict__ fp) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * g.nc) return;
    int d = t / g.nc, c = t - d * g.nc;
    size_t stride = 2 * (size_t)g.nc;
    double* rec = fp + (size_t)d * g.nc + c;
    if (rec[23 * stride] == 0.0) return;
    double rho = rec[0], U = rec[stride], V = rec[2 * stride], lam = rec[3 * stride];
    double b[4], A[4];
    for (int m = 0; m < 4; ++m) b[m] = -Ssum[((size_t)4 * d + m) * g.nc + c] / rho;
    micro_slope(b, U, V, lam, gas.K, A);
    for (int m = 0; m < 4; ++m) rec[(14 + m) * stride] = A[m];
}

// Step 1, first part: raw moments of the upwind interface distribution of
// the -x and -y faces of 64 cells over all velocities, then the interface
// records (equilibrium, Shakhov heat flux, micro-slopes, time coefficients)
template <typename T>
__global__ void __launch_bounds__(64 * FW) k_face_prep(Geo g, Vel vel, Gas gas, const T* __restrict__ f,
                                                       const double* __restrict__ W, double* __restrict__ fp) {
    __shared__ double sh[NRAW * FW * 64];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int c = blockIdx.x * 64 + lane;
    bool valid = c < g.nc;
    double a[2 * NRAW];
    for (int m = 0; m < 2 * NRAW; ++m) a[m] = 0.0;
    if (valid && !g.solid[c]) {
        for (int k = wave; k < vel.nk; k += FW) {
            double u = vel.u[k], v = vel.v[k], w = vel.w[k];
            for (int d = 0; d < 2; ++d) {
                double Gup, Hup, sG, sH;
                if (face_upwind<T, double>(g, c, d, f, vel.nk, k, d == 0 ? u : v, Gup, Hup, sG, sH))
                    raw_accumulate(a + d * NRAW, w, u, v, Gup, Hup);
            }
        }
    }
    block_sum_waves<2 * NRAW>(a, sh);
    if (wave == 0 && valid)
        for (int d = 0; d < 2; ++d) face_record(g, gas, a + d * NRAW, d, c, W, fp);
}

// G- and H-parts of (a1 + a2 u + a3 v + a4 (u^2+v^2+xi^2)/2) times the
// Maxwellian after integration over the K_int extra components
template <typename T>
__device__ __forceinline__ void slope_poly(const T* a, T u, T v, T lam, int K_int, T& pG, T& pH) {
    pG = a[0] + a[1] * u + a[2] * v + T(0.5) * a[3] * (u * u + v * v) + T(0.5) * a[3] * T(K_int) / (T(2) * lam);
    pH = pG + a[3] / (T(2) * lam);
}

// time slope Abar from the compatibility condition (discrete form):
// <Abar psi g0> = -sum_k w u_n (abar_side g0) psi
template <typename T>
__global__ void __launch_bounds__(256) k_face_timeslope_partial(Geo g, Vel vel, Gas gas,
                                                                const double* __restrict__ fp,
                                                                double* __restrict__ part, int kch) {
    __shared__ double sh[8 * WAVES * TILE];
    __shared__ double etab[EXP_TAB];   // double: the Maxwellian by Tang's exp (as the flux)
    if constexpr (sizeof(T) == 8) {
        exp_tab_fill(etab);
        __syncthreads();
    }
    Chunk ch = chunk_of(g.nc, vel.nk, kch);
    // the velocity is the same in every lane: the upwind side is a scalar branch
    const int wave = __builtin_amdgcn_readfirstlane(ch.wave);
    const int k0 = __builtin_amdgcn_readfirstlane(ch.k0), k1 = __builtin_amdgcn_readfirstlane(ch.k1);
    double a[8];
    for (int m = 0; m < 8; ++m) a[m] = 0.0;
    if (ch.valid && !g.solid[ch.c]) {
        size_t stride = 2 * (size_t)g.nc;
        // unrolled: a[4 d + m] in fixed registers (a runtime d indexed them)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const double* rec = fp + (size_t)d * g.nc + ch.c;
            if (rec[23 * stride] == 0.0) continue;
            T rho = T(rec[0]), U = T(rec[stride]), V = T(rec[2 * stride]), lam = T(rec[3 * stride]);
            T aL[4], aR[4];
            for (int m = 0; m < 4; ++m) {
                aL[m] = T(rec[(6 + m) * stride]);
                aR[m] = T(rec[(10 + m) * stride]);
            }
            T pref = rho * lam / T(M_PI);
            for (int k = k0 + wave; k < k1; k += WAVES) {
                T u = vel_u<T>(vel, k), v = vel_v<T>(vel, k);
                T un = d == 0 ? u : v;
                T du = u - U, dv = v - V;
                T G0;
                if constexpr (sizeof(T) == 8)
                    G0 = pref * exp_tab(-lam * (du * du + dv * dv), etab);
                else
                    G0 = pref * dexp(-lam * (du * du + dv * dv));
                T H0 = T(gas.K_int) / (T(2) * lam) * G0;
                T pG, pH, qG, qH;
                const int side = upwind_side(double(un));
                if (side == 0) {
                    slope_poly<T>(aL, u, v, lam, gas.K_int, pG, pH);
                } else if (side == 1) {
                    slope_poly<T>(aR, u, v, lam, gas.K_int, pG, pH);
                } else {
                    slope_poly<T>(aL, u, v, lam, gas.K_int, pG, pH);
                    slope_poly<T>(aR, u, v, lam, gas.K_int, qG, qH);
                    pG = T(0.5) * (pG + qG);
                    pH = T(0.5) * (pH + qH);
                }
                double sG = double(un) * double(pG * G0), sH = double(un) * double(pH * H0);
                double w = vel.w[k], ud = vel.u[k], vd = vel.v[k];
                a[4 * d + 0] += w * sG;
                a[4 * d + 1] += w * ud * sG;
                a[4 * d + 2] += w * vd * sG;
                a[4 * d + 3] += 0.5 * w * ((ud * ud + vd * vd) * sG + sH);
            }
        }
    }
    reduce_store<8>(a, sh, part, g.nc, ch.c, ch.valid);
}

// Step 1, second part: time slope Abar of each face from the compatibility
// condition in discrete form, over all velocities in one block
template <typename T>
__global__ void __launch_bounds__(64 * FW) k_face_timeslope(Geo g, Vel vel, Gas gas, double* __restrict__ fp) {
    __shared__ double sh[4 * FW * 64];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int c = blockIdx.x * 64 + lane;
    bool valid = c < g.nc;
    double a[8];
    for (int m = 0; m < 8; ++m) a[m] = 0.0;
    size_t stride = 2 * (size_t)g.nc;
    if (valid && !g.solid[c]) {
        for (int d = 0; d < 2; ++d) {
            const double* rec = fp + (size_t)d * g.nc + c;
            if (rec[23 * stride] == 0.0) continue;
            T rho = T(rec[0]), U = T(rec[stride]), V = T(rec[2 * stride]), lam = T(rec[3 * stride]);
            T aL[4], aR[4];
            for (int m = 0; m < 4; ++m) {
                aL[m] = T(rec[(6 + m) * stride]);
                aR[m] = T(rec[(10 + m) * stride]);
            }
            T pref = rho * lam / T(M_PI);
            for (int k = wave; k < vel.nk; k += FW) {
                T u = vel_u<T>(vel, k), v = vel_v<T>(vel, k);
                T un = d == 0 ? u : v;
                T du = u - U, dv = v - V;
                T G0 = pref * dexp(-lam * (du * du + dv * dv));
                T H0 = T(gas.K_int) / (T(2) * lam) * G0;
                T pG, pH, qG, qH;
                slope_poly<T>(un > T(0) ? aL : aR, u, v, lam, gas.K_int, pG, pH);
                if (un == T(0)) {
                    slope_poly<T>(aL, u, v, lam, gas.K_int, pG, pH);
                    slope_poly<T>(aR, u, v, lam, gas.K_int, qG, qH);
                    pG = T(0.5) * (pG + qG);
                    pH = T(0.5) * (pH + qH);
                }
                double sG = double(un) * double(pG * G0), sH = double(un) * double(pH * H0);
                double w = vel.w[k], ud = vel.u[k], vd = vel.v[k];
                a[4 * d + 0] += w * sG;
                a[4 * d + 1] += w * ud * sG;
                a[4 * d + 2] += w * vd * sG;
                a[4 * d + 3] += 0.5 * w * ((ud * ud + vd * vd) * sG + sH);
            }
        }
    }
    block_sum_waves<8>(a, sh);
    if (wave == 0 && valid && !g.solid[c])
        for (int d = 0; d < 2; ++d) {
            double* rec = fp + (size_t)d * g.nc + c;
            if (rec[23 * stride] == 0.0) continue;
            double rho = rec[0], U = rec[stride], V = rec[2 * stride], lam = rec[3 * stride];
            double b[4], A[4];
            for (int m = 0; m < 4; ++m) b[m] = -a[4 * d + m] / rho;
            micro_slope(b, U, V, lam, gas.K, A);
            for (int m = 0; m < 4; ++m) rec[(14 + m) * stride] = A[m];
        }
}

// Step 7 (and Step 6 when df != nullptr): f += df, then W and q of f, over
// all velocities in one block
template <typename T>
__global__ void __launch_bounds__(64 * FW) k_moments_full(Geo g, Vel vel, T* __restrict__ f,
                                                          const T* __restrict__ df, double* __restrict__ W,
                                                          double* __restrict__ q) {
    __shared__ double sh[6 * FW * 64];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int c = blockIdx.x * 64 + lane;
    bool valid = c < g.nc;
    double a[NRAW];
    for (int m = 0; m < NRAW; ++m) a[m] = 0.0;
    if (valid) {
        size_t nc = g.nc;
        for (int k = wave; k < vel.nk; k += FW) {
            size_t ig = (size_t)k * nc + c, ih = (size_t)(vel.nk + k) * nc + c;
            T G = f[ig], H = f[ih];
            if (df) {
                G += df[ig];
                H += df[ih];
                f[ig] = G;
                f[ih] = H;
            }
            raw_accumulate(a, vel.w[k], vel.u[k], vel.v[k], double(G), double(H));
        }
    }
    block_sum_waves<NRAW>(a, sh);
    if (wave == 0 && valid) {
        if (g.solid[c]) {
            for (int m = 0; m < 4; ++m) W[m * g.nc + c] = 0.0;
            q[c] = q[g.nc + c] = 0.0;
        } else {
            double w4[4], q2[2];
            raw_to_macro(a, w4, q2);
            for (int m = 0; m < 4; ++m) W[m * g.nc + c] = w4[m];
            q[c] = q2[0];
            q[g.nc + c] = q2[1];
        }
    }
}

__global__ void k_face_timeslope_finalize(Geo g, Gas gas, const double* __restrict__ part, int nkc,
                                          double* __restrict__ fp) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    size_t stride = 2 * (size_t)g.nc;
    for (int d = 0; d < 2; ++d) {
        double* rec = fp + (size_t)d * g.nc + c;
        if (rec[23 * stride] == 0.0) continue;
        double rho = rec[0], U = rec[stride], V = rec[2 * stride], lam = rec[3 * stride];
        double b[4], A[4];
        for (int m = 0; m < 4; ++m) {
            double s = 0.0;
            for (int j = 0; j < nkc; ++j) s += part[((size_t)j * 8 + 4 * d + m) * g.nc + c];
            b[m] = -s / rho;
        }
        micro_slope(b, U, V, lam, gas.K, A);
        for (int m = 0; m < 4; ++m) rec[(14 + m) * stride] = A[m];
    }
}

// diffuse-wall density from zero mass flux: out[j] = -sum_{u_n>0} w u_n G / den_j
// (Sec. III B); G is the first (G) plane of f or of a correction
template <typename T>
__global__ void __launch_bounds__(256) k_wall_partial(Geo g, Vel vel, const T* __restrict__ G,
                                                      double* __restrict__ part) {
    __shared__ double sh[WAVES * TILE];
    Chunk ch = chunk_of(g.n_wall, vel.nk);
    double a[1] = {0.0};
    if (ch.valid) {
        int j = ch.c, c = g.w_cell[j], s = g.w_side[j];
        double sign = (s & 1) ? 1.0 : -1.0;
        for (int k = ch.k0 + ch.wave; k < ch.k1; k += WAVES) {
            double un = sign * (s < 2 ? vel.u[k] : vel.v[k]);
            if (un > 0) a[0] += vel.w[k] * un * double(G[(size_t)k * g.nc + c]);
        }
    }
    reduce_store<1>(a, sh, part, g.n_wall, ch.c, ch.valid);
}

__global__ void k_wall_finalize(Geo g, const double* __restrict__ part, int nkc, double* __restrict__ out) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.n_wall) return;
    double s = 0.0;
    for (int i = 0; i < nkc; ++i) s += part[(size_t)i * g.n_wall + j];
    out[j] = -s / g.w_den[j];
}

// The velocity-independent parts of an interface record, formed once per
// face: the Maxwellian prefactor, K_int/(2 lam), and each micro-slope as
// a0' + a1 u + a2 v + a3 (u^2 + v^2)/2 for G with a0' = a0 + a3 K_int/(4 lam),
// plus a3/(2 lam) for H (the slope polynomials of slope_poly)
template <typename T>
struct FaceConst {
    T pre, U, V, lam, shx, shy, hK;
    T a[3][4];   // left, right and time slopes, constant term folded
    T dH[3];
    T q[5];
    T lam2;      // 2 lam
    T q1dH[2];   // q1 dH of the left and right slopes
    T q2dH2;     // q2 dH of the time slope
};

template <typename T>
__device__ __forceinline__ void face_const(const T* P, int K_int, FaceConst<T>& F) {
    T lam = P[3];
    T inv2l = T(1) / (T(2) * lam);
    F.pre = P[0] * lam / T(M_PI);
    F.U = P[1];
    F.V = P[2];
    F.lam = lam;
    F.shx = P[4];
    F.shy = P[5];
    F.hK = T(K_int) * inv2l;
    for (int i = 0; i < 3; ++i) {
        const T* a = P + 6 + 4 * i;
        F.a[i][0] = a[0] + T(0.5) * a[3] * F.hK;
        F.a[i][1] = a[1];
        F.a[i][2] = a[2];
        F.a[i][3] = T(0.5) * a[3];
        F.dH[i] = a[3] * inv2l;
    }
    for (int m = 0; m < 5; ++m) F.q[m] = P[18 + m];
    F.lam2 = T(2) * lam;
    F.q1dH[0] = F.q[1] * F.dH[0];
    F.q1dH[1] = F.q[1] * F.dH[1];
    F.q2dH2 = F.q[2] * F.dH[2];
}

// UGKS time-averaged flux of G and H through an interior face for one
// velocity, normal pointing from L to R (Sec. II A 1; see the interface record)
template <typename T>
__device__ __forceinline__ void face_flux(const FaceConst<T>& F, T u, T v, T un, T Gup, T Hup, T sGup, T sHup,
                                          T& PG, T& PH) {
    T cx = u - F.U, cy = v - F.V, c2 = cx * cx + cy * cy;
    T G0 = F.pre * dexp(-F.lam * c2);
    T H0 = F.hK * G0;
    T sk = F.shx * cx + F.shy * cy;
    T Geq = G0 * (T(1) + sk * (T(2) * F.lam * c2 - T(4)));
    T Heq = H0 * (T(1) + sk * (T(2) * F.lam * c2 - T(2)));
    T q2 = u * u + v * v;
    const int side = un > T(0) ? 0 : 1;
    T aG = F.a[side][0] + F.a[side][1] * u + F.a[side][2] * v + F.a[side][3] * q2;
    T aH = aG + F.dH[side];
    T bG = F.a[2][0] + F.a[2][1] * u + F.a[2][2] * v + F.a[2][3] * q2;
    T bH = bG + F.dH[2];
    PG = un * (F.q[0] * Geq + F.q[1] * un * aG * G0 + F.q[2] * bG * G0 + F.q[3] * Gup + F.q[4] * un * sGup);
    PH = un * (F.q[0] * Heq + F.q[1] * un * aH * H0 + F.q[2] * bH * H0 + F.q[3] * Hup + F.q[4] * un * sHup);
}

// face_flux with the upwind side known for the whole wavefront (side 0 or
// 1; a face with zero normal velocity carries no flux), the Maxwellian by
// exp_tab.  The same terms as face_flux, grouped so that G and H share them:
// with H0 = hK G0, Heq = hK G0 (1 + sk (2 lam c2 - 4) + 2 sk), and the H
// slopes those of G plus dH,
//   PG = un (q0 Geq + G0 (q1 un aG + q2 bG) + q3 Gup + q4 un sGup)
//   PH = un (hK (q0 Heq/hK + G0 (q1 un aG + q2 bG + un q1 dH_s + q2 dH_t))
//            + q3 Hup + q4 un sHup)
template <typename T>
__device__ __forceinline__ void face_flux_side(const FaceConst<T>& F, int side, T u, T v, T un, T Gup, T Hup,
                                               T sGup, T sHup, const double* __restrict__ etab, T& PG, T& PH) {
    const T cx = u - F.U, cy = v - F.V, c2 = cx * cx + cy * cy;
    const T G0 = F.pre * T(exp_tab(double(-F.lam * c2), etab));
    const T sk = F.shx * cx + F.shy * cy;
    const T eG = T(1) + sk * (F.lam2 * c2 - T(4));
    const T Geq = G0 * eG, HeqK = G0 * (eG + (sk + sk));   // Heq / hK
    const T q2 = u * u + v * v;
    // (side is uniform: a scalar branch, and the slopes stay in registers)
    T aG, qdH;
    if (side == 0) {
        aG = F.a[0][0] + F.a[0][1] * u + F.a[0][2] * v + F.a[0][3] * q2;
        qdH = F.q1dH[0];
    } else {
        aG = F.a[1][0] + F.a[1][1] * u + F.a[1][2] * v + F.a[1][3] * q2;
        qdH = F.q1dH[1];
    }
    const T bG = F.a[2][0] + F.a[2][1] * u + F.a[2][2] * v + F.a[2][3] * q2;
    const T t1 = F.q[1] * un, t4 = F.q[4] * un;
    const T inG = t1 * aG + F.q[2] * bG;
    const T inH = inG + (un * qdH + F.q2dH2);
    PG = un * (F.q[0] * Geq + G0 * inG + F.q[3] * Gup + t4 * sGup);
    PH = un * (F.hK * (F.q[0] * HeqK + G0 * inH) + F.q[3] * Hup + t4 * sHup);
}

// Step 1: div_ik = (1/V_i) sum_faces S u_n ftilde (outward) for G and H, and
// partial sums of the macroscopic residual R_i = -sum_k w psi div_ik.  The
// flux arithmetic runs in double on the stored (T) distribution: R is a
// difference of fluxes scaled by S/V, and single-precision products would
// leave ~1e-6 of rounding noise in it; div is stored in T.
//
// A block is a tile of cells (lanes) by a chunk of KCHF velocities, wave w
// taking velocities k0 + w + WAVES j.  The velocity is the same in every
// lane, so the upwind side of a face is a scalar branch, the stencil loads
// take scalar row offsets, and a thread's MKF velocities are unrolled into
// registers.
//
// A cell's +x face is the -x face of the next cell: every interior +x face
// flux is handed down a lane rather than formed again (a quarter fewer face
// evaluations).  Tiles step by tstride cells (flux_stride): 64 when rows
// pack whole into a tile (64 mod nx = 0, so a tile's last cell ends a row);
// otherwise 63, and lane 63 forms only the -x face flux of the next tile's
// first cell, for lane 62.
//
// MKF velocities per thread (16 or 24, against the other kernels' 8): the
// 23-word face records and the stencil set-up of each face are loaded once
// per MKF velocities, and the chunk partials of R shrink.  The velocity loops
// run as unrolled groups of 8 (a single loop of 16 is left rolled by the
// compiler, which then reaches the running sums by indexed register moves).
// Registers: 216 (float, 16), 250 (float, 24), 228 (double, 16): two
// wavefronts per SIMD; double with 24 would not fit.  flux_mk picks 24 for
// float where the launch keeps 4096 blocks with it; force (16, or 24 for
// float; MIUGKS_FLUX_MK) overrides the choice.
inline int flux_mk(bool is_float, int ntiles, int nk, int force = 0) {
    if (force == 16 || (force == 24 && is_float)) return force;
    return is_float && (long)ntiles * ((nk + WAVES * 24 - 1) / (WAVES * 24)) >= 4096 ? 24 : 16;
}

template <typename T, int MKF>
__global__ void __launch_bounds__(256) k_flux_div(Geo g, Vel vel, Gas gas, const T* __restrict__ f,
                                                  const double* __restrict__ fp,
                                                  const double* __restrict__ rho_w,
                                                  const T* __restrict__ finf, T* __restrict__ div,
                                                  double* __restrict__ part, int tstride) {
    typedef double A;
    constexpr int KCHF = WAVES * MKF;   // velocities per chunk
    __shared__ double sh[4 * WAVES * TILE];
    __shared__ double etab[EXP_TAB];
    exp_tab_fill(etab);
    __syncthreads();
    // XCD-contiguous logical blocks: each XCD takes whole velocity chunks,
    // so the rows of a tile's y-stencil are read by tiles of the same L2
    const int nt = gridDim.x, nb = gridDim.x * gridDim.y;
    const int Lb = xcd_swizzle(blockIdx.x + nt * blockIdx.y, nb);
    const int tile = Lb % nt, chunk = Lb / nt;
    const int lane = threadIdx.x & (TILE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / TILE);
    const int nk = vel.nk, k0 = chunk * KCHF, k1 = min(nk, k0 + KCHF);
    // this wave's velocities k0 + wave + WAVES j, j < nmine
    const int nmine = k1 - k0 > wave ? (k1 - k0 - wave + WAVES - 1) / WAVES : 0;
    const int c = tile * tstride + lane;
    const bool valid = c < g.nc, own = valid && lane < tstride;
    const size_t nc = g.nc, ho = (size_t)nk * nc;
    const unsigned rowb = (unsigned)(nc * sizeof(T));
    const unsigned chunkb = (unsigned)(k1 - k0) * rowb;
    const __amdgpu_buffer_rsrc_t RG = buf_rsrc(f + (size_t)k0 * nc, chunkb);
    const __amdgpu_buffer_rsrc_t RH = buf_rsrc(f + ho + (size_t)k0 * nc, chunkb);
    const unsigned so0 = (unsigned)wave * rowb, sostep = (unsigned)WAVES * rowb;
    double acc[4] = {0, 0, 0, 0};
    A dG[MKF], dH[MKF];
#pragma unroll
    for (int j = 0; j < MKF; ++j) dG[j] = dH[j] = A(0);
    if (valid && !g.solid[c]) {
        const int ix = c % g.nx, iy = c / g.nx;
        const unsigned oc = (unsigned)c * sizeof(T);
        // The -x side first.  Its face is also the +x face of the cell on
        // the left, the previous lane's: the face flux is formed once and
        // handed down a lane.  (An interior neighbour is a fluid cell whose
        // face across is interior too, so the lane on the right forms it;
        // with 64-cell tiles, lane 63's +x side ends a row.)
        const A sv_x = A(1.0 / g.dx[ix]);
        const bool take1 = g.nb[g.nc + c] == c + 1 && lane < TILE - 1;
        {
            const int code = g.nb[c];
            FaceConst<A> FC;
            FaceStencil<T> st;
            FaceVals<T> cur{}, nxt{};
            A lam = A(1), Uw = A(0), Vw = A(0), rw = A(0);
            const bool far = code == NB_FARFIELD, sym = code == NB_SYMMETRY, wall = is_wall(code);
            if (code >= 0) {
                const double* rec = fp + c;
                const size_t stride = 2 * nc;
                A P[23];
                for (int m = 0; m < 23; ++m) P[m] = A(rec[m * stride]);
                face_const<A>(P, gas.K_int, FC);
                face_stencil<T>(g, c, 0, st);
                if (nmine > 0) stencil_load<T>(st, RG, RH, so0, nxt);
            } else if (wall) {
                const int jw = wall_of(code);
                lam = A(1.0 / g.w_T[jw]);
                Uw = A(g.w_U[jw]);
                Vw = A(g.w_V[jw]);
                rw = A(rho_w[jw]);
            }
#pragma unroll
            for (int jh = 0; jh < MKF; jh += 8)
#pragma unroll
                for (int j = jh; j < jh + 8; ++j) {
                if (j >= nmine) break;
                const int k = k0 + wave + WAVES * j;
                const unsigned so = so0 + j * sostep;
                const A u = vel.u[k], v = vel.v[k];
                const int side = upwind_side(u);
                A PG = A(0), PH = A(0);
                if (code >= 0) {
                    cur = nxt;
                    if (j + 1 < nmine) stencil_load<T>(st, RG, RH, so + sostep, nxt);
                    if (side != 2) {
                        T Gu, Hu, sGt, sHt;
                        upwind_on_side<T>(st, cur, side, Gu, Hu, sGt, sHt);
                        face_flux_side<A>(FC, side, u, v, u, A(Gu), A(Hu), A(sGt), A(sHt), etab, PG, PH);
                    }
                    dG[j] += A(-1) * sv_x * PG;
                    dH[j] += A(-1) * sv_x * PH;
                } else {
                    const A un = A(-1) * u;
                    A Gf, Hf;
                    if (wall && !(un > A(0))) {
                        const A du = u - Uw, dv = v - Vw;
                        const A C = lam / A(M_PI) * dexp(-lam * (du * du + dv * dv));
                        Gf = rw * C;
                        Hf = rw * A(gas.K_int) / (A(2) * lam) * C;
                    } else if (far && un <= A(0)) {
                        Gf = A(finf[k]);
                        Hf = A(finf[nk + k]);
                    } else if (sym && un <= A(0)) {
                        const int km = mirror_of(vel, 0, k);
                        Gf = A(f[(size_t)km * nc + c]);
                        Hf = A(f[ho + (size_t)km * nc + c]);
                    } else {
                        Gf = A(buf_ld<T>(RG, oc, so));
                        Hf = A(buf_ld<T>(RH, oc, so));
                    }
                    dG[j] += sv_x * un * Gf;
                    dH[j] += sv_x * un * Hf;
                }
                // the +x side: the face flux of the lane on the right
                const A nG = __shfl_down(PG, 1, TILE), nH = __shfl_down(PH, 1, TILE);
                if (take1) {
                    dG[j] += A(1) * sv_x * nG;
                    dH[j] += A(1) * sv_x * nH;
                }
            }
        }
        for (int s = 1; s < 4 && own; ++s) {
            if (s == 1 && take1) continue;
            const int code = g.nb[s * g.nc + c];
            const int d = s >> 1;
            const A sign = (s & 1) ? A(1) : A(-1);
            const A sv = A(1.0 / (d == 0 ? g.dx[ix] : g.dy[iy]));   // S / V
            if (code >= 0) {
                // face record: the -d face of the cell on the positive side
                const int R = (s & 1) ? code : c;
                const double* rec = fp + (size_t)d * g.nc + R;
                const size_t stride = 2 * nc;
                A P[23];
                for (int m = 0; m < 23; ++m) P[m] = A(rec[m * stride]);
                FaceConst<A> FC;
                face_const<A>(P, gas.K_int, FC);
                FaceStencil<T> st;
                face_stencil<T>(g, R, d, st);
                // the stencil values of the next velocity load while this one computes
                FaceVals<T> cur{}, nxt{};
                if (nmine > 0) stencil_load<T>(st, RG, RH, so0, nxt);
#pragma unroll
                for (int jh = 0; jh < MKF; jh += 8)
#pragma unroll
                    for (int j = jh; j < jh + 8; ++j) {
                    if (j >= nmine) break;
                    const int k = k0 + wave + WAVES * j;
                    const unsigned so = so0 + j * sostep;
                    cur = nxt;
                    if (j + 1 < nmine) stencil_load<T>(st, RG, RH, so + sostep, nxt);
                    const A u = vel.u[k], v = vel.v[k];
                    const A un = d == 0 ? u : v;
                    const int side = upwind_side(un);
                    if (side != 2) {
                        T Gu, Hu, sGt, sHt;
                        upwind_on_side<T>(st, cur, side, Gu, Hu, sGt, sHt);
                        A PG, PH;
                        face_flux_side<A>(FC, side, u, v, un, A(Gu), A(Hu), A(sGt), A(sHt), etab, PG, PH);
                        dG[j] += sign * sv * PG;
                        dH[j] += sign * sv * PH;
                    }
                }
            } else if (is_wall(code)) {
                const int jw = wall_of(code);
                const A lam = A(1.0 / g.w_T[jw]), Uw = A(g.w_U[jw]), Vw = A(g.w_V[jw]);
                const A rw = A(rho_w[jw]);
#pragma unroll
                for (int jh = 0; jh < MKF; jh += 8)
#pragma unroll
                    for (int j = jh; j < jh + 8; ++j) {
                    if (j >= nmine) break;
                    const int k = k0 + wave + WAVES * j;
                    const A u = vel.u[k], v = vel.v[k];
                    const A un = sign * (d == 0 ? u : v);
                    A Gf, Hf;
                    if (un > A(0)) {
                        Gf = A(buf_ld<T>(RG, oc, so0 + j * sostep));
                        Hf = A(buf_ld<T>(RH, oc, so0 + j * sostep));
                    } else {
                        const A du = u - Uw, dv = v - Vw;
                        const A C = lam / A(M_PI) * dexp(-lam * (du * du + dv * dv));
                        Gf = rw * C;
                        Hf = rw * A(gas.K_int) / (A(2) * lam) * C;
                    }
                    dG[j] += sv * un * Gf;
                    dH[j] += sv * un * Hf;
                }
            } else {
                const bool far = code == NB_FARFIELD, sym = code == NB_SYMMETRY;
#pragma unroll
                for (int jh = 0; jh < MKF; jh += 8)
#pragma unroll
                    for (int j = jh; j < jh + 8; ++j) {
                    if (j >= nmine) break;
                    const int k = k0 + wave + WAVES * j;
                    const A un = sign * (d == 0 ? A(vel.u[k]) : A(vel.v[k]));
                    A Gf, Hf;
                    if (far && un <= A(0)) {
                        Gf = A(finf[k]);
                        Hf = A(finf[nk + k]);
                    } else if (sym && un <= A(0)) {
                        // specular reflection: the cell's own value at the mirror velocity
                        const int km = mirror_of(vel, d, k);
                        Gf = A(f[(size_t)km * nc + c]);
                        Hf = A(f[ho + (size_t)km * nc + c]);
                    } else {
                        Gf = A(buf_ld<T>(RG, oc, so0 + j * sostep));
                        Hf = A(buf_ld<T>(RH, oc, so0 + j * sostep));
                    }
                    dG[j] += sv * un * Gf;
                    dH[j] += sv * un * Hf;
                }
            }
        }
    }
    if (own) {
#pragma unroll
        for (int jh = 0; jh < MKF; jh += 8)
#pragma unroll
            for (int j = jh; j < jh + 8; ++j) {
            if (j >= nmine) break;
            const int k = k0 + wave + WAVES * j;
            div[(size_t)k * nc + c] = T(dG[j]);
            div[ho + (size_t)k * nc + c] = T(dH[j]);
            const double w = vel.w[k], u = vel.u[k], v = vel.v[k];
            const double gd = double(dG[j]), hd = double(dH[j]);
            acc[0] += w * gd;
            acc[1] += w * u * gd;
            acc[2] += w * v * gd;
            acc[3] += 0.5 * w * ((u * u + v * v) * gd + hd);
        }
    }
    reduce_store<4>(acc, sh, part, g.nc, c, own, chunk);
}

// tile stride of k_flux_div and its blocks along the cells
inline int flux_stride(const Geo& g) { return TILE % g.nx == 0 ? TILE : TILE - 1; }
inline int flux_tiles(const Geo& g) { return (g.nc + flux_stride(g) - 1) / flux_stride(g); }

// outward flux u_n ftilde through the non-interior side s (code < 0) of a
// fluid cell c for velocity k: at a wall the outgoing f and the incoming
// rho_w C_k, at a farfield side the incoming freestream, at a symmetry side
// the incoming mirror-velocity value, else f
template <typename T, typename A>
__device__ __forceinline__ void boundary_flux(const Geo& g, const Vel& vel, const Gas& gas, const T* __restrict__ f,
                                              const double* __restrict__ rho_w, const T* __restrict__ finf, int c,
                                              int s, int code, int k, A& oG, A& oH) {
    const size_t nc = g.nc, ho = (size_t)vel.nk * nc;
    int d = s >> 1;
    A sign = (s & 1) ? A(1) : A(-1);
    A u = vel.u[k], v = vel.v[k];
    A un = sign * (d == 0 ? u : v);
    A Gf, Hf;
    if (is_wall(code) && !(un > A(0))) {
        int jw = wall_of(code);
        A lam = A(1.0 / g.w_T[jw]), du = u - A(g.w_U[jw]), dv = v - A(g.w_V[jw]);
        A C = lam / A(M_PI) * dexp(-lam * (du * du + dv * dv));
        A rw = A(rho_w[jw]);
        Gf = rw * C;
        Hf = rw * A(gas.K_int) / (A(2) * lam) * C;
    } else if (code == NB_FARFIELD && un <= A(0)) {
        Gf = A(finf[k]);
        Hf = A(finf[vel.nk + k]);
    } else if (code == NB_SYMMETRY && un <= A(0)) {
        int km = mirror_of(vel, d, k);
        Gf = A(f[(size_t)km * nc + c]);
        Hf = A(f[ho + (size_t)km * nc + c]);
    } else {
        Gf = A(f[(size_t)k * nc + c]);
        Hf = A(f[ho + (size_t)k * nc + c]);
    }
    oG = un * Gf;
    oH = un * Hf;
}

__global__ void k_residual_finalize(Geo g, const double* __restrict__ part, int nkc, double* __restrict__ R) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    for (int m = 0; m < 4; ++m) {
        double s = 0.0;
        for (int j = 0; j < nkc; ++j) s += part[((size_t)j * 4 + m) * g.nc + c];
        R[m * g.nc + c] = g.solid[c] ? 0.0 : -s;
    }
}

// RMS residual of each conservative variable over fluid cells (Sec. IV A), one block
__global__ void k_residual_norm(Geo g, int n_fluid, const double* __restrict__ R, double* __restrict__ out) {
    __shared__ double sh[4][256];
    double s[4] = {0, 0, 0, 0};
    for (int c = threadIdx.x; c < g.nc; c += blockDim.x)
        if (!g.solid[c])
            for (int m = 0; m < 4; ++m) {
                double r = R[m * g.nc + c];
                s[m] += r * r;
            }
    for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] = s[m];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] += sh[m][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = sqrt(sh[threadIdx.x][0] / n_fluid);
}

// ---------------------------------------------------------------------------
// Steps 3-4: predicted Shakhov equilibrium and micro residual

// positivity guard, then per-cell record {rho lam/pi, U, V, lam, shx, shy, 1/tau}
__global__ void k_cell_prep(Geo g, Gas gas, double* __restrict__ Wt, const double* __restrict__ Wn,
                            const double* __restrict__ q, double* __restrict__ cp, double* __restrict__ tau_inv) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    if (g.solid[c]) {
        for (int m = 0; m < NCP; ++m) cp[m * g.nc + c] = 0.0;
        tau_inv[c] = 0.0;
        return;
    }
    double w[4];
    for (int m = 0; m < 4; ++m) w[m] = Wt[m * g.nc + c];
    double rho, U, V, lam;
    prim_of(w, gas.K, rho, U, V, lam);
    if (!(rho > 0.0) || !(lam > 0.0) || !isfinite(lam)) {
        for (int m = 0; m < 4; ++m) Wt[m * g.nc + c] = w[m] = Wn[m * g.nc + c];
        prim_of(w, gas.K, rho, U, V, lam);
    }
    double ti = (rho / (2.0 * lam)) / mu_of(gas, 1.0 / lam);
    double sh = shakhov_prefactor(gas) * lam * lam / rho;
    double vals[NCP] = {rho * lam / M_PI, U, V, lam, sh * q[c], sh * q[g.nc + c], ti};
    for (int m = 0; m < NCP; ++m) cp[m * g.nc + c] = vals[m];
    tau_inv[c] = ti;
}

template <typename T>
__global__ void __launch_bounds__(256) k_micro_residual(Geo g, Vel vel, Gas gas, const T* __restrict__ f,
                                                        const T* __restrict__ div,
                                                        const double* __restrict__ cp, T* __restrict__ r) {
    Chunk ch = chunk_of(g.nc, vel.nk);
    if (!ch.valid) return;
    int c = ch.c;
    size_t nc = g.nc, ho = (size_t)vel.nk * nc;
    bool fluid = !g.solid[c];
    T pref = T(cp[c]), U = T(cp[nc + c]), V = T(cp[2 * nc + c]), lam = T(cp[3 * nc + c]);
    T shx = T(cp[4 * nc + c]), shy = T(cp[5 * nc + c]), ti = T(cp[6 * nc + c]);
    for (int k = ch.k0 + ch.wave; k < ch.k1; k += WAVES) {
        size_t ig = (size_t)k * nc + c;
        if (!fluid) {
            r[ig] = T(0);
            r[ho + ig] = T(0);
            continue;
        }
        T u = vel_u<T>(vel, k), v = vel_v<T>(vel, k);
        T cx = u - U, cy = v - V, c2 = cx * cx + cy * cy;
        T G0 = pref * dexp(-lam * c2);
        T H0 = T(gas.K_int) / (T(2) * lam) * G0;
        T sk = shx * cx + shy * cy;
        T Gt = G0 * (T(1) + sk * (T(2) * lam * c2 - T(4)));
        T Ht = H0 * (T(1) + sk * (T(2) * lam * c2 - T(2)));
        r[ig] = (Gt - f[ig]) * ti - div[ig];
        r[ho + ig] = (Ht - f[ho + ig]) * ti - div[ho + ig];
    }
}

// ---------------------------------------------------------------------------
// Explicit, time-accurate UGKS (the scheme the paper's residuals come from):
// one global step dt, the interface fluxes integrated over it.

// out = W + dt R on every fluid cell (the macroscopic update), W elsewhere
__global__ void k_macro_step(Geo g, const double* __restrict__ W, const double* __restrict__ R, double dt,
                             double* __restrict__ out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * g.nc) return;
    int c = t % g.nc;
    out[t] = g.solid[c] ? W[t] : W[t] + dt * R[t];
}

// f = [f - dt div + dt/2 (g1/tau1 + (g0 - f)/tau0)] / (1 + dt/(2 tau1)): the
// trapezoidal collision term with the Shakhov equilibria g0 of W^n and g1 of
// the updated W (both with the heat flux q^n; cell records of k_cell_prep)
template <typename T>
__global__ void __launch_bounds__(256) k_explicit_update(Geo g, Vel vel, Gas gas, T* __restrict__ f,
                                                         const T* __restrict__ div, const double* __restrict__ cp0,
                                                         const double* __restrict__ cp1, double dt) {
    Chunk ch = chunk_of(g.nc, vel.nk);
    if (!ch.valid) return;
    const int c = ch.c;
    const size_t nc = g.nc, ho = (size_t)vel.nk * nc;
    const bool fluid = !g.solid[c];
    double P0[NCP], P1[NCP];
    for (int m = 0; m < NCP; ++m) {
        P0[m] = cp0[m * nc + c];
        P1[m] = cp1[m * nc + c];
    }
    auto shakhov = [&](const double* P, double u, double v, double& G, double& H) {
        double cx = u - P[1], cy = v - P[2], c2 = cx * cx + cy * cy, lam = P[3];
        double G0 = P[0] * exp(-lam * c2);
        double H0 = double(gas.K_int) / (2.0 * lam) * G0;
        double sk = P[4] * cx + P[5] * cy;
        G = G0 * (1.0 + sk * (2.0 * lam * c2 - 4.0));
        H = H0 * (1.0 + sk * (2.0 * lam * c2 - 2.0));
    };
    const double den = 1.0 / (1.0 + 0.5 * dt * P1[6]);
    for (int k = ch.k0 + ch.wave; k < ch.k1; k += WAVES) {
        size_t ig = (size_t)k * nc + c;
        if (!fluid) {
            f[ig] = T(0);
            f[ho + ig] = T(0);
            continue;
        }
        double u = vel.u[k], v = vel.v[k], G0, H0, G1, H1;
        shakhov(P0, u, v, G0, H0);
        shakhov(P1, u, v, G1, H1);
        double fG = f[ig], fH = f[ho + ig];
        fG = (fG - dt * double(div[ig]) + 0.5 * dt * (G1 * P1[6] + (G0 - fG) * P0[6])) * den;
        fH = (fH - dt * double(div[ho + ig]) + 0.5 * dt * (H1 * P1[6] + (H0 - fH) * P0[6])) * den;
        f[ig] = T(fG);
        f[ho + ig] = T(fH);
    }
}

// ---------------------------------------------------------------------------
// Step 5: correction equation (Sec. II A 2) on one level.

// transport part of the diagonal D_ik (outgoing normal speeds over the
// sides; an outflow side adds its inflow speed as well)
template <typename T>
__device__ __forceinline__ T transport_diag(const Geo& g, int c, T u, T v) {
    T invx = T(1.0 / g.dx[c % g.nx]), invy = T(1.0 / g.dy[c / g.nx]);
    T D = T(0);
    for (int s = 0; s < 4; ++s) {
        T un = ((s & 1) ? T(1) : T(-1)) * (s < 2 ? u : v);
        T a = g.nb[s * g.nc + c] == NB_OUTFLOW ? un : (un > T(0) ? un : T(0));
        D += a * (s < 2 ? invx : invy);
    }
    return D;
}

// D_jk times the correction across the upwind side s of cell c (the side
// with negative normal speed): neighbour value or, at a symmetry side, the
// cell's own at the mirror velocity (passed in), wall ghost C_k drho_w, or
// zero (farfield; outflow lives on the diagonal)
template <typename T>
__device__ __forceinline__ void upwind_term(const Geo& g, int c, int s, T u, T v, int K_int, T nbG, T nbH,
                                            const double* __restrict__ drho, T& tG, T& tH) {
    int code = g.nb[s * g.nc + c];
    T un = ((s & 1) ? T(1) : T(-1)) * (s < 2 ? u : v);
    T coef = (un < T(0) ? un : T(0)) * T(1.0 / (s < 2 ? g.dx[c % g.nx] : g.dy[c / g.nx]));
    if (code >= 0 || code == NB_SYMMETRY) {   // neighbour, or the cell's own at the mirror velocity
        tG = coef * nbG;
        tH = coef * nbH;
    } else if (is_wall(code)) {
        int j = wall_of(code);
        T lam = T(1.0 / g.w_T[j]);
        T du = u - T(g.w_U[j]), dv = v - T(g.w_V[j]);
        T C = lam / T(M_PI) * dexp(-lam * (du * du + dv * dv));
        T dr = T(drho[j]);
        tG = coef * C * dr;
        tH = coef * T(K_int) / (T(2) * lam) * C * dr;
    } else {
        tG = T(0);
        tH = T(0);
    }
}

// Side types packed per cell for the sweeps: 2 bits per side (0 interior,
// 1 wall, 2 farfield, 3 outflow), bit 8 = solid cell, bits 9-31 = index of
// the cell's first wall side in the level's wall list (the wall sides of a
// cell are listed consecutively in side order).
constexpr unsigned FLAG_SOLID = 0x100;
constexpr int FLAG_WALL_SHIFT = 9;

__device__ __forceinline__ int side_type(unsigned fl, int s) { return (fl >> (2 * s)) & 3; }

// wall-list index of side s of a cell whose flags are fl (side s is a wall)
__device__ __forceinline__ int wall_index_fl(unsigned fl, int s) {
    int j = (int)(fl >> FLAG_WALL_SHIFT);
    for (int q = 0; q < s; ++q) j += side_type(fl, q) == 1;
    return j;
}

// transport part of D_ik from the packed side types
template <typename T>
__device__ __forceinline__ T transport_diag_fl(unsigned fl, T u, T v, T invdx, T invdy) {
    T D = T(0);
    for (int s = 0; s < 4; ++s) {
        T un = ((s & 1) ? T(1) : T(-1)) * (s < 2 ? u : v);
        T a = side_type(fl, s) == 3 ? un : (un > T(0) ? un : T(0));
        D += a * (s < 2 ? invdx : invdy);
    }
    return D;
}

// wall ghost C_k drho_w of the G (part 0) or H (part 1) correction at wall j
template <typename T>
__device__ __forceinline__ T wall_ghost_j(const Geo& g, int j, T u, T v, int K_int, int part,
                                          const double* __restrict__ drho) {
    T lam = T(1.0 / g.w_T[j]);
    T du = u - T(g.w_U[j]), dv = v - T(g.w_V[j]);
    T C = lam / T(M_PI) * dexp(-lam * (du * du + dv * dv));
    if (part) C *= T(K_int) / (T(2) * lam);
    return C * T(drho[j]);
}

// After a sweep: w_k u_n dG_k at every wall side for this velocity (zero for
// u_n <= 0), the per-velocity terms of the next wall densities, stored
// velocity-major: wbuf[k][j] (the per-velocity partial sums of k_drho)
template <typename T>
__device__ __forceinline__ void wall_products(const Geo& g, const Vel& vel, int k, const T* Gk,
                                              double* __restrict__ wbuf, int tid, int nthr) {
    double u = vel.u[k], v = vel.v[k], w = vel.w[k];
    for (int j = tid; j < g.n_wall; j += nthr) {
        int s = g.w_side[j];
        double un = ((s & 1) ? 1.0 : -1.0) * (s < 2 ? u : v);
        wbuf[(size_t)k * g.n_wall + j] = un > 0.0 ? w * un * double(Gk[g.w_cell[j]]) : 0.0;
    }
}

// Copy n elements between global memory and LDS with every thread keeping
// four 16-byte accesses in flight (the tiles are latency-bound otherwise);
// element counts that are not a multiple of the vector width finish
// element by element.
template <typename T>
__device__ __forceinline__ void bulk_copy(T* __restrict__ dst, const T* __restrict__ src, int n) {
    constexpr int V = 16 / sizeof(T);
    typedef __attribute__((ext_vector_type(V))) T vec;
    int tid = threadIdx.x, nthr = blockDim.x;
    bool aligned = ((((size_t)dst) | ((size_t)src)) & 15) == 0;
    int nv = aligned ? n / V : 0;
    const vec* s = (const vec*)src;
    vec* d = (vec*)dst;
    int i = tid;
    for (; i + 3 * nthr < nv; i += 4 * nthr) {
        vec a = s[i], b = s[i + nthr], c = s[i + 2 * nthr], e = s[i + 3 * nthr];
        d[i] = a;
        d[i + nthr] = b;
        d[i + 2 * nthr] = c;
        d[i + 3 * nthr] = e;
    }
    for (; i < nv; i += nthr) d[i] = s[i];
    for (int j = nv * V + tid; j < n; j += nthr) dst[j] = src[j];
}

// One Gauss-Seidel sweep of every velocity in its own upwind order (the
// LU-SGS sweep of Sec. II A 2 taken along the direction of each velocity),
// staged in LDS.  A block runs P pipelines side by side; pipeline p sweeps
// item blockIdx.x * P + p, item = 2 k + part (G or H of velocity k), and the
// per-cell data (1/tau + 1/dt_n, side flags, 1/dx) is shared by the P tiles.
// Thread t of a pipeline owns row t (counted from the upwind y-side) and
// updates column s - t at step s, so both upwind neighbours were written one
// step earlier (one barrier per step); the thread keeps its own previous
// cell in a register and reads the one below it from LDS, and it loads the
// data of its next cell before the barrier.  The tile holds r and is
// overwritten by the correction, which needs no initial value.  Wall ghosts
// use the wall densities of the correction before the sweep, evaluated per
// item before the first step.
template <typename T>
__global__ void k_sweep_lds(Geo g, Vel vel, int K_int, const T* __restrict__ r, T* __restrict__ df,
                            const double* __restrict__ tau_inv, const double* __restrict__ dtn_inv,
                            const unsigned* __restrict__ flags_g, const double* __restrict__ drho,
                            double* __restrict__ wbuf, int npad, int P) {
    extern __shared__ double smem_d[];
    int nc = g.nc, nx = g.nx, ny = g.ny, nw = g.n_wall;
    T* tiles = (T*)smem_d;                 // [P][nc]
    T* coef = tiles + (size_t)P * nc;      // [nc]  1/tau + 1/dt_n
    T* invdx = coef + nc;                  // [nx]
    T* ghosts = invdx + nx;                // [P][n_wall]
    unsigned* flags = (unsigned*)(ghosts + (size_t)P * nw);   // [nc]
    int tid = threadIdx.x, nthr = blockDim.x;
    int nitems = 2 * vel.nk;
    int item0 = blockIdx.x * P;
    for (int i = tid; i < nc; i += nthr) {
        coef[i] = T(tau_inv[i] + dtn_inv[i]);
        flags[i] = flags_g[i];
    }
    for (int i = tid; i < nx; i += nthr) invdx[i] = T(1.0 / g.dx[i]);
    for (int q = 0; q < P; ++q) {
        int item = item0 + q;
        if (item >= nitems) break;
        int k = item >> 1, part = item & 1;
        bulk_copy<T>(tiles + (size_t)q * nc, r + ((size_t)part * vel.nk + k) * nc, nc);
        T u = vel_u<T>(vel, k), v = vel_v<T>(vel, k);
        for (int j = tid; j < nw; j += nthr)
            ghosts[(size_t)q * nw + j] = wall_ghost_j<T>(g, j, u, v, K_int, part, drho);
    }
    __syncthreads();
    int p = tid / npad, t = tid - p * npad;
    int item = item0 + p;
    bool live = p < P && item < nitems && t < ny;
    int k = live ? (item >> 1) : 0;
    T u = vel_u<T>(vel, k), v = vel_v<T>(vel, k);
    T* F = tiles + (size_t)(p < P ? p : 0) * nc;
    const T* ghost = ghosts + (size_t)(p < P ? p : 0) * nw;
    bool px = u >= T(0), py = v >= T(0);
    int upx = px ? 0 : 1, upy = py ? 2 : 3;
    int sx = px ? 1 : -1, sy = py ? 1 : -1;
    int iy = py ? t : ny - 1 - t;
    T invdy = live ? T(1.0 / g.dy[iy]) : T(0);
    T au = px ? u : -u, av = py ? v : -v;   // |u|, |v|
    T carry = T(0);
    // data of the next cell of this row (prefetched one step ahead)
    int c = 0, ix = 0;
    unsigned fl = 0;
    T rc = T(0), cf = T(0), idx = T(0);
    auto fetch = [&](int jx) {
        ix = px ? jx : nx - 1 - jx;
        c = iy * nx + ix;
        fl = flags[c];
        rc = F[c];
        cf = coef[c];
        idx = invdx[ix];
    };
    if (live && t == 0) fetch(0);
    int nsteps = nx + ny - 1;
    for (int s = 0; s < nsteps; ++s) {
        int jx = s - t;
        bool act = live && jx >= 0 && jx < nx;
        if (act) {
            T val = T(0);
            if (!(fl & FLAG_SOLID)) {
                T D = cf + transport_diag_fl<T>(fl, u, v, idx, invdy);
                T tx = T(0), ty = T(0);
                int tpx = side_type(fl, upx), tpy = side_type(fl, upy);
                if (tpx == 0)
                    tx = -au * idx * carry;
                else if (tpx == 1)
                    tx = -au * idx * ghost[wall_index_fl(fl, upx)];
                if (tpy == 0)
                    ty = -av * invdy * F[c - sy * nx];
                else if (tpy == 1)
                    ty = -av * invdy * ghost[wall_index_fl(fl, upy)];
                val = (rc - tx - ty) / D;
                F[c] = val;
            }
            carry = val;
        }
        // prefetch the next cell of this row (never written by other threads)
        if (live && jx + 1 >= 0 && jx + 1 < nx) fetch(jx + 1);
        __syncthreads();
    }
    for (int q = 0; q < P; ++q) {
        int it = item0 + q;
        if (it >= nitems) break;
        int kq = it >> 1, part = it & 1;
        const T* src = tiles + (size_t)q * nc;
        bulk_copy<T>(df + ((size_t)part * vel.nk + kq) * nc, src, nc);
        if (part == 0) wall_products<T>(g, vel, kq, src, wbuf, threadIdx.x, blockDim.x);
    }
}

// The same sweep with the tile in global memory, for levels whose tile does
// not fit in LDS (one thread per row handles G and H; the neighbour in the
// previous row is read back from global memory after the step barrier).
template <typename T>
__global__ void k_sweep(Geo g, Vel vel, int K_int, const T* __restrict__ r, T* __restrict__ df,
                        const double* __restrict__ tau_inv, const double* __restrict__ dtn_inv,
                        const unsigned* __restrict__ flags, const double* __restrict__ drho,
                        double* __restrict__ wbuf, const T* __restrict__ msnap) {
    int k = blockIdx.x, t = threadIdx.x;
    int nx = g.nx, ny = g.ny;
    size_t nc = g.nc, ho = (size_t)vel.nk * nc, kc = (size_t)k * nc;
    T u = vel_u<T>(vel, k), v = vel_v<T>(vel, k);
    bool px = u >= T(0), py = v >= T(0);
    int upx = px ? 0 : 1, upy = py ? 2 : 3;
    int sx = px ? 1 : -1, sy = py ? 1 : -1;
    int iy = py ? t : ny - 1 - t;
    bool row = t < ny;
    T invdy = row ? T(1.0 / g.dy[iy]) : T(0);
    T* G = df + kc;
    T* H = df + ho + kc;
    int nsteps = nx + ny - 1;
    for (int s = 0; s < nsteps; ++s) {
        int jx = s - t;
        if (row && jx >= 0 && jx < nx) {
            int ix = px ? jx : nx - 1 - jx;
            int c = iy * nx + ix;
            unsigned fl = flags[c];
            T nG = T(0), nH = T(0);
            if (!(fl & FLAG_SOLID)) {
                T idx = T(1.0 / g.dx[ix]);
                T D = T(tau_inv[c] + dtn_inv[c]) + transport_diag_fl<T>(fl, u, v, idx, invdy);
                T txG = 0, txH = 0, tyG = 0, tyH = 0;
                int tpx = side_type(fl, upx), tpy = side_type(fl, upy);
                T cx = (px ? -u : u) * idx, cy = (py ? -v : v) * invdy;
                if (tpx == 0) {
                    txG = cx * G[c - sx];
                    txH = cx * H[c - sx];
                } else if (tpx == 1) {
                    int j = wall_index_fl(fl, upx);
                    txG = cx * wall_ghost_j<T>(g, j, u, v, K_int, 0, drho);
                    txH = cx * wall_ghost_j<T>(g, j, u, v, K_int, 1, drho);
                } else if (msnap && g.nb[upx * nc + c] == NB_SYMMETRY) {
                    size_t m = (size_t)vel.mx[k] * nc + c;   // mirror velocity, correction before the sweep
                    txG = cx * msnap[m];
                    txH = cx * msnap[ho + m];
                }
                if (tpy == 0) {
                    tyG = cy * G[c - sy * nx];
                    tyH = cy * H[c - sy * nx];
                } else if (tpy == 1) {
                    int j = wall_index_fl(fl, upy);
                    tyG = cy * wall_ghost_j<T>(g, j, u, v, K_int, 0, drho);
                    tyH = cy * wall_ghost_j<T>(g, j, u, v, K_int, 1, drho);
                } else if (msnap && g.nb[upy * nc + c] == NB_SYMMETRY) {
                    size_t m = (size_t)vel.my[k] * nc + c;
                    tyG = cy * msnap[m];
                    tyH = cy * msnap[ho + m];
                }
                nG = (r[kc + c] - txG - tyG) / D;
                nH = (r[ho + kc + c] - txH - tyH) / D;
            }
            G[c] = nG;
            H[c] = nH;
        }
        __syncthreads();
    }
    wall_products<T>(g, vel, k, G, wbuf, threadIdx.x, blockDim.x);
}

// ---------------------------------------------------------------------------
// Ordered sweep with one wavefront per group of velocities.
//
// In the upwind order of one velocity, row t (counted from the upwind
// y-side) at anti-diagonal step s needs two results of step s - 1: its own
// previous cell (x-upwind) and the cell of row t - 1 in the same column
// (y-upwind).  With lane = row the second one is the previous result of the
// neighbouring lane, so a one-lane rotation of the wavefront (DPP wave_ror:1)
// carries it: no LDS exchange and no barrier per step.  Rows beyond 64 are
// held as R row slots per lane (slot p = rows 64 p .. 64 p + 63; the row
// below slot p of lane 0 is slot p - 1 of lane 63).  When ny <= 32,
// I = 64 / ny velocities share a wavefront, lanes q ny .. q ny + ny - 1
// holding velocity q; the rotation into the first row of a velocity is never
// used, because that row's y-upwind side is a domain boundary.
//
// The r tiles (G and H) are staged in LDS by direct global-to-LDS loads and
// overwritten in place by the correction.  The wall ghosts C_k drho_w are
// constant during a sweep, so their upwind terms are added to the staged
// r before the first step (x-sides, then y-sides: a cell has at most one
// upwind side per direction).  Per-cell data shared by the wavefronts of a
// block (1/tau + 1/dt_n, side types, 1/dx) is staged once per block, and
// each lane loads the data of its next cell one step ahead.

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;

// lane i takes the value of lane i - 1 (lane 0 that of lane 63)
__device__ __forceinline__ float lane_rotate1(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x13C, 0xf, 0xf,
                                                                 false));
}
__device__ __forceinline__ double lane_rotate1(double x) {
    unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x13C, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x13C, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// x where the mask m is all ones, +0 where it is zero (m = 0 or -1)
__device__ __forceinline__ float mask_keep(float x, int m) {
    return __builtin_bit_cast(float, __builtin_bit_cast(int, x) & m);
}
__device__ __forceinline__ double mask_keep(double x, int m) {
    return __builtin_bit_cast(double, __builtin_bit_cast(long long, x) & (long long)m);
}
// -1 where the sign bit of x is set, 0 otherwise
__device__ __forceinline__ int sign_mask(float x) { return __builtin_bit_cast(int, x) >> 31; }
__device__ __forceinline__ int sign_mask(double x) { return (int)(__builtin_bit_cast(long long, x) >> 63); }

// 1 / x: the hardware reciprocal (1 ulp) in float, a correctly rounded
// division in double
__device__ __forceinline__ float sweep_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sweep_rcp(double x) { return 1.0 / x; }

// n elements from global memory into LDS by the 64 lanes of one wavefront:
// 16-byte direct global-to-LDS loads when both ends are 16-byte aligned and
// the size is a multiple of 16 bytes, element by element otherwise
template <typename T>
__device__ __forceinline__ void wave_load_lds(T* dst, const T* __restrict__ src, int n, int lane) {
    size_t bytes = (size_t)n * sizeof(T);
    if (((((size_t)dst) | ((size_t)src) | bytes) & 15) == 0) {
        int nv = (int)(bytes >> 4);
        for (int i = 0; i < nv; i += 64)
            if (i + lane < nv)
                __builtin_amdgcn_global_load_lds((gbl_void_t*)((const char*)src + ((size_t)(i + lane) << 4)),
                                                 (lds_void_t*)((char*)dst + ((size_t)i << 4)), 16, 0, 0);
    } else {
        for (int i = lane; i < n; i += 64) dst[i] = src[i];
    }
}

// n elements from LDS to global memory by one wavefront (16-byte stores when
// aligned)
template <typename T>
__device__ __forceinline__ void wave_store(T* __restrict__ dst, const T* src, int n, int lane) {
    size_t bytes = (size_t)n * sizeof(T);
    if (((((size_t)dst) | ((size_t)src) | bytes) & 15) == 0) {
        typedef __attribute__((ext_vector_type(4))) unsigned u4;
        int nv = (int)(bytes >> 4);
        const u4* s = (const u4*)src;
        u4* d = (u4*)dst;
        for (int i = lane; i < nv; i += 64) d[i] = s[i];
    } else {
        for (int i = lane; i < n; i += 64) dst[i] = src[i];
    }
}

// dst[i] += src[i] for n elements, dst in global memory and src in LDS, by
// one wavefront: 16-byte accesses when aligned, U loads of dst in flight per
// lane (the sweep kernels run few wavefronts per CU)
template <typename T, int U = 16>
__device__ __forceinline__ void wave_add_store(T* __restrict__ dst, const T* src, int n, int lane) {
    size_t bytes = (size_t)n * sizeof(T);
    if (((((size_t)dst) | ((size_t)src) | bytes) & 15) == 0) {
        constexpr int E = 16 / sizeof(T);
        typedef __attribute__((ext_vector_type(E))) T v4;
        const int nv = (int)(bytes >> 4);
        const v4* s = (const v4*)src;
        v4* d = (v4*)dst;
        for (int i0 = lane; i0 < nv; i0 += 64 * U) {
            v4 a[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + 64 * u < nv) a[u] = d[i0 + 64 * u];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + 64 * u < nv) d[i0 + 64 * u] = a[u] + s[i0 + 64 * u];
        }
    } else {
        for (int i0 = lane; i0 < n; i0 += 64 * U) {
            T a[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + 64 * u < n) a[u] = dst[i0 + 64 * u];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + 64 * u < n) dst[i0 + 64 * u] = a[u] + src[i0 + 64 * u];
        }
    }
}

// wall sides of a level that k_sweep_wave handles
constexpr int SWEEP_WAVE_MAX_WALLS = 512;

// LDS bytes of k_sweep_wave for W wavefronts of I velocities each and NP
// planes (1: G only, 2: G and H)
// (the tile region also holds the per-wavefront wall sums of the epilogue)
template <typename T>
__host__ __device__ inline size_t sweep_wave_tiles_elems(int nc, int nw, int W, int I, int NP) {
    size_t t = (size_t)W * NP * I * nc, red = ((size_t)W * nw * sizeof(double) + sizeof(T) - 1) / sizeof(T);
    return t > red ? t : red;
}

// (GC: the per-cell coefficients and side types are read through the
// caches, not staged)
template <typename T>
size_t sweep_wave_lds_bytes(int nc, int nx, int nw, int W, int I, int NP, bool GC = false) {
    size_t b = 64 * (size_t)W * sizeof(double) +
               (sweep_wave_tiles_elems<T>(nc, nw, W, I, NP) + (GC ? 0 : nc) + nx + 5 * (size_t)nw) * sizeof(T) +
               4 * (size_t)nw + (GC ? 0 : (size_t)nc);
    return (b + 15) & ~(size_t)15;
}

// coef = 1/tau + 1/dt_n per cell (-1 on solid cells) in the sweep's type;
// drho != nullptr: wall densities of the correction before the sweep
// (nullptr: the correction starts from zero, no ghost terms).  NP = 1 sweeps
// the G plane only: the sweep reads no earlier correction except through the
// wall densities, which depend on G alone, so a sweep whose H result is
// overwritten before use needs only G.
// Epilogue: the block's sums over its velocities of w_k u_n dG_k at every
// wall side (u_n > 0) go to wpart[block][j], the partial sums of the next
// wall densities.  wprev != nullptr: the wall densities of this sweep are
// formed in the prologue from the nprev partial sums of the previous sweep
// (every block alike, in a fixed order; block 0 also stores them to
// drho_out; one thread per wall side, so n_wall <= blockDim.x); otherwise
// they are read from drho (nullptr: zero).
// GC: the per-cell coefficients and side types are read through the caches
// by each lane one step ahead instead of being staged in LDS (levels whose
// tile alone fills the LDS).  split (with NP = 1): the grid's first half of
// blocks sweeps the G plane, the second half the H plane (each wall ghost
// term then takes the H factor K_int / (2 lam)); the H blocks leave no wall
// partial sums (nprev and the next sweep count the G blocks only).
template <typename T, int R, int NP, bool GC>
__global__ void __launch_bounds__(256) k_sweep_wave(Geo g, Vel vel, int K_int, const T* __restrict__ r,
                                                    T* __restrict__ df, const T* __restrict__ coef_g,
                                                    const unsigned char* __restrict__ stype,
                                                    const double* __restrict__ drho, double* __restrict__ wpart,
                                                    int I, const double* __restrict__ wprev, int nprev,
                                                    double* __restrict__ drho_out, int split) {
    // (no static LDS in this kernel: the tiles must start 16-byte aligned
    // for the direct global-to-LDS loads)
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    const int nc = g.nc, nx = g.nx, ny = g.ny, nw = g.n_wall, nk = vel.nk;
    const int W = blockDim.x >> 6, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double* dsum = smem_d;                                  // [64 W]  partial sums of the wall densities
    T* tiles = (T*)(smem_d + 64 * W);                       // [W][NP][I][nc]
    T* coef = tiles + sweep_wave_tiles_elems<T>(nc, nw, W, I, NP);   // [nc] (not with GC)
    T* invdx = coef + (GC ? 0 : nc);                        // [nx]
    T* wl = invdx + nx;                                     // [5][n_wall]  1/d, lam_w, U_w, V_w, drho
    int* wsc = (int*)(wl + 5 * (size_t)nw);                 // [n_wall]  side + 4 cell
    unsigned char* st = (unsigned char*)(wsc + nw);         // [nc]  side predicates, 2 bits per side (not with GC)
    // plane of this block (split: G blocks first, then H blocks)
    const int nbG = split ? (int)(gridDim.x >> 1) : (int)gridDim.x;
    const int plane = (int)blockIdx.x >= nbG ? 1 : 0;
    const int blk = (int)blockIdx.x - plane * nbG;
    const T* rp = r + (size_t)plane * nk * nc;
    T* dfp = df + (size_t)plane * nk * nc;
    const int k0 = (blk * W + w) * I;                       // first velocity of this wavefront
    const int nq = max(0, min(I, nk - k0));                 // velocities it holds
    T* tw = tiles + (size_t)w * NP * I * nc;
    // every load of the prologue is issued before the first wait
    if (nq > 0) {
        wave_load_lds<T>(tw, rp + (size_t)k0 * nc, nq * nc, lane);
        if constexpr (NP == 2) wave_load_lds<T>(tw + (size_t)I * nc, r + ((size_t)nk + k0) * nc, nq * nc, lane);
    }
    if constexpr (!GC) {
        if (w == 0) wave_load_lds<T>(coef, coef_g, nc, lane);
        if (w == W - 1) wave_load_lds<unsigned char>(st, stype, nc, lane);
    }
    for (int i = threadIdx.x; i < nx; i += blockDim.x) invdx[i] = T(1.0 / g.dx[i]);
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        wl[j] = T(g.w_invd[j]);
        wl[nw + j] = T(1.0 / g.w_T[j]);
        wl[2 * nw + j] = T(g.w_U[j]);
        wl[3 * nw + j] = T(g.w_V[j]);
        wl[4 * nw + j] = drho ? T(drho[j]) : T(0);
        wsc[j] = g.w_side[j] + 4 * g.w_cell[j];
    }
    // wall densities from the previous sweep's partial sums: thread t adds
    // the sums b = grp, grp + ng, ... of wall j = t mod nw (grp = t / nw)
    const int ng = nw > 0 ? max(1, (int)blockDim.x / nw) : 1;
    if (wprev && threadIdx.x < ng * nw) {
        int j = threadIdx.x % nw, grp = threadIdx.x / nw;
        double sacc = 0.0;
        for (int b = grp; b < nprev; b += ng) sacc += wprev[(size_t)b * nw + j];
        dsum[threadIdx.x] = sacc;
    }
    // velocities of this wavefront: lane q < nq holds velocity k0 + q
    const T uq_l = lane < nq ? vel_u<T>(vel, k0 + lane) : T(0);
    const T vq_l = lane < nq ? vel_v<T>(vel, k0 + lane) : T(0);
    __syncthreads();
    if (wprev) {
        for (int j = threadIdx.x; j < nw; j += blockDim.x) {
            double sacc = 0.0;
            for (int grp = 0; grp < ng; ++grp) sacc += dsum[grp * nw + j];
            double dj = -sacc / g.w_den[j];
            wl[4 * nw + j] = T(dj);
            if (blockIdx.x == 0) drho_out[j] = dj;
        }
        __syncthreads();
    }
    // upwind wall-ghost terms into r (x-sides, then y-sides)
    if (drho || wprev) {
        for (int jb = 0; jb < nw; jb += 64) {
            const int j = jb + lane;
            const bool ok = j < nw;
            int sd = 0, cell = 0;
            T invd = T(0), lam = T(1), wu = T(0), wv = T(0), dr = T(0);
            if (ok) {
                sd = wsc[j] & 3;
                cell = wsc[j] >> 2;
                invd = wl[j];
                lam = wl[nw + j];
                wu = wl[2 * nw + j];
                wv = wl[3 * nw + j];
                dr = wl[4 * nw + j];
            }
            for (int dir = 0; dir < 2; ++dir) {
                for (int q = 0; q < nq; ++q) {
                    const T u = __shfl(uq_l, q, 64), v = __shfl(vq_l, q, 64);
                    const T un = ((sd & 1) ? T(1) : T(-1)) * (sd < 2 ? u : v);
                    if (ok && (sd >> 1) == dir && un < T(0)) {
                        T du = u - wu, dv = v - wv;
                        T C = lam / T(M_PI) * dexp(-lam * (du * du + dv * dv));
                        if (plane) C = C * (T(K_int) / (T(2) * lam));
                        T a = -un * invd;
                        tw[(size_t)q * nc + cell] += a * (C * dr);
                        if constexpr (NP == 2)
                            tw[((size_t)I + q) * nc + cell] += a * (C * T(K_int) / (T(2) * lam) * dr);
                    }
                }
                __syncthreads();
            }
        }
    }

    const int q = I > 1 ? lane / ny : 0;
    const bool live = q < nq;
    const int qq = live ? q : 0;
    const int t0 = I > 1 ? lane - q * ny : lane;
    const T u = __shfl(uq_l, qq, 64), v = __shfl(vq_l, qq, 64);
    const bool px = u >= T(0), py = v >= T(0);
    const int shx = px ? 0 : 2, shy = py ? 4 : 6;           // bit offset of the upwind x / y side's predicates
    const T au = px ? u : -u, av = py ? v : -v;
    T* tG = tw + (size_t)qq * nc;
    T* tH = tw + ((size_t)(NP == 2 ? I : 0) + qq) * nc;
    int rowc[R];                                            // first cell of the slot's row
    bool rowok[R];
    T by[R], cG[R], cH[R];
    // data of a cell the slot reaches later, in a ring of three buffers: a
    // step reads one and fills the one read the step before (for two steps
    // on), so an LDS read has a whole step to return
    struct Ahead {
        T cf, idx, rG, rH;
        unsigned sc;
    };
    Ahead nA[R], nB[R], nC[R], nD[R];
    // a lane outside the current diagonal fetches the dummy column t mod nx:
    // a clamped column would put every such lane on one LDS bank
    const int dcol = t0 % nx;
    auto fetch = [&](Ahead& n, int p, int jx) {
        int jc = (jx < 0 || jx >= nx) ? dcol : jx;
        int ix = px ? jc : nx - 1 - jc;
        int c = rowc[p] + ix;
        if constexpr (GC) {
            n.cf = coef_g[c];
            n.sc = stype[c];
        } else {
            n.cf = coef[c];
            n.sc = st[c];
        }
        n.idx = invdx[ix];
        n.rG = tG[c];
        n.rH = T(0);
        if constexpr (NP == 2) n.rH = tH[c];
    };
    // results of lanes off the diagonal go to a word of their own (the
    // prologue's partial sums are no longer needed): no branch per step
    T* dump = (T*)dsum + 64 * w + lane;
#pragma unroll
    for (int p = 0; p < R; ++p) {
        int row = t0 + 64 * p;
        rowok[p] = live && row < ny;
        int iy = rowok[p] ? (py ? row : ny - 1 - row) : 0;
        rowc[p] = iy * nx;
        by[p] = rowok[p] ? av * T(1.0 / g.dy[iy]) : T(0);
        cG[p] = T(0);
        cH[p] = T(0);
        fetch(nA[p], p, -row);
        fetch(nB[p], p, 1 - row);
        fetch(nC[p], p, 2 - row);
    }
    // step s with the data in cur; fill receives those of step s + 2
    auto step = [&](int s, const Ahead(&cur)[R], Ahead(&fill)[R]) {
        T rotG[R], rotH[R];
#pragma unroll
        for (int p = 0; p < R; ++p) {
            rotG[p] = lane_rotate1(cG[p]);
            if constexpr (NP == 2) rotH[p] = lane_rotate1(cH[p]);
        }
#pragma unroll
        for (int p = 0; p < R; ++p) {
            int jx = s - (t0 + 64 * p);
            bool valid = rowok[p] && (unsigned)jx < (unsigned)nx;
            const Ahead& d = cur[p];
            int c = rowc[p] + (px ? jx : nx - 1 - jx);
            fetch(fill[p], p, jx + 3);
            T nbG = rotG[p], nbH = NP == 2 ? rotH[p] : T(0);
            if (R > 1 && lane == 0) {
                nbG = p > 0 ? rotG[p > 0 ? p - 1 : 0] : T(0);
                if constexpr (NP == 2) nbH = p > 0 ? rotH[p > 0 ? p - 1 : 0] : T(0);
            }
            // the upwind sides' predicates: an interior face, not an outflow
            const bool x0 = (d.sc >> shx) & 1u, xn3 = (d.sc >> (shx + 1)) & 1u;
            const bool y0 = (d.sc >> shy) & 1u, yn3 = (d.sc >> (shy + 1)) & 1u;
            T bx = au * d.idx, byp = by[p];
            // transport diagonal: every downwind side, and an upwind side
            // only if it is an outflow (where the two cancel)
            T D = d.cf + (xn3 ? bx : T(0)) + (yn3 ? byp : T(0));
            T inv = sweep_rcp(D);
            T exG = x0 ? cG[p] : T(0), eyG = y0 ? nbG : T(0);
            T vG = (d.rG + bx * exG + byp * eyG) * inv;
            vG = d.cf < T(0) ? T(0) : vG;
            *(valid ? tG + c : dump) = vG;
            cG[p] = vG;
            if constexpr (NP == 2) {
                T exH = x0 ? cH[p] : T(0), eyH = y0 ? nbH : T(0);
                T vH = (d.rH + bx * exH + byp * eyH) * inv;
                vH = d.cf < T(0) ? T(0) : vH;
                *(valid ? tH + c : dump) = vH;
                cH[p] = vH;
            }
        }
    };
    const int nsteps = nx + ny - 1;
    int s = 0;
    for (; s + 3 < nsteps; s += 4) {
        step(s, nA, nD);
        step(s + 1, nB, nA);
        step(s + 2, nC, nB);
        step(s + 3, nD, nC);
    }
    if (s < nsteps) step(s, nA, nD);
    if (s + 1 < nsteps) step(s + 1, nB, nA);
    if (s + 2 < nsteps) step(s + 2, nC, nB);
    __syncthreads();
    if (nq > 0) {
        wave_store<T>(dfp + (size_t)k0 * nc, tw, nq * nc, lane);
        if constexpr (NP == 2) wave_store<T>(df + ((size_t)nk + k0) * nc, tw + (size_t)I * nc, nq * nc, lane);
    }
    // the H plane leaves no wall partial sums (uniform over the block)
    if (plane) return;
    // per-wavefront sums over its velocities of w_k u_n dG_k at the wall sides
    const double ud = lane < nq ? vel.u[k0 + lane] : 0.0, vd = lane < nq ? vel.v[k0 + lane] : 0.0,
                 wd = lane < nq ? vel.w[k0 + lane] : 0.0;
    // (at most SWEEP_WAVE_MAX_WALLS wall sides: one register per 64 of them)
    double wsum[SWEEP_WAVE_MAX_WALLS / 64];
#pragma unroll
    for (int jc = 0; jc < SWEEP_WAVE_MAX_WALLS / 64; ++jc) {
        const int j = jc * 64 + lane;
        const bool ok = j < nw;
        const int sd = ok ? wsc[j] & 3 : 0, cell = ok ? wsc[j] >> 2 : 0;
        double sum = 0.0;
        if (jc * 64 < nw)
            for (int qv = 0; qv < nq; ++qv) {
                double uu = __shfl(ud, qv, 64), vv = __shfl(vd, qv, 64), ww = __shfl(wd, qv, 64);
                double un = ((sd & 1) ? 1.0 : -1.0) * (sd < 2 ? uu : vv);
                if (ok && un > 0.0) sum += ww * un * double(tw[(size_t)qv * nc + cell]);
            }
        wsum[jc] = sum;
    }
    __syncthreads();   // every tile is read: the sums go where the tiles were
    double* red = (double*)tiles;   // [W][n_wall]
#pragma unroll
    for (int jc = 0; jc < SWEEP_WAVE_MAX_WALLS / 64; ++jc) {
        const int j = jc * 64 + lane;
        if (j < nw) red[(size_t)w * nw + j] = wsum[jc];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        double s = 0.0;
        for (int ww = 0; ww < W; ++ww) s += red[(size_t)ww * nw + j];
        wpart[(size_t)blk * nw + j] = s;
    }
}

// ---------------------------------------------------------------------------
// Ordered sweep of one plane in x-strips, for levels whose tile alone would
// fill the LDS (one wavefront per velocity, as k_sweep_wave with I = 1).
//
// The level is cut into nstrip strips of columns, taken in the upwind order
// of the velocity; only one strip's tile (all rows, sw columns) is resident,
// so several wavefronts share a CU.  A lane owns the same rows in every
// strip and keeps its last result of each row in a register (it is updated
// on valid steps only): at a strip's first column that register is the
// x-upwind value of the strip before, so the strips join without any
// exchange.  The W wavefronts of a block take consecutive velocities of one
// row of the grid (index k = ku nvrow + kv, one ku per block): they share
// the sign of u and so the order of the strips, and the strip's per-cell
// coefficients and side types are staged once for the block.  Each strip's
// tiles are staged by direct global-to-LDS loads where rows are 16-byte
// aligned, the wall ghost terms added, swept in nx_s + ny - 1 steps and
// stored; the wall sums of the G plane accumulate over the strips.  split
// as in k_sweep_wave (with the velocity mapping above per plane).
template <typename T>
__host__ __device__ inline int sweep_strip_width(int nx, int nstrip) {
    int sw = (nx + nstrip - 1) / nstrip;
    return (sw + 3) & ~3;   // 16-byte rows in float (8-byte multiples in double)
}

template <typename T>
__host__ __device__ inline size_t sweep_strip_tile_elems(int ny, int sw, int nw, int W) {
    size_t t = (size_t)W * ny * sw, red = ((size_t)W * nw * sizeof(double) + sizeof(T) - 1) / sizeof(T);
    return t > red ? t : red;
}

template <typename T>
size_t sweep_strip_lds_bytes(int nx, int ny, int nw, int W, int nstrip) {
    int sw = sweep_strip_width<T>(nx, nstrip);
    size_t b = 64 * (size_t)W * sizeof(double) +
               (sweep_strip_tile_elems<T>(ny, sw, nw, W) + (size_t)ny * sw + nx + 5 * (size_t)nw) * sizeof(T) +
               4 * (size_t)nw + (size_t)ny * sw;
    return (b + 15) & ~(size_t)15;
}

// rows x cols elements (row strides sstride in global memory, cols in LDS)
// from global memory into LDS by the 64 lanes of one wavefront: 16-byte
// direct loads when every row start is 16-byte aligned, element by element
// otherwise
template <typename T>
__device__ __forceinline__ void wave_load_lds_2d(T* dst, const T* __restrict__ src, int rows, int cols,
                                                 size_t sstride, int lane) {
    const size_t rb = (size_t)cols * sizeof(T);
    if (((((size_t)dst) | ((size_t)src) | rb | (sstride * sizeof(T))) & 15) == 0) {
        const int per = (int)(rb >> 4);   // 16-byte pieces per row
        const int n = rows * per;
        for (int i = lane; i - lane < n; i += 64) {
            // a wavefront-wide loop: lanes past the end issue nothing
            if (i < n) {
                int rr = i / per, cc = i - rr * per;
                __builtin_amdgcn_global_load_lds(
                    (gbl_void_t*)((const char*)src + rr * sstride * sizeof(T) + ((size_t)cc << 4)),
                    (lds_void_t*)((char*)dst + (size_t)(i - lane) * 16), 16, 0, 0);
            }
        }
    } else {
        const int n = rows * cols;
        for (int i = lane; i < n; i += 64) {
            int rr = i / cols, cc = i - rr * cols;
            dst[i] = src[rr * sstride + cc];
        }
    }
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_sweep_strips(Geo g, Vel vel, int K_int, const T* __restrict__ r,
                                                      T* __restrict__ df, const T* __restrict__ coef_g,
                                                      const unsigned char* __restrict__ stype,
                                                      const double* __restrict__ drho,
                                                      double* __restrict__ wpart, int nstrip,
                                                      const double* __restrict__ wprev, int nprev,
                                                      double* __restrict__ drho_out, int split, int nvrow) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    const int nc = g.nc, nx = g.nx, ny = g.ny, nw = g.n_wall, nk = vel.nk;
    const int W = blockDim.x >> 6, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int sw = sweep_strip_width<T>(nx, nstrip);
    double* dsum = smem_d;                                  // [64 W]
    T* tiles = (T*)(smem_d + 64 * W);                       // [W][ny][sw]
    T* cs = tiles + sweep_strip_tile_elems<T>(ny, sw, nw, W);   // [ny][sw]  the strip's coefficients
    T* invdx = cs + (size_t)ny * sw;                        // [nx]
    T* wl = invdx + nx;                                     // [5][n_wall]  1/d, lam_w, U_w, V_w, drho
    int* wsc = (int*)(wl + 5 * (size_t)nw);                 // [n_wall]  side + 4 cell
    unsigned char* ss = (unsigned char*)(wsc + nw);         // [ny][sw]  the strip's side predicates
    const int nbG = split ? (int)(gridDim.x >> 1) : (int)gridDim.x;
    const int plane = (int)blockIdx.x >= nbG ? 1 : 0;
    const int blk = (int)blockIdx.x - plane * nbG;
    // one row of the velocity grid per block (bpr blocks per row)
    const int bpr = (nvrow + W - 1) / W;
    const int ku = blk / bpr, kv = (blk - ku * bpr) * W + w;
    const int k = ku * nvrow + kv;
    const bool kok = kv < nvrow && k < nk;
    // a wavefront without a velocity takes its row's first one (the same
    // sign of u as the block's others); it loads, stores and sums nothing
    const int kk = kok ? k : ku * nvrow;
    const T* rk = r + ((size_t)plane * nk + kk) * nc;
    T* dk = df + ((size_t)plane * nk + kk) * nc;
    T* tw = tiles + (size_t)w * ny * sw;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) invdx[i] = T(1.0 / g.dx[i]);
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        wl[j] = T(g.w_invd[j]);
        wl[nw + j] = T(1.0 / g.w_T[j]);
        wl[2 * nw + j] = T(g.w_U[j]);
        wl[3 * nw + j] = T(g.w_V[j]);
        wl[4 * nw + j] = drho ? T(drho[j]) : T(0);
        wsc[j] = g.w_side[j] + 4 * g.w_cell[j];
    }
    const int ng = nw > 0 ? max(1, (int)blockDim.x / nw) : 1;
    if (wprev && threadIdx.x < ng * nw) {
        int j = threadIdx.x % nw, grp = threadIdx.x / nw;
        double sacc = 0.0;
        for (int b = grp; b < nprev; b += ng) sacc += wprev[(size_t)b * nw + j];
        dsum[threadIdx.x] = sacc;
    }
    __syncthreads();
    if (wprev) {
        for (int j = threadIdx.x; j < nw; j += blockDim.x) {
            double sacc = 0.0;
            for (int grp = 0; grp < ng; ++grp) sacc += dsum[grp * nw + j];
            double dj = -sacc / g.w_den[j];
            wl[4 * nw + j] = T(dj);
            if (blockIdx.x == 0) drho_out[j] = dj;
        }
        __syncthreads();
    }
    const bool ghosts = drho || wprev;
    const T u = vel_u<T>(vel, kk), v = vel_v<T>(vel, kk);
    const bool px = u >= T(0), py = v >= T(0);
    const int shx = px ? 0 : 2, shy = py ? 4 : 6;           // bit offset of the upwind x / y side's predicates
    const T au = px ? u : -u, av = py ? v : -v;
    int iyr[R];                                             // cell row of each slot
    bool rowok[R];
    T by[R], cG[R];
#pragma unroll
    for (int p = 0; p < R; ++p) {
        int row = lane + 64 * p;
        rowok[p] = kok && row < ny;
        iyr[p] = rowok[p] ? (py ? row : ny - 1 - row) : 0;
        by[p] = rowok[p] ? av * T(1.0 / g.dy[iyr[p]]) : T(0);
        cG[p] = T(0);
    }
    // per-wavefront sums over its velocity of w_k u_n dG_k at the wall sides
    const double ud = vel.u[kk], vd = vel.v[kk], wd = kok ? vel.w[kk] : 0.0;
    double wsum[SWEEP_WAVE_MAX_WALLS / 64];
#pragma unroll
    for (int jc = 0; jc < SWEEP_WAVE_MAX_WALLS / 64; ++jc) wsum[jc] = 0.0;
    // results of lanes off the diagonal go to a word of their own
    T* dump = (T*)dsum + 64 * w + lane;
    struct Ahead {
        T cf, idx, rG;
        unsigned sc;
    };
    for (int b = 0; b < nstrip; ++b) {
        const int x0 = b * sw;
        if (x0 >= nx) break;
        const int wb = min(sw, nx - x0);                    // columns of this strip
        const int pc0 = px ? x0 : nx - x0 - wb;             // its first physical column
        __syncthreads();   // the previous strip's tile is stored and summed
        if (kok) wave_load_lds_2d<T>(tw, rk + pc0, ny, wb, (size_t)nx, lane);
        if (w == 0) wave_load_lds_2d<T>(cs, coef_g + pc0, ny, wb, (size_t)nx, lane);
        if (w == W - 1) wave_load_lds_2d<unsigned char>(ss, stype + pc0, ny, wb, (size_t)nx, lane);
        __syncthreads();
        // upwind wall-ghost terms of the strip's wall cells (x-sides, then
        // y-sides; the barriers are reached by every wavefront of the block)
        if (ghosts) {
            for (int jb = 0; jb < nw; jb += 64) {
                const int j = jb + lane;
                int sd = 0, cell = 0;
                bool ok = kok && j < nw;
                if (ok) {
                    sd = wsc[j] & 3;
                    cell = wsc[j] >> 2;
                    const int ix = cell % nx;
                    ok = ix >= pc0 && ix < pc0 + wb;
                }
                for (int dir = 0; dir < 2; ++dir) {
                    const T un = ((sd & 1) ? T(1) : T(-1)) * (sd < 2 ? u : v);
                    if (ok && (sd >> 1) == dir && un < T(0)) {
                        const T lam = wl[nw + j], du = u - wl[2 * nw + j], dv = v - wl[3 * nw + j];
                        T C = lam / T(M_PI) * dexp(-lam * (du * du + dv * dv));
                        if (plane) C = C * (T(K_int) / (T(2) * lam));
                        const int ti = (cell / nx) * wb + (cell % nx - pc0);
                        tw[ti] += (-un * wl[j]) * (C * wl[4 * nw + j]);
                    }
                    __syncthreads();
                }
            }
        }
        const int dcol = lane % wb;
        auto fetch = [&](Ahead& n, int p, int jx) {
            int jc = (jx < 0 || jx >= wb) ? dcol : jx;
            int ixl = px ? jc : wb - 1 - jc;
            int ti = iyr[p] * wb + ixl;
            n.cf = cs[ti];
            n.sc = ss[ti];
            n.idx = invdx[pc0 + ixl];
            n.rG = tw[ti];
        };
        Ahead nA[R], nB[R], nC[R], nD[R];
#pragma unroll
        for (int p = 0; p < R; ++p) {
            int row = lane + 64 * p;
            fetch(nA[p], p, -row);
            fetch(nB[p], p, 1 - row);
            fetch(nC[p], p, 2 - row);
        }
        auto step = [&](int s, const Ahead(&cur)[R], Ahead(&fill)[R]) {
            T rotG[R];
#pragma unroll
            for (int p = 0; p < R; ++p) rotG[p] = lane_rotate1(cG[p]);
#pragma unroll
            for (int p = 0; p < R; ++p) {
                int jx = s - (lane + 64 * p);
                bool valid = rowok[p] && (unsigned)jx < (unsigned)wb;
                const Ahead& d = cur[p];
                int ixl = px ? jx : wb - 1 - jx;
                fetch(fill[p], p, jx + 3);
                T nbG = rotG[p];
                if (R > 1 && lane == 0) nbG = p > 0 ? rotG[p > 0 ? p - 1 : 0] : T(0);
                const bool x0 = (d.sc >> shx) & 1u, xn3 = (d.sc >> (shx + 1)) & 1u;
                const bool y0 = (d.sc >> shy) & 1u, yn3 = (d.sc >> (shy + 1)) & 1u;
                T bx = au * d.idx, byp = by[p];
                T D = d.cf + (xn3 ? bx : T(0)) + (yn3 ? byp : T(0));
                T inv = sweep_rcp(D);
                T exG = x0 ? cG[p] : T(0), eyG = y0 ? nbG : T(0);
                T vG = (d.rG + bx * exG + byp * eyG) * inv;
                vG = d.cf < T(0) ? T(0) : vG;
                *(valid ? tw + iyr[p] * wb + ixl : dump) = vG;
                cG[p] = valid ? vG : cG[p];
            }
        };
        const int nsteps = wb + ny - 1;
        int s = 0;
        for (; s + 3 < nsteps; s += 4) {
            step(s, nA, nD);
            step(s + 1, nB, nA);
            step(s + 2, nC, nB);
            step(s + 3, nD, nC);
        }
        if (s < nsteps) step(s, nA, nD);
        if (s + 1 < nsteps) step(s + 1, nB, nA);
        if (s + 2 < nsteps) step(s + 2, nC, nB);
        __syncthreads();
        if (kok) {
            // the strip's rows back to global memory
            const int n = ny * wb;
            for (int i = lane; i < n; i += 64) {
                int rr = i / wb, cc = i - rr * wb;
                dk[(size_t)rr * nx + pc0 + cc] = tw[i];
            }
            if (!plane) {
#pragma unroll
                for (int jc = 0; jc < SWEEP_WAVE_MAX_WALLS / 64; ++jc) {
                    const int j = jc * 64 + lane;
                    if (jc * 64 < nw && j < nw) {
                        const int sd = wsc[j] & 3, cell = wsc[j] >> 2, ix = cell % nx;
                        const double un = ((sd & 1) ? 1.0 : -1.0) * (sd < 2 ? ud : vd);
                        if (un > 0.0 && ix >= pc0 && ix < pc0 + wb)
                            wsum[jc] += wd * un * double(tw[(cell / nx) * wb + (ix - pc0)]);
                    }
                }
            }
        }
    }
    if (plane) return;
    __syncthreads();   // every tile is read: the sums go where the tiles were
    double* red = (double*)tiles;   // [W][n_wall]
#pragma unroll
    for (int jc = 0; jc < SWEEP_WAVE_MAX_WALLS / 64; ++jc) {
        const int j = jc * 64 + lane;
        if (j < nw) red[(size_t)w * nw + j] = wsum[jc];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        double sacc = 0.0;
        for (int ww = 0; ww < W; ++ww) sacc += red[(size_t)ww * nw + j];
        wpart[(size_t)blk * nw + j] = sacc;
    }
}

// ---------------------------------------------------------------------------
// Ordered sweep of one plane in bands of rows, one launch per band.
//
// Band b holds the rows b h .. b h + hb - 1 (hb = min(h, ny - b h)) counted in
// the y-upwind order of each velocity, so a velocity's bands are taken in its
// own upwind order by successive launches.  Within a band the sweep is that
// of k_sweep_wave with I = 64 / h velocities per wavefront: lane q h + t0
// holds row t0 of velocity q, which updates column s - t0 at step s, the
// y-upwind value carried by the one-lane rotation.  The first row of a band
// after the first takes its y-upwind value from the last row of the band
// before, which the launch before stored to df; that row is staged with the
// band.  A band of one velocity is hb whole rows, contiguous in memory, so
// it is staged by direct global-to-LDS loads and stored back in one piece.
// Short bands keep every lane of a wavefront on a cell of the anti-diagonal
// for all but hb - 1 of the nx + hb - 1 steps (a tall level swept by one
// wavefront per velocity keeps ny lanes busy only near the middle of its
// nx + ny - 1 steps).  The per-cell coefficients and side predicates are
// read through the caches: the I velocities of a wavefront are consecutive
// ones of one row of the velocity grid (the same sign of u), so their lanes
// read the same cells.  Wall ghosts are added to the staged band as in
// k_sweep_wave; the G plane's wall sums of a block accumulate over the
// bands in wpart[blk] (the first band writes them).  split as in
// k_sweep_wave.
//
// fout (null: unused) makes the sweep the last one of a correction that is
// applied at once (Step 6): the band's values are added to the distribution
// fout, f += df, and df receives only the row that the next band reads.
template <typename T>
__host__ __device__ inline size_t sweep_band_tile_elems(int nx, int h, int nw, int W, int I) {
    size_t t = (size_t)W * I * h * nx, red = ((size_t)W * nw * sizeof(double) + sizeof(T) - 1) / sizeof(T);
    return t > red ? t : red;
}

template <typename T>
size_t sweep_band_lds_bytes(int nx, int h, int nw, int W, int I) {
    size_t b = 64 * (size_t)W * sizeof(double) +
               (sweep_band_tile_elems<T>(nx, h, nw, W, I) + (size_t)W * I * nx + nx + 5 * (size_t)nw) * sizeof(T) +
               4 * (size_t)nw;
    return (b + 15) & ~(size_t)15;
}

template <typename T>
__global__ void __launch_bounds__(256) k_sweep_band(Geo g, Vel vel, int K_int, const T* __restrict__ r,
                                                    T* __restrict__ df, const T* __restrict__ coef_g,
                                                    const unsigned char* __restrict__ stype,
                                                    const double* __restrict__ drho, double* __restrict__ wpart,
                                                    int I, int h, int b, int nvrow, int split,
                                                    T* __restrict__ fout) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    const int nc = g.nc, nx = g.nx, ny = g.ny, nw = g.n_wall, nk = vel.nk;
    const int W = blockDim.x >> 6, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int hb = min(h, ny - b * h);                      // rows of this band
    const size_t tsz = (size_t)h * nx;                      // tile elements per velocity
    double* dsum = smem_d;                                  // [64 W]  words of lanes off the diagonal
    T* tiles = (T*)(smem_d + 64 * W);                       // [W][I][h][nx]
    T* edge = tiles + sweep_band_tile_elems<T>(nx, h, nw, W, I);   // [W][I][nx]  the row before the band
    T* invdx = edge + (size_t)W * I * nx;                   // [nx]
    T* wl = invdx + nx;                                     // [5][n_wall]  1/d, lam_w, U_w, V_w, drho
    int* wsc = (int*)(wl + 5 * (size_t)nw);                 // [n_wall]  side + 4 cell
    const int nbG = split ? (int)(gridDim.x >> 1) : (int)gridDim.x;
    const int plane = (int)blockIdx.x >= nbG ? 1 : 0;
    const int blk = (int)blockIdx.x - plane * nbG;
    // velocities: wavefronts of I consecutive ones along a row of the
    // velocity grid (wpr wavefronts, bpr blocks per row)
    const int wpr = (nvrow + I - 1) / I, bpr = (wpr + W - 1) / W;
    const int ku = blk / bpr, wi = (blk - ku * bpr) * W + w;
    const int kv0 = wi * I, k0 = ku * nvrow + kv0;
    const int nq = wi < wpr ? min(I, nvrow - kv0) : 0;      // velocities this wavefront holds
    const T* rp = r + (size_t)plane * nk * nc;
    T* dfp = df + (size_t)plane * nk * nc;
    T* tw = tiles + (size_t)w * I * tsz;
    T* ew = edge + (size_t)w * I * nx;
    // first physical row of the band of a velocity whose v has sign py, and
    // the physical row before it in that velocity's order
    auto band_y0 = [&](bool py) { return py ? b * h : ny - b * h - hb; };
    auto prev_y = [&](bool py) { return py ? b * h - 1 : ny - b * h; };
    // every load of the prologue is issued before the first wait
    for (int q = 0; q < nq; ++q) {
        const bool pyq = vel_v<T>(vel, k0 + q) >= T(0);
        const size_t kq = (size_t)(k0 + q) * nc;
        wave_load_lds<T>(tw + q * tsz, rp + kq + (size_t)band_y0(pyq) * nx, hb * nx, lane);
        if (b > 0) wave_load_lds<T>(ew + (size_t)q * nx, dfp + kq + (size_t)prev_y(pyq) * nx, nx, lane);
    }
    for (int i = threadIdx.x; i < nx; i += blockDim.x) invdx[i] = T(1.0 / g.dx[i]);
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        wl[j] = T(g.w_invd[j]);
        wl[nw + j] = T(1.0 / g.w_T[j]);
        wl[2 * nw + j] = T(g.w_U[j]);
        wl[3 * nw + j] = T(g.w_V[j]);
        wl[4 * nw + j] = drho ? T(drho[j]) : T(0);
        wsc[j] = g.w_side[j] + 4 * g.w_cell[j];
    }
    // velocities of this wavefront: lane q < nq holds velocity k0 + q
    const T uq_l = lane < nq ? vel_u<T>(vel, k0 + lane) : T(0);
    const T vq_l = lane < nq ? vel_v<T>(vel, k0 + lane) : T(0);
    __syncthreads();
    // upwind wall-ghost terms of the band's wall cells into r (x-sides, then
    // y-sides; the barriers are reached by every wavefront of the block)
    if (drho) {
        for (int jb = 0; jb < nw; jb += 64) {
            const int j = jb + lane;
            const bool ok = j < nw;
            int sd = 0, cell = 0;
            T invd = T(0), lam = T(1), wu = T(0), wv = T(0), dr = T(0);
            if (ok) {
                sd = wsc[j] & 3;
                cell = wsc[j] >> 2;
                invd = wl[j];
                lam = wl[nw + j];
                wu = wl[2 * nw + j];
                wv = wl[3 * nw + j];
                dr = wl[4 * nw + j];
            }
            const int iyc = cell / nx;
            for (int dir = 0; dir < 2; ++dir) {
                for (int q = 0; q < nq; ++q) {
                    const T u = __shfl(uq_l, q, 64), v = __shfl(vq_l, q, 64);
                    const T un = ((sd & 1) ? T(1) : T(-1)) * (sd < 2 ? u : v);
                    const int y0 = band_y0(v >= T(0));
                    if (ok && (sd >> 1) == dir && un < T(0) && iyc >= y0 && iyc < y0 + hb) {
                        const T du = u - wu, dv = v - wv;
                        T C = lam / T(M_PI) * dexp(-lam * (du * du + dv * dv));
                        if (plane) C = C * (T(K_int) / (T(2) * lam));
                        tw[(size_t)q * tsz + (size_t)(iyc - y0) * nx + cell % nx] += (-un * invd) * (C * dr);
                    }
                }
                __syncthreads();
            }
        }
    }

    const int q = lane / h;
    const bool live = q < nq;
    const int qq = live ? q : 0;
    const int t0 = lane - q * h;                            // row within the band
    const T u = __shfl(uq_l, qq, 64), v = __shfl(vq_l, qq, 64);
    const bool px = u >= T(0), py = v >= T(0);
    const int shx = px ? 0 : 2, shy = py ? 4 : 6;           // bit offset of the upwind x / y side's predicates
    const T au = px ? u : -u, av = py ? v : -v;
    const bool rowok = live && t0 < hb;
    const int y0 = band_y0(py);
    const int iy = rowok ? (py ? b * h + t0 : ny - 1 - b * h - t0) : y0;   // physical row
    const int trow = iy - y0;                               // its tile row
    const T by = rowok ? av * T(1.0 / g.dy[iy]) : T(0);
    // the band's first row takes its y-upwind value from the row before
    const bool first = t0 == 0 && b > 0;
    T* tG = tw + (size_t)qq * tsz + (size_t)trow * nx;
    const T* eG = ew + (size_t)qq * nx;
    const unsigned char* srow = stype + (size_t)iy * nx;
    const T* crow = coef_g + (size_t)iy * nx;
    T cG = T(0);
    // The per-cell data of a step depend only on its column, so they are
    // fetched a batch of SB steps ahead, into two alternating register
    // batches: a batch's loads are in flight while the batch before is swept
    // (fetching each step's data a few steps ahead left the compiler free to
    // hoist the independent part of later steps above the wait, so the wait
    // came about one step after the load).
    constexpr int SB = 8;
    struct Batch {
        T cf[SB], idx[SB], rG[SB], ey[SB];
        unsigned sc[SB];
        int so[SB];   // where the step's value goes: its tile cell, or the lane's dump word
    };
    // A step's index work is done at fetch time, without lane masks combined
    // in scalar registers: the column jx = s - t0 of a lane off the grid
    // becomes the dummy column t0 mod nx (one unsigned compare), so every
    // read stays inside the lane's row; the cell of the row is (jc ^ xm) + xa
    // (jc upwind in x, nx - 1 - jc downwind); the store goes to the tile only
    // where jx < lim (nx on a row of the band, 0 elsewhere).
    const int dcol = t0 % nx;
    const int xm = px ? 0 : -1, xa = px ? 0 : nx;
    const unsigned lim = rowok ? (unsigned)nx : 0u;
    T* const sbase = (T*)dsum;
    const int tgo = (int)(tG - sbase), dumpo = 64 * w + lane;   // dump words: [64 W] at the start of dsum
    auto fetch = [&](Batch& n, int s0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int jx = s0 + u - t0;
            const int jc = (unsigned)jx < (unsigned)nx ? jx : dcol;
            const int ix = (jc ^ xm) + xa;   // in [0, nx)
            n.cf[u] = crow[(unsigned)ix];
            n.sc[u] = srow[(unsigned)ix];
            n.idx[u] = invdx[ix];
            n.rG[u] = tG[ix];
            n.ey[u] = eG[ix];
            n.so[u] = (unsigned)jx < lim ? tgo + ix : dumpo;
        }
    };
    // SB steps with the data in d
    auto sweep = [&](const Batch& d) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const T rot = lane_rotate1(cG);
            const T nbG = first ? d.ey[u] : rot;
            // the upwind sides' predicates as all-ones / zero masks (a
            // sign-extending bit extract each; no compares, so no lane masks)
            const int sc = (int)d.sc[u];
            const int mx0 = __builtin_amdgcn_sbfe(sc, shx, 1), mxn3 = __builtin_amdgcn_sbfe(sc, shx + 1, 1);
            const int my0 = __builtin_amdgcn_sbfe(sc, shy, 1), myn3 = __builtin_amdgcn_sbfe(sc, shy + 1, 1);
            const T bx = au * d.idx[u];
            // transport diagonal: every downwind side, and an upwind side only
            // if it is an outflow (where the two cancel)
            const T D = d.cf[u] + mask_keep(bx, mxn3) + mask_keep(by, myn3);
            const T inv = sweep_rcp(D);
            const T exG = mask_keep(cG, mx0), eyG = mask_keep(nbG, my0);
            T vG = (d.rG[u] + bx * exG + by * eyG) * inv;
            vG = mask_keep(vG, ~sign_mask(d.cf[u]));   // zero in a solid cell (negative coefficient)
            sbase[d.so[u]] = vG;
            cG = vG;
        }
    };
    // whole pairs of batches: the steps past the last one find every lane
    // off the grid (their stores go to the dump words).  The loads of a batch
    // are kept above the steps of the batch before by a scheduling barrier
    // (the scheduler otherwise moves them down to shorten live ranges), and
    // there is no exit between the two batches of a pair (with one, the loads
    // of the second batch were sunk to the block that uses them).
    const int nsteps = nx + hb - 1;
    Batch bA, bB;
    fetch(bA, 0);
    for (int s0 = 0; s0 < nsteps; s0 += 2 * SB) {
        fetch(bB, s0 + SB);
        __builtin_amdgcn_sched_barrier(0);
        sweep(bA);
        fetch(bA, s0 + 2 * SB);
        __builtin_amdgcn_sched_barrier(0);
        sweep(bB);
    }
    __syncthreads();
    if (!fout) {
        for (int qv = 0; qv < nq; ++qv) {
            const bool pyq = vel_v<T>(vel, k0 + qv) >= T(0);
            wave_store<T>(dfp + (size_t)(k0 + qv) * nc + (size_t)band_y0(pyq) * nx, tw + qv * tsz, hb * nx, lane);
        }
    } else {
        // f += df over the band; df only for the band's last row in the
        // velocity's order (tile row hb - 1 upward, 0 downward), which the
        // next band reads
        T* fp = fout + (size_t)plane * nk * nc;
        const bool more = (b + 1) * h < ny;
        for (int qv = 0; qv < nq; ++qv) {
            const bool pyq = vel_v<T>(vel, k0 + qv) >= T(0);
            const size_t off = (size_t)(k0 + qv) * nc + (size_t)band_y0(pyq) * nx;
            wave_add_store<T>(fp + off, tw + qv * tsz, hb * nx, lane);
            if (more) {
                const size_t tr = pyq ? (size_t)(hb - 1) * nx : 0;
                wave_store<T>(dfp + off + tr, tw + qv * tsz + tr, nx, lane);
            }
        }
    }
    // the H plane leaves no wall partial sums (uniform over the block)
    if (plane) return;
    // per-wavefront sums over its velocities of w_k u_n dG_k at the wall
    // sides of its bands
    const double ud = lane < nq ? vel.u[k0 + lane] : 0.0, vd = lane < nq ? vel.v[k0 + lane] : 0.0,
                 wd = lane < nq ? vel.w[k0 + lane] : 0.0;
    double wsum[SWEEP_WAVE_MAX_WALLS / 64];
#pragma unroll
    for (int jc = 0; jc < SWEEP_WAVE_MAX_WALLS / 64; ++jc) {
        const int j = jc * 64 + lane;
        const bool ok = j < nw;
        const int sd = ok ? wsc[j] & 3 : 0, cell = ok ? wsc[j] >> 2 : 0;
        const int iyc = cell / nx;
        double sum = 0.0;
        if (jc * 64 < nw)
            for (int qv = 0; qv < nq; ++qv) {
                const double uu = __shfl(ud, qv, 64), vv = __shfl(vd, qv, 64), ww = __shfl(wd, qv, 64);
                const double un = ((sd & 1) ? 1.0 : -1.0) * (sd < 2 ? uu : vv);
                const int yq = band_y0(__shfl(vq_l, qv, 64) >= T(0));
                if (ok && un > 0.0 && iyc >= yq && iyc < yq + hb)
                    sum += ww * un * double(tw[(size_t)qv * tsz + (size_t)(iyc - yq) * nx + cell % nx]);
            }
        wsum[jc] = sum;
    }
    __syncthreads();   // every tile is read: the sums go where the tiles were
    double* red = (double*)tiles;   // [W][n_wall]
#pragma unroll
    for (int jc = 0; jc < SWEEP_WAVE_MAX_WALLS / 64; ++jc) {
        const int j = jc * 64 + lane;
        if (j < nw) red[(size_t)w * nw + j] = wsum[jc];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        double sacc = 0.0;
        for (int ww = 0; ww < W; ++ww) sacc += red[(size_t)ww * nw + j];
        // a block's sums accumulate over the bands (launches in order)
        double* wp = wpart + (size_t)blk * nw + j;
        *wp = (b > 0 ? *wp : 0.0) + sacc;
    }
}

// ---------------------------------------------------------------------------
// Ordered sweep with the distributions streamed through the cache hierarchy,
// for levels whose tiles do not fit in LDS next to enough wavefronts.
//
// One wavefront per velocity, lane = row and R row slots per lane as in
// k_sweep_wave, with the same one-lane rotation for the y-upwind neighbour.
// Each lane walks its own rows, so the cells it reads at successive steps are
// adjacent in memory: it loads r, the cell coefficient and the cell flags of
// the cell it will reach SD steps later into a register ring (the cache
// lines it touches are reused over the following steps) and stores each
// result directly.  The wall ghosts C_k drho_w of the velocity are formed
// once per wavefront in LDS and added when the sweep reaches their cell; the
// G values at wall cells are kept in LDS for the wall sums of the epilogue.
// No tile lives in LDS, so the footprint does not grow with the level.
// Arguments as for k_sweep_wave (wprev: n_wall <= blockDim.x).

// prefetch distance in steps (the ring takes SD x R x (NP + 2) registers)
template <typename T>
constexpr int sweep_stream_sd() {
    return sizeof(T) == 8 ? 4 : 8;
}

// LDS bytes of k_sweep_stream for W wavefronts and NP planes
template <typename T>
size_t sweep_stream_lds_bytes(int nx, int nw, int W, int NP) {
    size_t b = 64 * (size_t)W * sizeof(double)                          // dsum
               + ((size_t)nx + 5 * (size_t)nw + (size_t)W * (NP + 1) * nw) * sizeof(T) + 4 * (size_t)nw;
    return (b + 15) & ~(size_t)15;
}

template <typename T, int R, int NP>
__global__ void __launch_bounds__(512) k_sweep_stream(Geo g, Vel vel, int K_int, const T* __restrict__ r,
                                                      T* __restrict__ df, const T* __restrict__ coef_g,
                                                      const unsigned* __restrict__ flags_g,
                                                      const double* __restrict__ drho, double* __restrict__ wpart,
                                                      const double* __restrict__ wprev, int nprev,
                                                      double* __restrict__ drho_out) {
    extern __shared__ __attribute__((aligned(16))) double smem_d[];
    constexpr int SD = sweep_stream_sd<T>();
    const int nc = g.nc, nx = g.nx, ny = g.ny, nw = g.n_wall, nk = vel.nk;
    const int W = blockDim.x >> 6, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double* dsum = smem_d;                                  // [64 W]
    T* invdx = (T*)(dsum + 64 * W);                         // [nx]
    T* wl = invdx + nx;                                     // [5][n_wall]  1/d, lam_w, U_w, V_w, drho
    T* gw = wl + 5 * (size_t)nw;                            // [W][NP][n_wall]  ghost terms per wavefront
    T* wv = gw + (size_t)W * NP * nw;                       // [W][n_wall]  G at the wall cells
    int* wsc = (int*)(wv + (size_t)W * nw);                 // [n_wall]  side + 4 cell
    const int k = blockIdx.x * W + w;
    const bool kok = k < nk;
    const int kk = kok ? k : 0;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) invdx[i] = T(1.0 / g.dx[i]);
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        wl[j] = T(g.w_invd[j]);
        wl[nw + j] = T(1.0 / g.w_T[j]);
        wl[2 * nw + j] = T(g.w_U[j]);
        wl[3 * nw + j] = T(g.w_V[j]);
        wl[4 * nw + j] = drho ? T(drho[j]) : T(0);
        wsc[j] = g.w_side[j] + 4 * g.w_cell[j];
    }
    const int ng = nw > 0 ? max(1, (int)blockDim.x / nw) : 1;
    if (wprev && threadIdx.x < ng * nw) {
        int j = threadIdx.x % nw, grp = threadIdx.x / nw;
        double sacc = 0.0;
        for (int b = grp; b < nprev; b += ng) sacc += wprev[(size_t)b * nw + j];
        dsum[threadIdx.x] = sacc;
    }
    const T u = vel_u<T>(vel, kk), v = vel_v<T>(vel, kk);
    __syncthreads();
    if (wprev) {
        for (int j = threadIdx.x; j < nw; j += blockDim.x) {
            double sacc = 0.0;
            for (int grp = 0; grp < ng; ++grp) sacc += dsum[grp * nw + j];
            double dj = -sacc / g.w_den[j];
            wl[4 * nw + j] = T(dj);
            if (blockIdx.x == 0) drho_out[j] = dj;
        }
        __syncthreads();
    }
    // ghost terms of this velocity: |u_n| / d * C_k drho_w at upwind wall sides
    T* gwG = gw + (size_t)w * NP * nw;
    T* gwH = gwG + (NP == 2 ? nw : 0);
    T* wvw = wv + (size_t)w * nw;
    for (int j = lane; j < nw; j += 64) {
        const int sd = wsc[j] & 3;
        const T un = ((sd & 1) ? T(1) : T(-1)) * (sd < 2 ? u : v);
        T a = T(0), aH = T(0);
        if (un < T(0) && (drho || wprev)) {
            const T lam = wl[nw + j], du = u - wl[2 * nw + j], dv = v - wl[3 * nw + j];
            const T C = lam / T(M_PI) * dexp(-lam * (du * du + dv * dv));
            a = -un * wl[j] * (C * wl[4 * nw + j]);
            aH = -un * wl[j] * (C * T(K_int) / (T(2) * lam) * wl[4 * nw + j]);
        }
        gwG[j] = a;
        if constexpr (NP == 2) gwH[j] = aH;
        wvw[j] = T(0);
    }
    __syncthreads();

    const bool px = u >= T(0), py = v >= T(0);
    const int shx = px ? 0 : 2, shy = py ? 4 : 6;           // bit offset of the upwind x / y side type
    const T au = px ? u : -u, av = py ? v : -v;
    const size_t kc = (size_t)kk * nc, hc = ((size_t)nk + kk) * nc;
    int rowc[R];
    bool rowok[R];
    T by[R], cG[R], cH[R];
    // ring of the data of steps s .. s + SD - 1
    T qG[SD][R], qH[SD][R], qc[SD][R];
    unsigned qf[SD][R];
#pragma unroll
    for (int p = 0; p < R; ++p) {
        const int row = lane + 64 * p;
        rowok[p] = kok && row < ny;
        const int iy = rowok[p] ? (py ? row : ny - 1 - row) : 0;
        rowc[p] = iy * nx;
        by[p] = rowok[p] ? av * T(1.0 / g.dy[iy]) : T(0);
        cG[p] = T(0);
        cH[p] = T(0);
    }
    auto load = [&](int p, int s, T& rg, T& rh, T& cf, unsigned& fl) {
        const int jx = s - (lane + 64 * p);
        if (rowok[p] && (unsigned)jx < (unsigned)nx) {
            const int c = rowc[p] + (px ? jx : nx - 1 - jx);
            rg = r[kc + c];
            if constexpr (NP == 2) rh = r[hc + c];
            cf = coef_g[c];
            fl = flags_g[c];
        }
    };
#pragma unroll
    for (int i = 0; i < SD; ++i)
#pragma unroll
        for (int p = 0; p < R; ++p) {
            qG[i][p] = T(0);
            qH[i][p] = T(0);
            qc[i][p] = T(-1);
            qf[i][p] = 0u;
            load(p, i, qG[i][p], qH[i][p], qc[i][p], qf[i][p]);
        }
    const int nsteps = nx + ny - 1;
    for (int s0 = 0; s0 < nsteps; s0 += SD) {
#pragma unroll
        for (int i = 0; i < SD; ++i) {
            const int s = s0 + i;
            T rotG[R], rotH[R];
#pragma unroll
            for (int p = 0; p < R; ++p) {
                rotG[p] = lane_rotate1(cG[p]);
                if constexpr (NP == 2) rotH[p] = lane_rotate1(cH[p]);
            }
#pragma unroll
            for (int p = 0; p < R; ++p) {
                const int jx = s - (lane + 64 * p);
                const bool valid = rowok[p] && (unsigned)jx < (unsigned)nx;
                const int c = rowc[p] + (px ? jx : nx - 1 - jx);
                T rG = qG[i][p], rH = qH[i][p], cf = qc[i][p];
                const unsigned fl = qf[i][p];
                load(p, s + SD, qG[i][p], qH[i][p], qc[i][p], qf[i][p]);
                T nbG = rotG[p], nbH = NP == 2 ? rotH[p] : T(0);
                if (R > 1 && lane == 0) {
                    nbG = p > 0 ? rotG[p > 0 ? p - 1 : 0] : T(0);
                    if constexpr (NP == 2) nbH = p > 0 ? rotH[p > 0 ? p - 1 : 0] : T(0);
                }
                const unsigned tpx = (fl >> shx) & 3u, tpy = (fl >> shy) & 3u;
                const int ix = px ? jx : nx - 1 - jx;
                const T idx = invdx[valid ? ix : 0];
                const T bx = au * idx, byp = by[p];
                if (valid && (tpx == 1u || tpy == 1u)) {
                    // upwind wall sides: their ghost terms (wall sides of a
                    // cell are numbered in side order from fl >> 9)
                    int j = (int)(fl >> FLAG_WALL_SHIFT);
                    for (int q = 0; q < 4; ++q) {
                        if (((fl >> (2 * q)) & 3u) != 1u) continue;
                        if (2 * q == shx || 2 * q == shy) {
                            rG += gwG[j];
                            if constexpr (NP == 2) rH += gwH[j];
                        }
                        ++j;
                    }
                }
                const T D = cf + (tpx == 3u ? T(0) : bx) + (tpy == 3u ? T(0) : byp);
                const T inv = sweep_rcp(D);
                const T exG = tpx == 0u ? cG[p] : T(0), eyG = tpy == 0u ? nbG : T(0);
                T vG = (rG + bx * exG + byp * eyG) * inv;
                vG = cf < T(0) ? T(0) : vG;
                cG[p] = vG;
                if (valid) {
                    df[kc + c] = vG;
                    if (fl & (0x55u)) {   // a side of type 1 (wall): keep G there
                        int j = (int)(fl >> FLAG_WALL_SHIFT);
                        for (int q = 0; q < 4; ++q)
                            if (((fl >> (2 * q)) & 3u) == 1u) wvw[j++] = vG;
                    }
                }
                if constexpr (NP == 2) {
                    const T exH = tpx == 0u ? cH[p] : T(0), eyH = tpy == 0u ? nbH : T(0);
                    T vH = (rH + bx * exH + byp * eyH) * inv;
                    vH = cf < T(0) ? T(0) : vH;
                    cH[p] = vH;
                    if (valid) df[hc + c] = vH;
                }
            }
        }
    }
    __syncthreads();
    // the block's sums over its velocities of w_k u_n dG_k at the wall sides
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        const int sd = wsc[j] & 3;
        double s = 0.0;
        for (int ww = 0; ww < W; ++ww) {
            const int kw = blockIdx.x * W + ww;
            if (kw >= nk) break;
            const double un = ((sd & 1) ? 1.0 : -1.0) * (sd < 2 ? vel.u[kw] : vel.v[kw]);
            if (un > 0.0) s += vel.w[kw] * un * double(wv[(size_t)ww * nw + j]);
        }
        wpart[(size_t)blockIdx.x * nw + j] = s;
    }
}

// drho_w = -sum_b wpart[b][j] / den_j over the partial sums of the last sweep
// (per block or per velocity), in part order: one wavefront per wall side
__global__ void k_drho(Geo g, int nparts, const double* __restrict__ wpart, double* __restrict__ drho) {
    int j = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    int lane = threadIdx.x & 63;
    double s = 0.0;
    if (j < g.n_wall)
        for (int b = lane; b < nparts; b += 64) s += wpart[(size_t)b * g.n_wall + j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0 && j < g.n_wall) drho[j] = -s / g.w_den[j];
}

// renewed residual r - A df on the fine level, restricted to the coarse
// level by the volume-weighted mean (Sec. II C 1); thread per coarse cell
template <typename T>
__global__ void __launch_bounds__(256) k_defect_restrict(Geo g, Geo gc, Vel vel, int K_int,
                                                         const T* __restrict__ r, const T* __restrict__ df,
                                                         const double* __restrict__ tau_inv,
                                                         const double* __restrict__ dtn_inv,
                                                         const double* __restrict__ drho,
                                                         T* __restrict__ rc) {
    Chunk ch = chunk_of(gc.nc, vel.nk);
    if (!ch.valid) return;
    int C = ch.c, I = C % gc.nx, J = C / gc.nx;
    size_t nc = g.nc, ho = (size_t)vel.nk * nc, ncc = gc.nc, hoc = (size_t)vel.nk * ncc;
    for (int k = ch.k0 + ch.wave; k < ch.k1; k += WAVES) {
        T u = vel_u<T>(vel, k), v = vel_v<T>(vel, k);
        size_t kc = (size_t)k * nc;
        double sG = 0.0, sH = 0.0, vol = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                int c = (2 * J + a) * g.nx + 2 * I + b;
                if (g.solid[c]) continue;
                T D = T(tau_inv[c]) + T(dtn_inv[c]) + transport_diag<T>(g, c, u, v);
                int sx = u >= T(0) ? 0 : 1, sy = v >= T(0) ? 2 : 3;
                int ox = g.nb[sx * g.nc + c], oy = g.nb[sy * g.nc + c];
                // across a symmetry side: the cell's own correction at the mirror velocity
                size_t xo = ox >= 0 ? kc + ox : (ox == NB_SYMMETRY ? (size_t)vel.mx[k] * nc + c : 0);
                size_t yo = oy >= 0 ? kc + oy : (oy == NB_SYMMETRY ? (size_t)vel.my[k] * nc + c : 0);
                bool xs = ox >= 0 || ox == NB_SYMMETRY, ys = oy >= 0 || oy == NB_SYMMETRY;
                T xnG = xs ? df[xo] : T(0), xnH = xs ? df[ho + xo] : T(0);
                T ynG = ys ? df[yo] : T(0), ynH = ys ? df[ho + yo] : T(0);
                T xG, xH, yG, yH;
                upwind_term<T>(g, c, sx, u, v, K_int, xnG, xnH, drho, xG, xH);
                upwind_term<T>(g, c, sy, u, v, K_int, ynG, ynH, drho, yG, yH);
                T eG = r[kc + c] - D * df[kc + c] - xG - yG;
                T eH = r[ho + kc + c] - D * df[ho + kc + c] - xH - yH;
                double V = g.dx[c % g.nx] * g.dy[c / g.nx];
                sG += V * double(eG);
                sH += V * double(eH);
                vol += V;
            }
        size_t o = (size_t)k * ncc + C;
        rc[o] = vol > 0 ? T(sG / vol) : T(0);
        rc[hoc + o] = vol > 0 ? T(sH / vol) : T(0);
    }
}

// drho_w as k_drho, also keeping the change from
// the densities the last sweep used (old_zero: that sweep used zero)
__global__ void k_drho_delta(Geo g, int nparts, const double* __restrict__ wpart, double* __restrict__ drho,
                             double* __restrict__ ddrho, int old_zero) {
    int j = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    int lane = threadIdx.x & 63;
    double s = 0.0;
    if (j < g.n_wall)
        for (int b = lane; b < nparts; b += 64) s += wpart[(size_t)b * g.n_wall + j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0 && j < g.n_wall) {
        double d = -s / g.w_den[j];
        ddrho[j] = d - (old_zero ? 0.0 : drho[j]);
        drho[j] = d;
    }
}

// Restricted defect after a complete ordered sweep.  The sweep solves every
// cell's equation exactly with the wall densities it used, so r - A df
// vanishes except at cells with an upwind wall side, where it is that side's
// ghost term times the change of the wall density (ddrho).  cw[C] holds the
// two ranges of the fine wall list that belong to the children of coarse
// cell C (rows 2J and 2J+1), civol[C] the inverse fluid volume of C.
template <typename T>
__global__ void __launch_bounds__(256) k_defect_walls(Geo g, Geo gc, Vel vel, int K_int,
                                                      const int4* __restrict__ cw,
                                                      const double* __restrict__ civol,
                                                      const double* __restrict__ ddrho, T* __restrict__ rc,
                                                      int planes) {
    Chunk ch = chunk_of(gc.nc, vel.nk);
    if (!ch.valid) return;
    const int C = ch.c;
    const size_t ncc = gc.nc, hoc = (size_t)vel.nk * ncc;
    const int4 rg = cw[C];
    // the thread's velocities k = k0 + wave + WAVES i (statically indexed)
    double sG[MK], sH[MK], uk[MK], vk[MK];
#pragma unroll
    for (int i = 0; i < MK; ++i) {
        int k = min(ch.k0 + ch.wave + WAVES * i, vel.nk - 1);
        uk[i] = vel.u[k];
        vk[i] = vel.v[k];
        sG[i] = sH[i] = 0.0;
    }
    for (int part = 0; part < 2; ++part) {
        int j0 = part ? rg.z : rg.x, j1 = part ? rg.w : rg.y;
        for (int j = j0; j < j1; ++j) {
            // wall data once, then every velocity of the thread
            const int sd = g.w_side[j];
            const double aw = g.w_invd[j] * g.w_vol[j] * ddrho[j];
            const T lam = T(1.0 / g.w_T[j]), wu = T(g.w_U[j]), wv = T(g.w_V[j]);
            const double hfac = double(T(K_int) / (T(2) * lam));
            const double sgn = (sd & 1) ? 1.0 : -1.0;
#pragma unroll
            for (int i = 0; i < MK; ++i) {
                double un = sgn * (sd < 2 ? uk[i] : vk[i]);
                // ghost term in the sweep's type, as the sweep added it
                T du = T(uk[i]) - wu, dv = T(vk[i]) - wv;
                T Ck = lam / T(M_PI) * dexp(-lam * (du * du + dv * dv));
                double e = un < 0.0 ? -un * double(Ck) * aw : 0.0;
                sG[i] += e;
                sH[i] += e * hfac;
            }
        }
    }
    const double iv = civol[C];
#pragma unroll
    for (int i = 0; i < MK; ++i) {
        int k = ch.k0 + ch.wave + WAVES * i;
        if (k < ch.k1) {
            rc[(size_t)k * ncc + C] = T(sG[i] * iv);
            if (planes == 2) rc[hoc + (size_t)k * ncc + C] = T(sH[i] * iv);
        }
    }
}

// Full-multigrid start (Sec. III C): the distribution itself, not a
// correction, moves between levels.
//
// fc = volume-weighted mean of f over the fluid children of every coarse
// cell (the restriction of Sec. II C 1; zero where no child is fluid), both
// planes, level layout [2][Nk][nc]
template <typename T>
__global__ void __launch_bounds__(256) k_restrict_full(Geo g, Geo gc, Vel vel, const T* __restrict__ f,
                                                       T* __restrict__ fc) {
    Chunk ch = chunk_of(gc.nc, vel.nk);
    if (!ch.valid) return;
    const int C = ch.c, I = C % gc.nx, J = C / gc.nx;
    const size_t nc = g.nc, ho = (size_t)vel.nk * nc, ncc = gc.nc, hoc = (size_t)vel.nk * ncc;
    int cc[4];
    double V[4], vol = 0.0;
    for (int a = 0; a < 4; ++a) {
        int c = (2 * J + (a >> 1)) * g.nx + 2 * I + (a & 1);
        cc[a] = c;
        V[a] = g.solid[c] ? 0.0 : g.dx[c % g.nx] * g.dy[c / g.nx];
        vol += V[a];
    }
    const double iv = vol > 0.0 ? 1.0 / vol : 0.0;
    for (int k = ch.k0 + ch.wave; k < ch.k1; k += WAVES) {
        size_t kc = (size_t)k * nc;
        double sG = 0.0, sH = 0.0;
        for (int a = 0; a < 4; ++a) {
            sG += V[a] * double(f[kc + cc[a]]);
            sH += V[a] * double(f[ho + kc + cc[a]]);
        }
        fc[(size_t)k * ncc + C] = T(sG * iv);
        fc[hoc + (size_t)k * ncc + C] = T(sH * iv);
    }
}

// f = FMG interpolation of fc on every fluid cell of the fine level: the
// bilinear prolongation (Sec. II C 3) where its stencil interpolates (every
// weight non-negative), the parent cell's value where it would extrapolate,
// so that a positive distribution stays positive; zero on solid cells; both
// planes
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_full(Geo g, Vel vel, int ncc, const T* __restrict__ fc,
                                                      T* __restrict__ f) {
    Chunk ch = chunk_of(g.nc, vel.nk);
    if (!ch.valid) return;
    const int c = ch.c;
    const size_t nc = g.nc, ho = (size_t)vel.nk * nc, hoc = (size_t)vel.nk * ncc;
    const bool solid = g.solid[c];
    int id[4];
    double w[4];
    bool inside = true;
    for (int a = 0; a < 4; ++a) {
        id[a] = solid ? 0 : g.p_idx[a * g.nc + c];
        w[a] = solid ? 0.0 : g.p_w[a * g.nc + c];
        inside = inside && w[a] >= 0.0;
    }
    if (!inside)   // the parent alone (stencil entry 0)
        for (int a = 0; a < 4; ++a) w[a] = a == 0 ? 1.0 : 0.0;
    for (int k = ch.k0 + ch.wave; k < ch.k1; k += WAVES) {
        size_t kc = (size_t)k * ncc;
        double aG = 0.0, aH = 0.0;
        for (int a = 0; a < 4; ++a) {
            aG += w[a] * double(fc[kc + id[a]]);
            aH += w[a] * double(fc[hoc + kc + id[a]]);
        }
        f[(size_t)k * nc + c] = T(aG);
        f[ho + (size_t)k * nc + c] = T(aH);
    }
}

// df_fine += I_H^h df_coarse (bilinear with extrapolation, Sec. II C 3)
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(Geo g, Vel vel, int ncc, const T* __restrict__ dfc,
                                                     T* __restrict__ df) {
    Chunk ch = chunk_of(g.nc, vel.nk);
    if (!ch.valid) return;
    int c = ch.c;
    if (g.solid[c]) return;
    size_t nc = g.nc, ho = (size_t)vel.nk * nc, hoc = (size_t)vel.nk * ncc;
    int id[4];
    T w[4];
    for (int a = 0; a < 4; ++a) {
        id[a] = g.p_idx[a * g.nc + c];
        w[a] = T(g.p_w[a * g.nc + c]);
    }
    for (int k = ch.k0 + ch.wave; k < ch.k1; k += WAVES) {
        size_t kc = (size_t)k * ncc;
        T aG = w[0] * dfc[kc + id[0]] + w[1] * dfc[kc + id[1]] + w[2] * dfc[kc + id[2]] + w[3] * dfc[kc + id[3]];
        T aH = w[0] * dfc[hoc + kc + id[0]] + w[1] * dfc[hoc + kc + id[1]] + w[2] * dfc[hoc + kc + id[2]] +
               w[3] * dfc[hoc + kc + id[3]];
        df[(size_t)k * nc + c] += aG;
        df[ho + (size_t)k * nc + c] += aH;
    }
}

// restrict a per-cell double field (volume-weighted mean over fluid children)
__device__ __forceinline__ void restrict_cell(const Geo& g, const Geo& gc, int m, const double* __restrict__ a,
                                              double* __restrict__ ac, int C) {
    int I = C % gc.nx, J = C / gc.nx;
    for (int q = 0; q < m; ++q) {
        double s = 0.0, vol = 0.0;
        for (int aa = 0; aa < 2; ++aa)
            for (int b = 0; b < 2; ++b) {
                int c = (2 * J + aa) * g.nx + 2 * I + b;
                if (g.solid[c]) continue;
                double V = g.dx[c % g.nx] * g.dy[c / g.nx];
                s += V * a[(size_t)q * g.nc + c];
                vol += V;
            }
        ac[(size_t)q * gc.nc + C] = vol > 0 ? s / vol : 0.0;
    }
}

__global__ void k_restrict_cells(Geo g, Geo gc, int m, const double* __restrict__ a, double* __restrict__ ac) {
    int C = blockIdx.x * blockDim.x + threadIdx.x;
    if (C < gc.nc) restrict_cell(g, gc, m, a, ac, C);
}

// ---------------------------------------------------------------------------
// Step 2: FAS cycle of the macroscopic prediction (Sec. II A 1, Sec. II C 2)

__device__ __forceinline__ void euler_flux(const double* W, int d, double sign, double K, double* F) {
    double rho = W[0], U = W[1] / rho, V = W[2] / rho;
    double p = (2.0 / K) * (W[3] - 0.5 * rho * (U * U + V * V));
    double un = sign * (d == 0 ? U : V);
    F[0] = rho * un;
    F[1] = W[1] * un + (d == 0 ? sign * p : 0.0);
    F[2] = W[2] * un + (d == 1 ? sign * p : 0.0);
    F[3] = (W[3] + p) * un;
}

// state across side s of cell c: neighbour, wall ghost (Sec. III B wall
// relation), freestream, copy or mirror image; kind 0 interior, 1 farfield,
// 2 outflow, 3 wall, 4 symmetry
__device__ __forceinline__ int side_state(const Geo& g, const Gas& gas, const double* W, int c, int s,
                                          const double* Wi, double* Wj, int& wall) {
    int code = g.nb[s * g.nc + c];
    if (code >= 0) {
        for (int m = 0; m < 4; ++m) Wj[m] = W[m * g.nc + code];
        return 0;
    }
    if (code == NB_FARFIELD) {
        for (int m = 0; m < 4; ++m) Wj[m] = gas.W_inf[m];
        return 1;
    }
    if (code == NB_OUTFLOW) {
        for (int m = 0; m < 4; ++m) Wj[m] = Wi[m];
        return 2;
    }
    if (code == NB_SYMMETRY) {   // mirror image: the normal momentum reversed
        for (int m = 0; m < 4; ++m) Wj[m] = Wi[m];
        Wj[1 + (s >> 1)] = -Wi[1 + (s >> 1)];
        return 4;
    }
    wall = wall_of(code);
    double rho, U, V, lam;
    prim_of_r(Wi, gas.K, rho, U, V, lam);
    cons_of(rho, 2.0 * g.w_U[wall] - U, 2.0 * g.w_V[wall] - V, 2.0 * rcp_refined(g.w_T[wall]) - lam, gas.K, Wj);
    return 3;
}

// Gamma per side (frozen for a level visit): mean primitive state of the cell
// and its neighbour or ghost
__device__ __forceinline__ void fas_gamma_cell(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                               double* __restrict__ Gam, int c) {
    if (g.solid[c]) {
        for (int s = 0; s < 4; ++s) Gam[s * g.nc + c] = 0.0;
        return;
    }
    double Wi[4], Wj[4];
    for (int m = 0; m < 4; ++m) Wi[m] = W[m * g.nc + c];
    double ri, Ui, Vi, li;
    prim_of(Wi, gas.K, ri, Ui, Vi, li);
    for (int s = 0; s < 4; ++s) {
        int wall = -1;
        side_state(g, gas, W, c, s, Wi, Wj, wall);
        double rj, Uj, Vj, lj;
        prim_of(Wj, gas.K, rj, Uj, Vj, lj);
        double rm = 0.5 * (ri + rj), Um = 0.5 * (Ui + Uj), Vm = 0.5 * (Vi + Vj);
        double Tm = 0.5 * (1.0 / li + 1.0 / lj);
        double un = fabs(s < 2 ? Um : Vm);
        double as = sqrt(gas.gamma * Tm / 2.0);
        double nu = mu_of(gas, Tm) / rm;
        Gam[s * g.nc + c] = un + as + 2.0 * nu / g.dcent[s * g.nc + c];
    }
}

// out = base + sgn * R_split(W), R_split_i = -(1/V_i) sum_j S_ij F_ij(W)
__device__ __forceinline__ void fas_rsplit_cell(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                                const double* __restrict__ Gam, const double* __restrict__ base,
                                                double sgn, double* __restrict__ out, int c) {
    if (g.solid[c]) {
        for (int m = 0; m < 4; ++m) out[m * g.nc + c] = 0.0;
        return;
    }
    double Wi[4], Wj[4], Fi[4], Fj[4], acc[4] = {0, 0, 0, 0};
    for (int m = 0; m < 4; ++m) Wi[m] = W[m * g.nc + c];
    double dx = g.dx[c % g.nx], dy = g.dy[c / g.nx];
    for (int s = 0; s < 4; ++s) {
        int wall = -1;
        side_state(g, gas, W, c, s, Wi, Wj, wall);
        int d = s >> 1;
        double sign = (s & 1) ? 1.0 : -1.0;
        euler_flux(Wi, d, sign, gas.K, Fi);
        euler_flux(Wj, d, sign, gas.K, Fj);
        double S = d == 0 ? dy : dx, G = Gam[s * g.nc + c];
        for (int m = 0; m < 4; ++m) acc[m] += S * 0.5 * (Fi[m] + Fj[m] + G * (Wi[m] - Wj[m]));
    }
    double V = dx * dy;
    for (int m = 0; m < 4; ++m) out[m * g.nc + c] = base[m * g.nc + c] + sgn * (-acc[m] / V);
}

// one red-black half-sweep of the linearised defect equation of Sec. II A 1
// on cell c (if it has the colour)
__device__ __forceinline__ void fas_halfsweep_cell(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                                   double* __restrict__ E, const double* __restrict__ Rm,
                                                   const double* __restrict__ Gam,
                                                   const double* __restrict__ dtn_inv, int colour, int c) {
    int ix = c % g.nx, iy = c / g.nx;
    if (((ix + iy) & 1) != colour || g.solid[c]) return;
    double Wi[4], Ei[4], Wj[4], Ej[4], A[4], B[4], acc[4] = {0, 0, 0, 0};
    for (int m = 0; m < 4; ++m) {
        Wi[m] = W[m * g.nc + c];
        Ei[m] = E[m * g.nc + c];
    }
    double dx = g.dx[ix], dy = g.dy[iy], V = dx * dy, Dsum = 0.0;
    for (int s = 0; s < 4; ++s) {
        int wall = -1;
        int kind = side_state(g, gas, W, c, s, Wi, Wj, wall);
        int d = s >> 1;
        double sign = (s & 1) ? 1.0 : -1.0;
        double S = d == 0 ? dy : dx, G = Gam[s * g.nc + c];
        if (kind == 0) {
            int o = g.nb[s * g.nc + c];
            for (int m = 0; m < 4; ++m) Ej[m] = E[m * g.nc + o];
        } else if (kind == 1) {
            for (int m = 0; m < 4; ++m) Ej[m] = 0.0;
        } else if (kind == 2) {
            for (int m = 0; m < 4; ++m) Ej[m] = Ei[m];
        } else if (kind == 4) {
            for (int m = 0; m < 4; ++m) Ej[m] = Ei[m];
            Ej[1 + d] = -Ei[1 + d];
        } else {
            // linearised wall ghost dW_j = J dW_i (Sec. III B), K total degrees of freedom
            double rho, U, V2, lam;
            prim_of(Wi, gas.K, rho, U, V2, lam);
            double Uw = g.w_U[wall], Vw = g.w_V[wall], lw = 1.0 / g.w_T[wall];
            double Y = lam / (lam - 2.0 * lw);
            Ej[0] = Ei[0];
            Ej[1] = 2.0 * Uw * Ei[0] - Ei[1];
            Ej[2] = 2.0 * Vw * Ei[0] - Ei[2];
            Ej[3] = (2.0 * (Uw * Uw + Vw * Vw) - 0.5 * (U * U + V2 * V2) * (1.0 + Y * Y) +
                     gas.K / (4.0 * lam) * (Y * Y - Y)) * Ei[0] +
                    (U - 2.0 * Uw + U * Y * Y) * Ei[1] + (V2 - 2.0 * Vw + V2 * Y * Y) * Ei[2] - Y * Y * Ei[3];
        }
        double WE[4];
        for (int m = 0; m < 4; ++m) WE[m] = Wj[m] + Ej[m];
        euler_flux(WE, d, sign, gas.K, A);
        euler_flux(Wj, d, sign, gas.K, B);
        for (int m = 0; m < 4; ++m) acc[m] += S * (A[m] - B[m] - G * Ej[m]);
        Dsum += S * G;
    }
    double D = Dsum / (2.0 * V) + dtn_inv[c];
    for (int m = 0; m < 4; ++m) E[m * g.nc + c] = (Rm[m * g.nc + c] - acc[m] / (2.0 * V)) / D;
}

// W += E (fluid cells) and clear E
__device__ __forceinline__ void fas_apply_cell(const Geo& g, double* __restrict__ W, double* __restrict__ E, int c) {
    for (int m = 0; m < 4; ++m) {
        if (!g.solid[c]) W[m * g.nc + c] += E[m * g.nc + c];
        E[m * g.nc + c] = 0.0;
    }
}

// W_fine += I_H^h (W_coarse - W0_coarse)
__device__ __forceinline__ void fas_prolong_cell(const Geo& g, int ncc, const double* __restrict__ Wc,
                                                 const double* __restrict__ Wc0, double* __restrict__ W, int c) {
    if (g.solid[c]) return;
    for (int m = 0; m < 4; ++m) {
        double s = 0.0;
        for (int a = 0; a < 4; ++a) {
            int id = g.p_idx[a * g.nc + c];
            s += g.p_w[a * g.nc + c] * (Wc[(size_t)m * ncc + id] - Wc0[(size_t)m * ncc + id]);
        }
        W[m * g.nc + c] += s;
    }
}

// --- the same operations with four lanes per cell, lane s taking side s
// (and conservative component s where a cell writes its four results); the
// four consecutive lanes of a cell add their side terms by two butterfly
// shuffles.  Used by the kernels below: a cell's dependent chain of FP64
// work is a quarter as long, which is what bounds these small levels.

// lane i of every group of four takes lane i ^ m (m = 1, 2) by a DPP quad
// permutation (quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E)
template <int CTRL>
__device__ __forceinline__ double quad_perm(double x) {
    unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double quad_sum(double x) {
    x += quad_perm<0xB1>(x);
    x += quad_perm<0x4E>(x);
    return x;
}


// Euler flux of W through a side of normal sign * e_d (division-free: the
// reciprocal density is refined to full precision)
__device__ __forceinline__ void euler_flux_r(const double* W, int d, double sign, double K, double* F) {
    double ir = rcp_refined(W[0]);
    double U = W[1] * ir, V = W[2] * ir;
    double p = (2.0 / K) * (W[3] - 0.5 * W[0] * (U * U + V * V));
    double un = sign * (d == 0 ? U : V);
    F[0] = W[0] * un;
    F[1] = W[1] * un + (d == 0 ? sign * p : 0.0);
    F[2] = W[2] * un + (d == 1 ? sign * p : 0.0);
    F[3] = (W[3] + p) * un;
}

__device__ __forceinline__ double fas_gamma_side(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                                 int c, int s) {
    double Wi[4], Wj[4];
    for (int m = 0; m < 4; ++m) Wi[m] = W[m * g.nc + c];
    int wall = -1;
    side_state(g, gas, W, c, s, Wi, Wj, wall);
    double ri, Ui, Vi, li, rj, Uj, Vj, lj;
    prim_of(Wi, gas.K, ri, Ui, Vi, li);
    prim_of(Wj, gas.K, rj, Uj, Vj, lj);
    double rm = 0.5 * (ri + rj), Um = 0.5 * (Ui + Uj), Vm = 0.5 * (Vi + Vj);
    double Tm = 0.5 * (1.0 / li + 1.0 / lj);
    double un = fabs(s < 2 ? Um : Vm);
    double as = sqrt(gas.gamma * Tm / 2.0);
    double nu = mu_of(gas, Tm) / rm;
    return un + as + 2.0 * nu / g.dcent[s * g.nc + c];
}

// side-s term of sum_j S_ij F_ij(W) (the split flux of Sec. II A 1)
__device__ __forceinline__ void fas_rsplit_side(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                                double G, int c, int s, double* acc) {
    double Wi[4], Wj[4], Fi[4], Fj[4];
    for (int m = 0; m < 4; ++m) Wi[m] = W[m * g.nc + c];
    int wall = -1;
    side_state(g, gas, W, c, s, Wi, Wj, wall);
    int d = s >> 1;
    double sign = (s & 1) ? 1.0 : -1.0;
    euler_flux_r(Wi, d, sign, gas.K, Fi);
    euler_flux_r(Wj, d, sign, gas.K, Fj);
    double S = d == 0 ? g.dy[c / g.nx] : g.dx[c % g.nx];
    for (int m = 0; m < 4; ++m) acc[m] = S * 0.5 * (Fi[m] + Fj[m] + G * (Wi[m] - Wj[m]));
}

// side-s terms of the linearised defect equation of one half-sweep:
// S (F(W_j + E_j) - F(W_j) - Gam E_j) and S Gam
__device__ __forceinline__ void fas_half_side(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                              const double* __restrict__ E, const double* __restrict__ Gam,
                                              int c, int s, double* acc, double& sg) {
    double Wi[4], Ei[4], Wj[4], Ej[4], A[4], B[4];
    for (int m = 0; m < 4; ++m) {
        Wi[m] = W[m * g.nc + c];
        Ei[m] = E[m * g.nc + c];
    }
    int wall = -1;
    int kind = side_state(g, gas, W, c, s, Wi, Wj, wall);
    int d = s >> 1;
    double sign = (s & 1) ? 1.0 : -1.0;
    double S = d == 0 ? g.dy[c / g.nx] : g.dx[c % g.nx], G = Gam[s * g.nc + c];
    if (kind == 0) {
        int o = g.nb[s * g.nc + c];
        for (int m = 0; m < 4; ++m) Ej[m] = E[m * g.nc + o];
    } else if (kind == 1) {
        for (int m = 0; m < 4; ++m) Ej[m] = 0.0;
    } else if (kind == 2) {
        for (int m = 0; m < 4; ++m) Ej[m] = Ei[m];
    } else if (kind == 4) {
        for (int m = 0; m < 4; ++m) Ej[m] = Ei[m];
        Ej[1 + d] = -Ei[1 + d];
    } else {
        // linearised wall ghost dW_j = J dW_i (Sec. III B), K total degrees of freedom
        double rho, U, V2, lam;
        prim_of_r(Wi, gas.K, rho, U, V2, lam);
        double Uw = g.w_U[wall], Vw = g.w_V[wall], lw = rcp_refined(g.w_T[wall]);
        double Y = lam * rcp_refined(lam - 2.0 * lw);
        Ej[0] = Ei[0];
        Ej[1] = 2.0 * Uw * Ei[0] - Ei[1];
        Ej[2] = 2.0 * Vw * Ei[0] - Ei[2];
        Ej[3] = (2.0 * (Uw * Uw + Vw * Vw) - 0.5 * (U * U + V2 * V2) * (1.0 + Y * Y) +
                 gas.K * rcp_refined(4.0 * lam) * (Y * Y - Y)) * Ei[0] +
                (U - 2.0 * Uw + U * Y * Y) * Ei[1] + (V2 - 2.0 * Vw + V2 * Y * Y) * Ei[2] - Y * Y * Ei[3];
    }
    double WE[4];
    for (int m = 0; m < 4; ++m) WE[m] = Wj[m] + Ej[m];
    euler_flux_r(WE, d, sign, gas.K, A);
    euler_flux_r(Wj, d, sign, gas.K, B);
    for (int m = 0; m < 4; ++m) acc[m] = S * (A[m] - B[m] - G * Ej[m]);
    sg = S * G;
}

// phases with four lanes per cell: item t = 4 c + s over [0, 4 nc)

// entering a level: W0 := W, the frozen Gamma of every side and the forcing
// P = R - R_split(W0) (lane s uses the Gamma of side s it has just formed)
__device__ __forceinline__ void fas4_enter(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                           double* __restrict__ W0, double* __restrict__ Gam,
                                           const double* __restrict__ R, double* __restrict__ P, int t) {
    int c = t >> 2, s = t & 3;
    bool solid = g.solid[c];
    W0[s * g.nc + c] = W[s * g.nc + c];
    double G = solid ? 0.0 : fas_gamma_side(g, gas, W, c, s);
    Gam[s * g.nc + c] = G;
    double acc[4] = {0, 0, 0, 0};
    if (!solid) fas_rsplit_side(g, gas, W, G, c, s, acc);
    double tot[4];
    for (int m = 0; m < 4; ++m) tot[m] = quad_sum(acc[m]);
    double iv = 1.0 / (g.dx[c % g.nx] * g.dy[c / g.nx]);
    double mine = s == 0 ? tot[0] : s == 1 ? tot[1] : s == 2 ? tot[2] : tot[3];
    P[s * g.nc + c] = solid ? 0.0 : R[s * g.nc + c] + mine * iv;
}

// out = base + sgn * R_split(W), R_split_i = -(1/V_i) sum_j S_ij F_ij(W);
// E != nullptr: also clear E (a smoothing restarts its correction from zero)
__device__ __forceinline__ void fas4_rsplit(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                            const double* __restrict__ Gam, const double* __restrict__ base,
                                            double sgn, double* __restrict__ out, double* __restrict__ E, int t) {
    int c = t >> 2, s = t & 3;
    bool solid = g.solid[c];
    double acc[4] = {0, 0, 0, 0};
    if (!solid) fas_rsplit_side(g, gas, W, Gam[s * g.nc + c], c, s, acc);
    double tot[4];
    for (int m = 0; m < 4; ++m) tot[m] = quad_sum(acc[m]);
    double iv = 1.0 / (g.dx[c % g.nx] * g.dy[c / g.nx]);
    double mine = s == 0 ? tot[0] : s == 1 ? tot[1] : s == 2 ? tot[2] : tot[3];
    out[s * g.nc + c] = solid ? 0.0 : base[s * g.nc + c] + sgn * (-mine * iv);
    if (E) E[s * g.nc + c] = 0.0;
}

// the first phase of a smoothing: the renewed residual Rm = P + R_split(W)
// and the first half-sweep (colour 0) together.  E starts from zero, so in
// that half-sweep every side term F(W_j + E_j) - F(W_j) - Gam E_j is zero and
// a colour-0 cell's correction is Rm / D (D = sum S Gam / (2 V) + 1/dt_n);
// colour-1 and solid cells get E = 0
__device__ __forceinline__ void fas4_rsplit_first(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                                  const double* __restrict__ Gam, const double* __restrict__ P,
                                                  const double* __restrict__ dtn_inv, double* __restrict__ Rm,
                                                  double* __restrict__ E, int t) {
    int c = t >> 2, s = t & 3;
    int ix = c % g.nx, iy = c / g.nx;
    bool solid = g.solid[c];
    double G = Gam[s * g.nc + c];
    double acc[4] = {0, 0, 0, 0};
    if (!solid) fas_rsplit_side(g, gas, W, G, c, s, acc);
    double tot[4];
    for (int m = 0; m < 4; ++m) tot[m] = quad_sum(acc[m]);
    double S = (s >> 1) == 0 ? g.dy[iy] : g.dx[ix];
    double Dsum = quad_sum(S * G);
    double iv = 1.0 / (g.dx[ix] * g.dy[iy]);
    double mine = s == 0 ? tot[0] : s == 1 ? tot[1] : s == 2 ? tot[2] : tot[3];
    double rm = solid ? 0.0 : P[s * g.nc + c] + 1.0 * (-mine * iv);
    Rm[s * g.nc + c] = rm;
    double e = 0.0;
    if (!solid && ((ix + iy) & 1) == 0) {
        double ih = rcp_refined(2.0 * g.dx[ix] * g.dy[iy]);
        double D = Dsum * ih + dtn_inv[c];
        e = rm * rcp_refined(D);
    }
    E[s * g.nc + c] = e;
}

// new correction of a cell of the given colour from the linearised defect
// equation (lanes of the cell only; the caller guarantees the colour)
__device__ __forceinline__ double fas4_half_value(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                                  const double* __restrict__ E, const double* __restrict__ Rm,
                                                  const double* __restrict__ Gam,
                                                  const double* __restrict__ dtn_inv, int c, int s) {
    int ix = c % g.nx, iy = c / g.nx;
    double acc[4], sg;
    fas_half_side(g, gas, W, E, Gam, c, s, acc, sg);
    double tot[4];
    for (int m = 0; m < 4; ++m) tot[m] = quad_sum(acc[m]);
    double Dsum = quad_sum(sg);
    double ih = rcp_refined(2.0 * g.dx[ix] * g.dy[iy]);   // 1 / (2 V)
    double D = Dsum * ih + dtn_inv[c];
    double mine = s == 0 ? tot[0] : s == 1 ? tot[1] : s == 2 ? tot[2] : tot[3];
    return (Rm[s * g.nc + c] - mine * ih) * rcp_refined(D);
}

// one red-black half-sweep on the cells of the given colour
__device__ __forceinline__ void fas4_halfsweep(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                               double* __restrict__ E, const double* __restrict__ Rm,
                                               const double* __restrict__ Gam,
                                               const double* __restrict__ dtn_inv, int colour, int t) {
    int c = t >> 2, s = t & 3;
    int ix = c % g.nx, iy = c / g.nx;
    if (((ix + iy) & 1) != colour || g.solid[c]) return;   // all four lanes of the cell alike
    double e = fas4_half_value(g, gas, W, E, Rm, Gam, dtn_inv, c, s);
    E[s * g.nc + c] = e;
}

// the last half-sweep of a smoothing (colour 0) together with W += E: the
// result goes to Wout (neighbours still read W, the linearisation point)
__device__ __forceinline__ void fas4_halfsweep_apply(const Geo& g, const Gas& gas, const double* __restrict__ W,
                                                     const double* __restrict__ E, const double* __restrict__ Rm,
                                                     const double* __restrict__ Gam,
                                                     const double* __restrict__ dtn_inv,
                                                     double* __restrict__ Wout, int t) {
    int c = t >> 2, s = t & 3;
    int ix = c % g.nx, iy = c / g.nx;
    bool solid = g.solid[c];
    double e = E[s * g.nc + c];
    if (((ix + iy) & 1) == 0 && !solid) e = fas4_half_value(g, gas, W, E, Rm, Gam, dtn_inv, c, s);
    Wout[s * g.nc + c] = W[s * g.nc + c] + (solid ? 0.0 : e);
}

// Wout = W + I_H^h (W_coarse - W0_coarse) (fluid cells; solid cells copied)
__device__ __forceinline__ void fas4_prolong(const Geo& g, int ncc, const double* __restrict__ Wc,
                                             const double* __restrict__ Wc0, const double* __restrict__ W,
                                             double* __restrict__ Wout, int t) {
    int c = t >> 2, m = t & 3;
    double s = 0.0;
    if (!g.solid[c])
        for (int a = 0; a < 4; ++a) {
            int id = g.p_idx[a * g.nc + c];
            s += g.p_w[a * g.nc + c] * (Wc[(size_t)m * ncc + id] - Wc0[(size_t)m * ncc + id]);
        }
    Wout[m * g.nc + c] = W[m * g.nc + c] + s;
}

// component m of coarse cell C: volume-weighted mean over fluid children
__device__ __forceinline__ void restrict_comp(const Geo& g, const Geo& gc, const double* __restrict__ a,
                                              double* __restrict__ ac, int C, int m) {
    int I = C % gc.nx, J = C / gc.nx;
    double s = 0.0, vol = 0.0;
    for (int aa = 0; aa < 2; ++aa)
        for (int b = 0; b < 2; ++b) {
            int c = (2 * J + aa) * g.nx + 2 * I + b;
            if (g.solid[c]) continue;
            double V = g.dx[c % g.nx] * g.dy[c / g.nx];
            s += V * a[(size_t)m * g.nc + c];
            vol += V;
        }
    ac[(size_t)m * gc.nc + C] = vol > 0 ? s / vol : 0.0;
}

#define ITEM4_KERNEL_INDEX                              \
    int t = blockIdx.x * blockDim.x + threadIdx.x;      \
    if (t >= 4 * g.nc) return;

__global__ void k_fas4_enter(Geo g, Gas gas, const double* __restrict__ W, double* __restrict__ W0,
                             double* __restrict__ Gam, const double* __restrict__ R, double* __restrict__ P) {
    ITEM4_KERNEL_INDEX
    fas4_enter(g, gas, W, W0, Gam, R, P, t);
}

__global__ void k_fas4_rsplit(Geo g, Gas gas, const double* __restrict__ W, const double* __restrict__ Gam,
                              const double* __restrict__ base, double sgn, double* __restrict__ out,
                              double* __restrict__ E) {
    ITEM4_KERNEL_INDEX
    fas4_rsplit(g, gas, W, Gam, base, sgn, out, E, t);
}

__global__ void k_fas4_rsplit_first(Geo g, Gas gas, const double* __restrict__ W, const double* __restrict__ Gam,
                                    const double* __restrict__ P, const double* __restrict__ dtn_inv,
                                    double* __restrict__ Rm, double* __restrict__ E) {
    ITEM4_KERNEL_INDEX
    fas4_rsplit_first(g, gas, W, Gam, P, dtn_inv, Rm, E, t);
}

__global__ void k_fas4_halfsweep(Geo g, Gas gas, const double* __restrict__ W, double* __restrict__ E,
                                 const double* __restrict__ Rm, const double* __restrict__ Gam,
                                 const double* __restrict__ dtn_inv, int colour) {
    ITEM4_KERNEL_INDEX
    fas4_halfsweep(g, gas, W, E, Rm, Gam, dtn_inv, colour, t);
}

__global__ void k_fas4_halfsweep_apply(Geo g, Gas gas, const double* __restrict__ W, const double* __restrict__ E,
                                       const double* __restrict__ Rm, const double* __restrict__ Gam,
                                       const double* __restrict__ dtn_inv, double* __restrict__ Wout) {
    ITEM4_KERNEL_INDEX
    fas4_halfsweep_apply(g, gas, W, E, Rm, Gam, dtn_inv, Wout, t);
}

__global__ void k_fas4_prolong(Geo g, int ncc, const double* __restrict__ Wc, const double* __restrict__ Wc0,
                               const double* __restrict__ W, double* __restrict__ Wout) {
    ITEM4_KERNEL_INDEX
    fas4_prolong(g, ncc, Wc, Wc0, W, Wout, t);
}

// W and R of level l + 1 from level l (fine W and the renewed residual)
__global__ void k_fas4_restrict(Geo g, Geo gc, const double* __restrict__ W, const double* __restrict__ Rm,
                                double* __restrict__ Wc, double* __restrict__ Rc) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * gc.nc) return;
    restrict_comp(g, gc, W, Wc, t >> 2, t & 3);
    restrict_comp(g, gc, Rm, Rc, t >> 2, t & 3);
}

#define CELL_KERNEL_INDEX                               \
    int c = blockIdx.x * blockDim.x + threadIdx.x;      \
    if (c >= g.nc) return;

__global__ void k_fas_gamma(Geo g, Gas gas, const double* __restrict__ W, double* __restrict__ Gam) {
    CELL_KERNEL_INDEX
    fas_gamma_cell(g, gas, W, Gam, c);
}

__global__ void k_fas_rsplit(Geo g, Gas gas, const double* __restrict__ W, const double* __restrict__ Gam,
                             const double* __restrict__ base, double sgn, double* __restrict__ out) {
    CELL_KERNEL_INDEX
    fas_rsplit_cell(g, gas, W, Gam, base, sgn, out, c);
}

__global__ void k_fas_halfsweep(Geo g, Gas gas, const double* __restrict__ W, double* __restrict__ E,
                                const double* __restrict__ Rm, const double* __restrict__ Gam,
                                const double* __restrict__ dtn_inv, int colour) {
    CELL_KERNEL_INDEX
    fas_halfsweep_cell(g, gas, W, E, Rm, Gam, dtn_inv, colour, c);
}

__global__ void k_fas_apply(Geo g, double* __restrict__ W, double* __restrict__ E) {
    CELL_KERNEL_INDEX
    fas_apply_cell(g, W, E, c);
}

__global__ void k_fas_prolong(Geo g, int ncc, const double* __restrict__ Wc, const double* __restrict__ Wc0,
                              double* __restrict__ W) {
    CELL_KERNEL_INDEX
    fas_prolong_cell(g, ncc, Wc, Wc0, W, c);
}

// The FAS V-cycle on levels l0 .. L-1, all in one workgroup: every phase of
// the recursion (copy, Gamma, forcing, smoothing sweeps, renewal,
// restriction, prolongation) is a loop over the cells of one level followed
// by a workgroup barrier.  Used for the small levels, where a phase is far
// shorter than a kernel launch.
constexpr int FAS_MAXL = 8;

struct FasSet {
    int l0, L, nu1, nu2, nuc;
    Geo geo[FAS_MAXL];
    double *W[FAS_MAXL], *W0[FAS_MAXL], *R[FAS_MAXL], *P[FAS_MAXL], *E[FAS_MAXL], *Gam[FAS_MAXL],
        *Rm[FAS_MAXL], *dtn[FAS_MAXL], *W2[FAS_MAXL];
};

// current W of level l: W[l] or W2[l] by bit l of par (every thread swaps
// alike, so the choice needs no shared state)
__device__ __forceinline__ double* fas_w(const FasSet& F, unsigned par, int l) {
    return ((par >> l) & 1u) ? F.W2[l] : F.W[l];
}
__device__ __forceinline__ double* fas_walt(const FasSet& F, unsigned par, int l) {
    return ((par >> l) & 1u) ? F.W[l] : F.W2[l];
}

// smoothings of Sec. II C 2: renewed residual (E cleared), half-sweeps of
// colours 0 and 1, and the last colour-0 half-sweep with W += E into the
// other W buffer
__device__ __forceinline__ void fas_block_smooth(const FasSet& F, const Gas& gas, int l, int count,
                                                 unsigned& par) {
    const Geo& g = F.geo[l];
    const int n4 = 4 * g.nc;
    for (int it = 0; it < count; ++it) {
        const double* W = fas_w(F, par, l);
        for (int t = threadIdx.x; t < n4; t += blockDim.x)
            fas4_rsplit_first(g, gas, W, F.Gam[l], F.P[l], F.dtn[l], F.Rm[l], F.E[l], t);
        __syncthreads();
        for (int t = threadIdx.x; t < n4; t += blockDim.x)
            fas4_halfsweep(g, gas, W, F.E[l], F.Rm[l], F.Gam[l], F.dtn[l], 1, t);
        __syncthreads();
        for (int t = threadIdx.x; t < n4; t += blockDim.x)
            fas4_halfsweep_apply(g, gas, W, F.E[l], F.Rm[l], F.Gam[l], F.dtn[l], fas_walt(F, par, l), t);
        __syncthreads();
        par ^= 1u << l;
    }
}

__device__ __forceinline__ void fas_block_enter(const FasSet& F, const Gas& gas, int l, unsigned par) {
    const Geo& g = F.geo[l];
    const int n4 = 4 * g.nc;
    for (int t = threadIdx.x; t < n4; t += blockDim.x)
        fas4_enter(g, gas, fas_w(F, par, l), F.W0[l], F.Gam[l], F.R[l], F.P[l], t);
    __syncthreads();
}

// LDS layout of k_fas_cycle_block: for every level from l0 on, the FAS
// arrays (W, W0, R, P, E, Gam, Rm: 4 per cell), 1/dt_n, and the geometry the
// smoother reads (side codes, centre distances, widths, solid flags,
// prolongation stencil); wall states stay in global memory.
__host__ __device__ inline size_t fas_lds_align(size_t b) { return (b + 15) & ~(size_t)15; }

__host__ __device__ inline size_t fas_level_lds_bytes(int nx, int ny) {
    size_t nc = (size_t)nx * ny;
    return 8 * fas_lds_align(4 * nc * 8) + fas_lds_align(nc * 8) + fas_lds_align(4 * nc * 4) +
           fas_lds_align(4 * nc * 8) + fas_lds_align(nx * 8) + fas_lds_align(ny * 8) + fas_lds_align(nc) +
           fas_lds_align(4 * nc * 4) + fas_lds_align(4 * nc * 8);
}

template <typename P>
__device__ __forceinline__ void block_copy(P* dst, const P* __restrict__ src, size_t n) {
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

__global__ void __launch_bounds__(1024) k_fas_cycle_block(FasSet G, Gas gas) {
    extern __shared__ double fsm[];
    __shared__ FasSet F;
    if (threadIdx.x == 0) {
        F = G;
        char* p = (char*)fsm;
        auto take = [&](size_t bytes) {
            char* q = p;
            p += fas_lds_align(bytes);
            return q;
        };
        for (int l = G.l0; l < G.L; ++l) {
            const Geo& g = G.geo[l];
            size_t nc = g.nc;
            F.W[l] = (double*)take(4 * nc * 8);
            F.W2[l] = (double*)take(4 * nc * 8);
            F.W0[l] = (double*)take(4 * nc * 8);
            F.R[l] = (double*)take(4 * nc * 8);
            F.P[l] = (double*)take(4 * nc * 8);
            F.E[l] = (double*)take(4 * nc * 8);
            F.Gam[l] = (double*)take(4 * nc * 8);
            F.Rm[l] = (double*)take(4 * nc * 8);
            F.dtn[l] = (double*)take(nc * 8);
            F.geo[l].nb = (const int*)take(4 * nc * 4);
            F.geo[l].dcent = (const double*)take(4 * nc * 8);
            F.geo[l].dx = (const double*)take(g.nx * 8);
            F.geo[l].dy = (const double*)take(g.ny * 8);
            F.geo[l].solid = (const unsigned char*)take(nc);
            F.geo[l].p_idx = (const int*)take(4 * nc * 4);
            F.geo[l].p_w = (const double*)take(4 * nc * 8);
        }
    }
    __syncthreads();
    for (int l = G.l0; l < G.L; ++l) {
        const Geo& g = G.geo[l];
        size_t nc = g.nc;
        block_copy((int*)F.geo[l].nb, g.nb, 4 * nc);
        block_copy((double*)F.geo[l].dcent, g.dcent, 4 * nc);
        block_copy((double*)F.geo[l].dx, g.dx, (size_t)g.nx);
        block_copy((double*)F.geo[l].dy, g.dy, (size_t)g.ny);
        block_copy((unsigned char*)F.geo[l].solid, g.solid, nc);
        block_copy((int*)F.geo[l].p_idx, g.p_idx, 4 * nc);
        block_copy((double*)F.geo[l].p_w, g.p_w, 4 * nc);
        block_copy(F.dtn[l], G.dtn[l], nc);
        for (size_t i = threadIdx.x; i < 4 * nc; i += blockDim.x) F.E[l][i] = 0.0;
    }
    block_copy(F.W[G.l0], G.W[G.l0], 4 * (size_t)G.geo[G.l0].nc);
    block_copy(F.R[G.l0], G.R[G.l0], 4 * (size_t)G.geo[G.l0].nc);
    __syncthreads();

    const int L = F.L;
    unsigned par = 0;   // bit l: W of level l currently in W2[l]
    for (int l = F.l0; l < L - 1; ++l) {
        const Geo& g = F.geo[l];
        const Geo& gc = F.geo[l + 1];
        fas_block_enter(F, gas, l, par);
        fas_block_smooth(F, gas, l, F.nu1, par);
        const double* W = fas_w(F, par, l);
        for (int t = threadIdx.x; t < 4 * g.nc; t += blockDim.x)
            fas4_rsplit(g, gas, W, F.Gam[l], F.P[l], 1.0, F.Rm[l], (double*)nullptr, t);
        __syncthreads();
        for (int t = threadIdx.x; t < 4 * gc.nc; t += blockDim.x) {
            restrict_comp(g, gc, W, fas_w(F, par, l + 1), t >> 2, t & 3);
            restrict_comp(g, gc, F.Rm[l], F.R[l + 1], t >> 2, t & 3);
        }
        __syncthreads();
    }
    fas_block_enter(F, gas, L - 1, par);
    fas_block_smooth(F, gas, L - 1, F.nuc, par);
    for (int l = L - 2; l >= F.l0; --l) {
        const Geo& g = F.geo[l];
        for (int t = threadIdx.x; t < 4 * g.nc; t += blockDim.x)
            fas4_prolong(g, F.geo[l + 1].nc, fas_w(F, par, l + 1), F.W0[l + 1], fas_w(F, par, l),
                         fas_walt(F, par, l), t);
        __syncthreads();
        par ^= 1u << l;
        fas_block_smooth(F, gas, l, F.nu2, par);
    }
    // result and the state the parent level prolongs from
    block_copy(G.W[G.l0], (const double*)fas_w(F, par, G.l0), 4 * (size_t)G.geo[G.l0].nc);
    block_copy(G.W0[G.l0], (const double*)F.W0[G.l0], 4 * (size_t)G.geo[G.l0].nc);
}

// ---------------------------------------------------------------------------
// small utilities

template <typename T>
__global__ void k_zero(T* __restrict__ a, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = T(0);
}

template <typename T>
__global__ void k_copy_t(const T* __restrict__ a, T* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <typename A, typename B>
__global__ void k_convert(const A* __restrict__ a, B* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = B(a[i]);
}

// 1/dt_n = a^{-n} / dt_p per cell; the factor a^{-n} is read from device
// memory so that a captured graph serves every cycle
__global__ void k_dtn(Geo g, const double* __restrict__ factor, double* __restrict__ out) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    double f = factor[0];
    if (c < g.nc) out[c] = f > 0.0 ? f / g.dt[c] : 0.0;
}

// copy n doubles from up to two sources to two destinations each (b may be
// null); keeps graph captures free of memcpy nodes
__global__ void k_copy2(const double* __restrict__ a, double* __restrict__ a1, double* __restrict__ a2,
                        const double* __restrict__ b, double* __restrict__ b1, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double x = a[i];
        a1[i] = x;
        if (a2) a2[i] = x;
        if (b) b1[i] = b[i];
    }
}

// 1/tau + 1/dt_n of every level in the sweep's type (-1 on solid cells),
// one launch for all levels (threads over the cells of the finest level)
struct CoefSet {
    int L;
    int nc[FAS_MAXL];
    const unsigned char* solid[FAS_MAXL];
    const double *tau[FAS_MAXL], *dtn[FAS_MAXL];
    void* out[FAS_MAXL];
};

template <typename T>
__global__ void k_sweep_coef(CoefSet S) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int l = 0; l < S.L; ++l)
        if (i < S.nc[l]) ((T*)S.out[l])[i] = S.solid[l][i] ? T(-1) : T(S.tau[l][i] + S.dtn[l][i]);
}

}  // namespace miugks
