// Host setup: velocity quadrature, mesh hierarchy, boundary tables and grid
// transfer tables of the multigrid (Sec. II C, Sec. III A, Sec. III B).
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "miugks.h"

namespace miugks {

namespace {

// Orthonormal Hermite polynomials (weight exp(-x^2)) by their three-term
// recurrence; returns p_n(x) and p_{n-1}(x).
void hermite_pair(int n, double x, double& pn, double& pn1) {
    double p0 = std::pow(M_PI, -0.25);
    if (n == 0) {
        pn = p0;
        pn1 = 0.0;
        return;
    }
    double p1 = std::sqrt(2.0) * x * p0;
    for (int j = 1; j < n; ++j) {
        double p2 = std::sqrt(2.0 / (j + 1)) * x * p1 - std::sqrt(double(j) / (j + 1)) * p0;
        p0 = p1;
        p1 = p2;
    }
    pn = p1;
    pn1 = p0;
}

// Gauss-Hermite rule: roots of p_n bracketed by a sign scan of [-B, B]
// (all roots lie inside |x| < sqrt(2n+1)), refined by bisection and Newton;
// weights 2 / p_n'(x)^2 with p_n' = sqrt(2n) p_{n-1} (orthonormal form).
bool gauss_hermite(int n, double* x, double* w) {
    if (n < 1 || n > 400) return false;
    double B = std::sqrt(2.0 * n + 1.0) + 1.0;
    int m = 64 * n + 1;                 // odd: the origin is never a scan point
    double prev_x = -B, pn, pn1;
    hermite_pair(n, prev_x, pn, pn1);
    double prev_v = pn;
    int found = 0;
    for (int i = 1; i <= m && found < n; ++i) {
        double xi = -B + 2.0 * B * i / m, vi;
        hermite_pair(n, xi, vi, pn1);
        if ((prev_v < 0) != (vi < 0)) {
            double a = prev_x, b = xi, fa = prev_v;
            for (int it = 0; it < 200; ++it) {
                double c = 0.5 * (a + b), fc, t;
                hermite_pair(n, c, fc, t);
                if ((fc < 0) == (fa < 0)) {
                    a = c;
                    fa = fc;
                } else {
                    b = c;
                }
            }
            double r = 0.5 * (a + b);
            for (int it = 0; it < 3; ++it) {
                hermite_pair(n, r, pn, pn1);
                if (pn1 != 0.0) r -= pn / (std::sqrt(2.0 * n) * pn1);
            }
            x[found++] = r;
        }
        prev_x = xi;
        prev_v = vi;
    }
    if (found != n) return false;
    for (int i = 0; i < n / 2; ++i) {   // exact symmetry
        double s = 0.5 * (x[n - 1 - i] - x[i]);
        x[i] = -s;
        x[n - 1 - i] = s;
    }
    if (n % 2) x[n / 2] = 0.0;
    for (int i = 0; i < n; ++i) {
        hermite_pair(n, x[i], pn, pn1);
        double d = std::sqrt(2.0 * n) * pn1;
        w[i] = 2.0 / (d * d);
    }
    for (int i = 0; i < n / 2; ++i) {
        double s = 0.5 * (w[i] + w[n - 1 - i]);
        w[i] = w[n - 1 - i] = s;
    }
    for (int i = 0; i < n; ++i) w[i] *= std::exp(x[i] * x[i]);
    return true;
}

}  // namespace

bool quadrature_rule(int kind, int n, double lo, double hi, double* nodes, double* weights) {
    if (!nodes || !weights || n < 2) return false;
    if (kind == MIUGKS_QUAD_GAUSS_HERMITE) return gauss_hermite(n, nodes, weights);
    if (!(hi > lo)) return false;
    double h = (hi - lo) / (n - 1);
    for (int i = 0; i < n; ++i) nodes[i] = lo + h * i;
    nodes[n - 1] = hi;
    if (kind == MIUGKS_QUAD_TRAPEZOID) {
        for (int i = 0; i < n; ++i) weights[i] = h;
        weights[0] = weights[n - 1] = 0.5 * h;
        return true;
    }
    if (kind == MIUGKS_QUAD_SIMPSON38) {
        if ((n - 1) % 3) return false;
        for (int i = 0; i < n; ++i) weights[i] = 0.0;
        const double p[4] = {1.0, 3.0, 3.0, 1.0};
        for (int q = 0; q < (n - 1) / 3; ++q)
            for (int j = 0; j < 4; ++j) weights[3 * q + j] += p[j] * 3.0 * h / 8.0;
        return true;
    }
    return false;
}

namespace {

bool make_level(HostLevel& L, const HostVel& vel, double cfl, std::string& err) {
    int nx = L.nx, ny = L.ny, nc = nx * ny;
    L.nc = nc;
    L.xc.resize(nx);
    L.dx.resize(nx);
    L.yc.resize(ny);
    L.dy.resize(ny);
    for (int i = 0; i < nx; ++i) {
        L.xc[i] = 0.5 * (L.xn[i] + L.xn[i + 1]);
        L.dx[i] = L.xn[i + 1] - L.xn[i];
        if (!(L.dx[i] > 0)) {
            err = "x node lines must increase";
            return false;
        }
    }
    for (int j = 0; j < ny; ++j) {
        L.yc[j] = 0.5 * (L.yn[j] + L.yn[j + 1]);
        L.dy[j] = L.yn[j + 1] - L.yn[j];
        if (!(L.dy[j] > 0)) {
            err = "y node lines must increase";
            return false;
        }
    }
    L.nb.assign(4 * nc, NB_NONE);
    L.dcent.assign(4 * nc, 0.0);
    L.dt.assign(nc, 0.0);
    L.w_cell.clear();
    L.w_side.clear();
    L.w_T.clear();
    L.w_U.clear();
    L.w_V.clear();
    L.w_den.clear();
    L.n_fluid = 0;
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            int c = j * nx + i;
            L.dt[c] = cfl / (vel.umax / L.dx[i] + vel.vmax / L.dy[j]);
            if (L.solid[c]) continue;
            ++L.n_fluid;
            for (int s = 0; s < 4; ++s) {
                uint8_t tag;
                const double* wl;
                int oi = i, oj = j;
                double dface, dcen = 0.0;
                bool inside;
                if (s < 2) {
                    int fi = i + s;
                    tag = L.ftx[j * (nx + 1) + fi];
                    wl = &L.wallx[3 * (j * (nx + 1) + fi)];
                    oi = s == 0 ? i - 1 : i + 1;
                    inside = oi >= 0 && oi < nx;
                    dface = 0.5 * L.dx[i];
                    if (inside) dcen = std::fabs(L.xc[oi] - L.xc[i]);
                } else {
                    int fj = j + (s - 2);
                    tag = L.fty[fj * nx + i];
                    wl = &L.wally[3 * (fj * nx + i)];
                    oj = s == 2 ? j - 1 : j + 1;
                    inside = oj >= 0 && oj < ny;
                    dface = 0.5 * L.dy[j];
                    if (inside) dcen = std::fabs(L.yc[oj] - L.yc[j]);
                }
                int at = s * nc + c;
                if (tag == MIUGKS_FACE_INTERIOR) {
                    if (!inside) {
                        err = "a domain-boundary face is tagged interior";
                        return false;
                    }
                    int o = oj * nx + oi;
                    if (L.solid[o]) {
                        err = "a face between fluid and solid cells must be a wall";
                        return false;
                    }
                    L.nb[at] = o;
                    L.dcent[at] = dcen;
                } else if (tag == MIUGKS_FACE_WALL) {
                    int widx = int(L.w_cell.size());
                    L.nb[at] = NB_WALL0 - widx;
                    L.dcent[at] = 2.0 * dface;
                    L.w_cell.push_back(c);
                    L.w_side.push_back(s);
                    if (!(wl[0] > 0)) {
                        err = "wall temperature must be positive";
                        return false;
                    }
                    L.w_T.push_back(wl[0]);
                    L.w_U.push_back(wl[1]);
                    L.w_V.push_back(wl[2]);
                } else if (tag == MIUGKS_FACE_FARFIELD) {
                    L.nb[at] = NB_FARFIELD;
                    L.dcent[at] = 2.0 * dface;
                } else if (tag == MIUGKS_FACE_SYMMETRY) {
                    L.nb[at] = NB_SYMMETRY;
                    L.dcent[at] = 2.0 * dface;
                } else if (tag == MIUGKS_FACE_OUTFLOW) {
                    L.nb[at] = NB_OUTFLOW;
                    L.dcent[at] = 2.0 * dface;
                } else {
                    err = "unsupported face tag";
                    return false;
                }
            }
        }
    }
    // denominators of the diffuse-wall density: sum over incoming velocities
    for (size_t jw = 0; jw < L.w_cell.size(); ++jw) {
        int s = L.w_side[jw];
        double lam = 1.0 / L.w_T[jw], den = 0.0;
        for (int k = 0; k < vel.nk; ++k) {
            double un = (s < 2 ? vel.u[k] : vel.v[k]) * (s % 2 ? 1.0 : -1.0);
            if (un < 0) {
                double du = vel.u[k] - L.w_U[jw], dv = vel.v[k] - L.w_V[jw];
                den += vel.w[k] * un * (lam / M_PI) * std::exp(-lam * (du * du + dv * dv));
            }
        }
        L.w_den.push_back(den);
    }
    if (L.n_fluid == 0) {
        err = "no fluid cells";
        return false;
    }
    return true;
}

bool coarsen(const HostLevel& F, HostLevel& C, std::string& err) {
    if (F.nx % 2 || F.ny % 2) {
        err = "cannot coarsen an odd number of cells";
        return false;
    }
    int NX = F.nx / 2, NY = F.ny / 2;
    C.nx = NX;
    C.ny = NY;
    C.xn.resize(NX + 1);
    C.yn.resize(NY + 1);
    for (int i = 0; i <= NX; ++i) C.xn[i] = F.xn[2 * i];
    for (int j = 0; j <= NY; ++j) C.yn[j] = F.yn[2 * j];
    C.ftx.assign((NX + 1) * NY, 0);
    C.fty.assign(NX * (NY + 1), 0);
    C.wallx.assign(3 * (NX + 1) * NY, 0.0);
    C.wally.assign(3 * NX * (NY + 1), 0.0);
    for (int J = 0; J < NY; ++J)
        for (int I = 0; I <= NX; ++I) {
            int a = (2 * J) * (F.nx + 1) + 2 * I, b = (2 * J + 1) * (F.nx + 1) + 2 * I;
            if (F.ftx[a] != F.ftx[b]) {
                err = "coarse x-face with mixed tags";
                return false;
            }
            int cf = J * (NX + 1) + I;
            C.ftx[cf] = F.ftx[a];
            double sa = F.dy[2 * J], sb = F.dy[2 * J + 1];
            for (int q = 0; q < 3; ++q)
                C.wallx[3 * cf + q] = (sa * F.wallx[3 * a + q] + sb * F.wallx[3 * b + q]) / (sa + sb);
        }
    for (int J = 0; J <= NY; ++J)
        for (int I = 0; I < NX; ++I) {
            int a = (2 * J) * F.nx + 2 * I, b = (2 * J) * F.nx + 2 * I + 1;
            if (F.fty[a] != F.fty[b]) {
                err = "coarse y-face with mixed tags";
                return false;
            }
            int cf = J * NX + I;
            C.fty[cf] = F.fty[a];
            double sa = F.dx[2 * I], sb = F.dx[2 * I + 1];
            for (int q = 0; q < 3; ++q)
                C.wally[3 * cf + q] = (sa * F.wally[3 * a + q] + sb * F.wally[3 * b + q]) / (sa + sb);
        }
    C.solid.assign(NX * NY, 0);
    for (int J = 0; J < NY; ++J)
        for (int I = 0; I < NX; ++I) {
            int n = 0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) n += F.solid[(2 * J + a) * F.nx + 2 * I + b] ? 1 : 0;
            if (n != 0 && n != 4) {
                err = "coarse cell with mixed solid and fluid children";
                return false;
            }
            C.solid[J * NX + I] = n == 4;
        }
    return true;
}

// Bilinear prolongation weights (Sec. II C 3) on the rectilinear mesh: the
// tensor product of 1-D linear interpolation through the parent centre and a
// partner centre on the side of the fine centre, or extrapolation through
// the opposite partner when the near one lies across a non-interior face.
void prolongation(HostLevel& F, const HostLevel& C) {
    int nc = F.nc, NX = C.nx;
    F.p_idx.assign(4 * nc, 0);
    F.p_w.assign(4 * nc, 0.0);
    for (int c = 0; c < nc; ++c) {
        if (F.solid[c]) continue;
        int ix = c % F.nx, iy = c / F.nx, I = ix / 2, J = iy / 2, A = J * NX + I;
        double x = F.xc[ix], y = F.yc[iy];
        int sx = x > C.xc[I] ? 1 : -1, sy = y > C.yc[J] ? 1 : -1;
        int cx[2], cy[2], ncx = 0, ncy = 0;
        for (int t = 0; t < 2; ++t) {
            int d = t == 0 ? sx : -sx;
            if (C.nb[(d > 0 ? 1 : 0) * C.nc + A] >= 0) cx[ncx++] = I + d;
            d = t == 0 ? sy : -sy;
            if (C.nb[(d > 0 ? 3 : 2) * C.nc + A] >= 0) cy[ncy++] = J + d;
        }
        int px = -1, py = -1;
        bool found = false;
        for (int b = 0; b < ncy && !found; ++b)
            for (int a = 0; a < ncx && !found; ++a)
                if (!C.solid[cy[b] * NX + cx[a]]) {
                    px = cx[a];
                    py = cy[b];
                    found = true;
                }
        if (!found) {
            if (ncx) {
                px = cx[0];
                py = -1;
            } else if (ncy) {
                px = -1;
                py = cy[0];
            }
        }
        double wxa = 1.0, wxb = 0.0, wya = 1.0, wyb = 0.0;
        int IB = I, JD = J;
        if (px >= 0) {
            double Xa = C.xc[I], Xb = C.xc[px];
            wxa = (Xb - x) / (Xb - Xa);
            wxb = (x - Xa) / (Xb - Xa);
            IB = px;
        }
        if (py >= 0) {
            double Ya = C.yc[J], Yb = C.yc[py];
            wya = (Yb - y) / (Yb - Ya);
            wyb = (y - Ya) / (Yb - Ya);
            JD = py;
        }
        F.p_idx[0 * nc + c] = A;
        F.p_idx[1 * nc + c] = J * NX + IB;
        F.p_idx[2 * nc + c] = JD * NX + IB;
        F.p_idx[3 * nc + c] = JD * NX + I;
        F.p_w[0 * nc + c] = wxa * wya;
        F.p_w[1 * nc + c] = wxb * wya;
        F.p_w[2 * nc + c] = wxb * wyb;
        F.p_w[3 * nc + c] = wxa * wyb;
    }
}

}  // namespace

bool build_levels(int nx, int ny, int n_levels, const double* x, const double* y,
                  const uint8_t* ftx, const uint8_t* fty, const double* wallx,
                  const double* wally, const uint8_t* solid, const HostVel& vel, double cfl,
                  std::vector<HostLevel>& out, std::string& err) {
    if (nx < 1 || ny < 1 || n_levels < 1 || !x || !y || !ftx || !fty) {
        err = "bad mesh description";
        return false;
    }
    if ((nx % (1 << (n_levels - 1))) || (ny % (1 << (n_levels - 1)))) {
        err = "nx and ny must be divisible by 2^(n_levels-1)";
        return false;
    }
    out.assign(n_levels, HostLevel());
    HostLevel& L0 = out[0];
    L0.nx = nx;
    L0.ny = ny;
    L0.xn.assign(x, x + nx + 1);
    L0.yn.assign(y, y + ny + 1);
    L0.ftx.assign(ftx, ftx + (nx + 1) * ny);
    L0.fty.assign(fty, fty + nx * (ny + 1));
    L0.wallx.assign(3 * (nx + 1) * ny, 0.0);
    L0.wally.assign(3 * nx * (ny + 1), 0.0);
    if (wallx) L0.wallx.assign(wallx, wallx + 3 * (nx + 1) * ny);
    if (wally) L0.wally.assign(wally, wally + 3 * nx * (ny + 1));
    L0.solid.assign(nx * ny, 0);
    if (solid)
        for (int c = 0; c < nx * ny; ++c) L0.solid[c] = solid[c] ? 1 : 0;
    if (!make_level(L0, vel, cfl, err)) return false;
    for (int l = 1; l < n_levels; ++l) {
        if (!coarsen(out[l - 1], out[l], err)) return false;
        if (!make_level(out[l], vel, cfl, err)) return false;
        prolongation(out[l - 1], out[l]);
    }
    return true;
}

}  // namespace miugks
