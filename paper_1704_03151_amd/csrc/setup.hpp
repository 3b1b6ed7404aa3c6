// Host-side description of the mesh hierarchy and velocity grid of one
// MIUGKS problem (Sec. III A mesh coarsening, Sec. III B boundary tags).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace miugks {

// Encoding of what lies across one side of a cell (side 0: -x, 1: +x,
// 2: -y, 3: +y).  Non-negative: index of the neighbouring fluid cell.
constexpr int NB_FARFIELD = -1;
constexpr int NB_OUTFLOW = -2;
constexpr int NB_NONE = -3;       // side of a solid cell
constexpr int NB_SYMMETRY = -4;   // symmetry face (specular reflection)
constexpr int NB_WALL0 = -16;     // wall side j is encoded as NB_WALL0 - j

inline bool nb_is_wall(int code) { return code <= NB_WALL0; }
inline int nb_wall_index(int code) { return NB_WALL0 - code; }

struct HostLevel {
    int nx = 0, ny = 0, nc = 0, n_fluid = 0;
    std::vector<double> xn, yn, xc, yc, dx, dy;
    std::vector<uint8_t> ftx, fty, solid;       // (ny)(nx+1), (ny+1)(nx), (ny)(nx)
    std::vector<double> wallx, wally;           // 3 doubles per face: T, U, V
    std::vector<int> nb;                        // [4][nc]
    std::vector<double> dcent;                  // [4][nc] centre distance across the side
    std::vector<double> dt;                     // [nc] CFL physical step
    // wall sides of fluid cells
    std::vector<int> w_cell, w_side;
    std::vector<double> w_T, w_U, w_V, w_den;   // den = sum_{u_n<0} w u_n C_k^G
    // prolongation from the next coarser level into this level: [4][nc]
    std::vector<int> p_idx;
    std::vector<double> p_w;
};

struct HostVel {
    int nu = 0, nv = 0, nk = 0;
    std::vector<double> u, v, w;   // [nk], k = ku * nv + kv
    std::vector<int> mx, my;       // [nk] the velocity with u (mx) or v (my) reversed, -1 if the grid lacks it
    double umax = 0, vmax = 0;
};

// 1-D rules; return false on bad arguments.
bool quadrature_rule(int kind, int n, double lo, double hi, double* nodes, double* weights);

// Build all levels; on failure returns false and sets err.
bool build_levels(int nx, int ny, int n_levels, const double* x, const double* y,
                  const uint8_t* ftx, const uint8_t* fty, const double* wallx,
                  const double* wally, const uint8_t* solid, const HostVel& vel, double cfl,
                  std::vector<HostLevel>& out, std::string& err);

}  // namespace miugks
