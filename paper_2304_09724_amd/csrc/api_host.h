// api_host.h -- host-side helpers shared by the C ABI's translation units:
// argument checks, sizes, the device workspace layout and the kernels' view
// of the scheme parameters.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>

#include "../../include/shweno.h"
#include "shw_kernels.h"

namespace shw {
namespace host {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline int ncomp(int eq, int dim) { return eq == SHW_EULER ? (dim == 1 ? 3 : 4) : 1; }

inline bool valid_params(const shw_params *p)
{
    if (!p) return false;
    if (p->eq < SHW_ADVECTION || p->eq > SHW_EULER) return false;
    if (p->weights < SHW_W_NONLINEAR || p->weights > SHW_W_LEARNED) return false;
    if (p->weights == SHW_W_LEARNED &&
        (!(p->gate_threshold > 0.0 && p->gate_threshold < 1.0) || p->gate_every < 1 ||
         p->gate_every > 1024))
        return false;
    if (p->eq == SHW_EULER && !(p->gamma > 1.0)) return false;
    if (!(p->cfl > 0.0) || !(p->eps > 0.0)) return false;
    for (int k = 0; k < 3; ++k)
        if (!(p->lin_w[k] > 0.0)) return false;
    if (std::fabs(p->lin_w[0] + p->lin_w[1] + p->lin_w[2] - 1.0) > 1e-12) return false;
    if (p->positivity != 0 && p->positivity != 1) return false;
    return true;
}

inline bool valid_mesh(const shw_mesh *m)
{
    if (!m) return false;
    if (m->dim != 1 && m->dim != 2) return false;
    if (m->nx < 3 || !(m->x1 > m->x0)) return false;
    if (m->dim == 1 && m->ny != 1) return false;
    if (m->dim == 2 && (m->ny < 3 || !(m->y1 > m->y0))) return false;
    for (int k = 0; k < (m->dim == 1 ? 2 : 4); ++k)
        if (m->bc[k] < SHW_BC_PERIODIC || m->bc[k] > SHW_BC_REFLECTIVE) return false;
    if ((m->bc[0] == SHW_BC_PERIODIC) != (m->bc[1] == SHW_BC_PERIODIC)) return false;
    if (m->dim == 2 && (m->bc[2] == SHW_BC_PERIODIC) != (m->bc[3] == SHW_BC_PERIODIC))
        return false;
    return true;
}

inline size_t state_doubles(const shw_mesh *m, int eq)
{
    return (size_t)(m->dim == 1 ? 2 : 4) * ncomp(eq, m->dim) * (size_t)m->nx * m->ny;
}

// Tile variants the autotuner chooses between: 1D, 128 / 256 / 512 threads
// (2, 4, 8 waves) per instance; 2D, 1 / 2 / 4 lines of 60 cells per tile.
constexpr int N_TILE_VARIANTS = 3;
constexpr int lines2d(int v) { return 1 << v; }

// Device workspace carved out of the caller's buffer.
struct Layout {
    size_t alt = 0, inst = 0, order = 0, queue = 0, ist = 0, t_end = 0, dt = 0,
           flags = 0, tiles0 = 0, tiles1 = 0, act_inst = 0, act_off0 = 0, act_off1 = 0,
           act_n = 0, parity = 0, last = 0, dt_fixed = 0,
           steps_left = 0, smax = 0, bad = 0, active = 0, gate = 0, faces = 0, trouble = 0,
           guard = 0, total = 0;
};

inline Layout make_layout(const shw_mesh *meshes, int n_inst, const shw_params *p)
{
    Layout L;
    size_t state = 0, cells = 0;
    for (int i = 0; i < n_inst; ++i) {
        state += state_doubles(&meshes[i], p->eq);
        cells += (size_t)meshes[i].nx * meshes[i].ny;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes, 256); return at; };
    L.alt = take(state * sizeof(double));
    L.inst = take((size_t)n_inst * std::max(sizeof(Inst1D), sizeof(Inst2D)));
    L.order = take((size_t)n_inst * sizeof(int));
    L.queue = take(256);
    L.ist = take((size_t)n_inst * sizeof(InstState));
    L.t_end = take((size_t)n_inst * sizeof(double));
    L.dt = take((size_t)n_inst * sizeof(double));
    L.flags = take(cells);
    L.tiles0 = take((size_t)N_TILE_VARIANTS * (n_inst + 1) * sizeof(int));
    L.tiles1 = take((size_t)N_TILE_VARIANTS * (n_inst + 1) * sizeof(int));
    L.act_inst = take((size_t)n_inst * sizeof(int));
    L.act_off0 = take((size_t)(n_inst + 1) * sizeof(int));
    L.act_off1 = take((size_t)(n_inst + 1) * sizeof(int));
    L.act_n = take(256);
    L.parity = take((size_t)n_inst * sizeof(int));
    L.last = take((size_t)n_inst * sizeof(int));
    L.dt_fixed = take((size_t)n_inst * sizeof(double));
    L.steps_left = take((size_t)n_inst * sizeof(long long));
    L.smax = take((size_t)n_inst * sizeof(double));
    L.bad = take((size_t)n_inst * sizeof(int));
    L.active = take(256);
    L.gate = take(64 * sizeof(GateLane));
    // positivity safeguard (Euler): each face's flux and value(s) at t_{n+1}
    // (1D: planes [6][n+1] per instance; 2D: [20][ny][nx+1] for the x-faces and
    // [20][ny+1][nx] for the y-faces), a byte per cell, an int per instance
    size_t face_doubles = 0;
    for (int i = 0; i < n_inst; ++i) {
        const shw_mesh &m = meshes[i];
        face_doubles += m.dim == 1 ? 6 * ((size_t)m.nx + 1)
                                   : 20 * ((size_t)m.ny * (m.nx + 1) + (size_t)(m.ny + 1) * m.nx);
    }
    L.faces = take(p->positivity ? face_doubles * sizeof(double) : 0);
    L.trouble = take(p->positivity ? cells : 0);
    L.guard = take(p->positivity ? (size_t)n_inst * sizeof(int) : 0);
    L.total = off;
    return L;
}

// a batch: valid meshes of one dimension, and an equation / weight mode the
// library runs in that dimension (Burgers 1D only, the learned gate Euler only)
inline bool valid_batch(const shw_mesh *meshes, int n_inst, const shw_params *params)
{
    if (!meshes || n_inst < 1 || !valid_params(params)) return false;
    for (int i = 0; i < n_inst; ++i)
        if (!valid_mesh(&meshes[i]) || meshes[i].dim != meshes[0].dim) return false;
    if (params->eq == SHW_BURGERS && meshes[0].dim != 1) return false;
    if (params->weights == SHW_W_LEARNED && params->eq != SHW_EULER) return false;
    if (params->positivity && params->eq != SHW_EULER) return false;
    return true;
}

// The kernels' view of the scheme parameters.
inline DevParams make_devparams(const shw_params *p)
{
    DevParams dp{};
    dp.gamma = p->gamma;
    dp.adv_a = p->adv_a;
    dp.adv_b = p->adv_b;
    dp.cfl = p->cfl;
    dp.eps = p->eps;
    dp.g1 = p->lin_w[0];
    dp.g2 = p->lin_w[1];
    dp.g3 = p->lin_w[2];
    dp.inv_g1 = 1.0 / p->lin_w[0];
    dp.charwise = p->charwise;
    dp.weights = p->weights;
    return dp;
}

} // namespace host
} // namespace shw
