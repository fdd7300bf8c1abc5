// geometry.cpp -- host preprocessing of a solid mask: node classes and the
// compact list of wall nodes.
//
// A wall node is a solid node that the force stencil of Eq. 5 reaches from
// a fluid node, i.e. a solid node with at least one fluid neighbour along a
// non-rest lattice velocity; these are the solid points next to the curved
// boundary that carry a virtual density (Sec. III B).  No other solid node is
// ever read by the step.
#include <cmath>

#include "lbm_host.hpp"

namespace lbm {

namespace {
const int E9[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                      {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
const int E19[19][3] = {{0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                        {0, 0, 1},   {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                        {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                        {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
inline int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}
}  // namespace

int build_geometry(const lbm_params& p, const uint8_t* solid, Geometry& g) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t N = (int64_t)nx * ny * nz;
    const int Q = p.lattice;
    const int(*E)[3] = (Q == 9) ? E9 : E19;
    g.cls.assign(N, CLS_FLUID);
    g.widx.assign(N, -1);
    g.walls.clear();
    g.n_fluid = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
                if (!solid[n]) {
                    ++g.n_fluid;
                    continue;
                }
                bool wall = false;
                for (int a = 1; a < Q && !wall; ++a) {
                    const int64_t m = wrap(x + E[a][0], nx) +
                                      (int64_t)nx * (wrap(y + E[a][1], ny) +
                                                     (int64_t)ny * wrap(z + E[a][2], nz));
                    wall = !solid[m];
                }
                if (wall) {
                    g.cls[n] = CLS_WALL;
                    g.widx[n] = (int32_t)g.walls.size();
                    g.walls.push_back(n);
                } else {
                    g.cls[n] = CLS_SOLID;
                }
            }
    return LBM_OK;
}

// Geometric-formulation stencils.  Per wall node P: the solid normal n_s of
// Eq. 13 with the 8th-order isotropic weights of Eq. 14 over the 24 offsets
// with |e|^2 = 1, 2, 4, 5, 8; the two characteristic directions of Eq. 15;
// along each, the first mesh line crossed (x_P +- 1 or y_P +- 1, whichever
// comes first; ties go to the vertical line) and the two lattice nodes that
// bracket the crossing on that line.  Arithmetic in double, in the order
// written here; the step kernel then interpolates the densities.
void build_gf_stencils(const lbm_params& p, const Geometry& g, const double* theta_deg,
                       std::vector<int32_t>& code, std::vector<double>& t) {
    static const int off[24][2] = {
        {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1},
        {2, 0}, {-2, 0}, {0, 2}, {0, -2}, {2, 1}, {1, 2}, {-1, 2}, {-2, 1},
        {-2, -1}, {-1, -2}, {1, -2}, {2, -1}, {2, 2}, {-2, 2}, {-2, -2}, {2, -2}};
    const int nx = p.nx, ny = p.ny;
    const size_t nw = g.walls.size();
    code.assign(nw, 0);
    t.assign(2 * nw, 0.0);
    auto solid_at = [&](int x, int y) {
        return g.cls[(int64_t)wrap(y, ny) * nx + wrap(x, nx)] != CLS_FLUID;
    };
    const double pi = 3.14159265358979323846;
    for (size_t w = 0; w < nw; ++w) {
        const int x = (int)(g.walls[w] % nx), y = (int)(g.walls[w] / nx);
        double sx = 0.0, sy = 0.0;
        for (int i = 0; i < 24; ++i) {
            const int e2 = off[i][0] * off[i][0] + off[i][1] * off[i][1];
            const double om = e2 == 1 ? 4.0 / 21.0 : e2 == 2 ? 4.0 / 45.0 : e2 == 4 ? 1.0 / 60.0
                            : e2 == 5 ? 2.0 / 315.0 : 1.0 / 5040.0;
            if (solid_at(x + off[i][0], y + off[i][1])) {
                sx += om * off[i][0];
                sy += om * off[i][1];
            }
        }
        const double norm = std::sqrt(sx * sx + sy * sy);
        int32_t c = theta_deg[w] > 90.0 ? (1 << 20) : 0;
        if (norm == 0.0) {  // no direction: both points void (neighbour mean)
            code[w] = c;
            continue;
        }
        const double nxs = -sx / norm, nys = -sy / norm;
        const double th = theta_deg[w] * (pi / 180.0), tp = 0.5 * pi - th;
        const double cs = std::cos(tp), sn = std::sin(tp);
        const double v[2][2] = {{nxs * cs - nys * sn, nxs * sn + nys * cs},
                                {nxs * cs + nys * sn, -nxs * sn + nys * cs}};
        for (int k = 0; k < 2; ++k) {
            const double vx = v[k][0], vy = v[k][1];
            const double tx = std::fabs(vx) > 1e-12 ? 1.0 / std::fabs(vx) : 1e300;
            const double ty = std::fabs(vy) > 1e-12 ? 1.0 / std::fabs(vy) : 1e300;
            int ax, ay, bx, by;
            double tt;
            if (tx <= ty) {
                const int sgn = vx > 0 ? 1 : -1;
                const double yc = tx * vy;
                const int y0 = (int)std::floor(yc);
                tt = yc - y0;
                ax = sgn; ay = y0; bx = sgn; by = y0 + 1;
            } else {
                const int sgn = vy > 0 ? 1 : -1;
                const double xc = ty * vx;
                const int x0 = (int)std::floor(xc);
                tt = xc - x0;
                ax = x0; ay = sgn; bx = x0 + 1; by = sgn;
            }
            // a crossing within 1e-12 of a lattice node is that node alone
            // (whatever the rounding of the crossing); b can fall outside the
            // 3x3 block only when the crossing is node a
            const bool at_a = tt < 1e-12, at_b = tt > 1.0 - 1e-12;
            const bool fa = !at_b && ax >= -1 && ax <= 1 && ay >= -1 && ay <= 1 &&
                            !solid_at(x + ax, y + ay);
            const bool fb = !at_a && bx >= -1 && bx <= 1 && by >= -1 && by <= 1 &&
                            !solid_at(x + bx, y + by);
            const int ia = (fa ? (ax + 1) + 3 * (ay + 1) : 0), ib = (fb ? (bx + 1) + 3 * (by + 1) : 0);
            c |= (ia | (ib << 4) | ((int)fa << 8) | ((int)fb << 9)) << (10 * k);
            t[2 * w + k] = tt;
        }
        code[w] = c;
    }
}

}  // namespace lbm
