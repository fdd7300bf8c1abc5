// geometry.cpp -- host preprocessing of a solid mask: node classes and the
// compact list of wall nodes.
//
// A wall node is a solid node that the force stencil of Eq. 5 reaches from
// a fluid node, i.e. a solid node with at least one fluid neighbour along a
// non-rest lattice velocity; these are the solid points next to the curved
// boundary that carry a virtual density (Sec. III B).  No other solid node is
// ever read by the step.
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

}  // namespace lbm
