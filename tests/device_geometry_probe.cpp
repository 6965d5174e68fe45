// Test helper: the device geometry of libpsc (psc_core.h: stencils, walls,
// colours, hop vectors, brick layout) and its Philox generator, compiled for the host so that the CPU
// tests can compare it with the oracle voxel by voxel.  Not part of the
// library.
#include "psc_core.h"

using namespace psc;

static Geo make_geo(uint32_t ni, uint32_t nj, uint32_t nk, int lattice, int walls, int brick) {
  Geo g{};
  g.ni = ni;
  g.nj = nj;
  g.nk = nk;
  g.dni = make_div(ni);
  g.dnj = make_div(nj);
  g.brick = brick ? 1u : 0u;
  g.walls = walls ? 1u : 0u;
  g.fcc = lattice ? 1u : 0u;
  g.nbi = ni / 4;
  g.nbj = nj / 4;
  g.dnbi = make_div(ni / 4);
  g.dnbj = make_div(nj / 4);
  return g;
}

extern "C" {

// neighbour n of every voxel (linear indices, 0xFFFFFFFF beyond a wall),
// computed through the layout the kernels use: out[12 v + n]
void probe_neighbours(uint32_t ni, uint32_t nj, uint32_t nk, int lattice, int walls, int brick,
                      uint32_t *out) {
  const Geo g = make_geo(ni, nj, nk, lattice, walls, brick);
  const uint64_t nv = (uint64_t)ni * nj * nk;
  for (uint64_t v = 0; v < nv; ++v) {
    const Coord c = coord_of(g, to_layout(g, (uint32_t)v));
    for (uint32_t n = 0; n < 12; ++n) {
      Coord t;
      const bool open = step_target(g, c, n, t);
      out[12 * v + n] = open ? to_linear(g, index_of(g, t)) : 0xFFFFFFFFu;
    }
  }
}

// stage colour of every voxel
void probe_colours(uint32_t ni, uint32_t nj, uint32_t nk, int lattice, uint32_t *out) {
  const Geo g = make_geo(ni, nj, nk, lattice, 0, 1);
  const uint64_t nv = (uint64_t)ni * nj * nk;
  for (uint64_t v = 0; v < nv; ++v) out[v] = colour_of(g, coord_of(g, to_layout(g, (uint32_t)v)));
}

// hop vector (X, Y, Z) of row n from a voxel in layer k
void probe_hop(uint32_t n, int32_t k, int lattice, int32_t *out) {
  if (lattice) hop_vector_t<1>(n, k & 1, out[0], out[1], out[2]);
  else hop_vector_t<0>(n, k & 1, out[0], out[1], out[2]);
}

// the kernels' Philox4x32-10: out = philox(counter c, key k)
void probe_philox(const uint32_t *c, const uint32_t *k, uint32_t *out) {
  const U4 r = philox(c[0], c[1], c[2], c[3], k[0], k[1]);
  out[0] = r.x;
  out[1] = r.y;
  out[2] = r.z;
  out[3] = r.w;
}

int probe_n_colours(int lattice) {
  const Geo g = make_geo(4, 4, 12, lattice, 0, 1);
  return (int)n_colours(g);
}
}
