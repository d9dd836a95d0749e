// Host-only check of the tile kernels' global and LDS indexing: for every
// workgroup and thread of a launch, the slots a thread loads, the cells it
// reads or writes and the neighbour records the adjoint gathers must lie
// inside their buffers.  Runs the same __host__ __device__ index functions the
// kernels use; no device code is executed.
#include <cstdio>
#include <cstdlib>

#include "../../paper_2309_12019_amd/csrc/dg_launch.hpp"

using namespace dgk;

static int failures = 0;
#define CHECK(c, ...)                  \
  do {                                 \
    if (!(c)) {                        \
      if (failures < 20) {             \
        std::printf(__VA_ARGS__);      \
        std::printf("\n");            \
      }                                \
      ++failures;                      \
    }                                  \
  } while (0)

template <int DIM, int TX, int TY>
void check(int nx, int ny, int per_x, int per_y) {
  using G = TileGeom<DIM, TX, TY>;
  StageArgs A{};
  A.nx = nx;
  A.ny = DIM == 2 ? ny : 1;
  A.per_x = per_x;
  A.per_y = DIM == 2 ? per_y : 0;
  const size_t ncells = (size_t)A.nx * A.ny;
  const int gx_blocks = (nx + TX - 1) / TX, gy_blocks = DIM == 2 ? (ny + TY - 1) / TY : 1;
  for (int by = 0; by < gy_blocks; ++by)
    for (int bx = 0; bx < gx_blocks; ++bx)
      for (int t = 0; t < G::NT; ++t) {
        const int ix0 = bx * TX, iy0 = DIM == 2 ? by * TY : 0;
        int sc, gx, gy, hs, hgx, hgy;
        const bool halo = tile_slots<DIM, TX, TY>(t, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
        CHECK(sc >= 0 && sc < G::NS, "dim %d tile %dx%d: own slot %d out of [0,%d)", DIM, TX, TY, sc, G::NS);
        size_t cell;
        if (slot_cell<DIM>(A, gx, gy, cell))
          CHECK(cell < ncells, "dim %d %dx%d per %d%d: own load cell %zu >= %zu (t %d block %d,%d)", DIM, nx, ny,
                per_x, per_y, cell, ncells, t, bx, by);
        if (halo) {
          CHECK(hs >= 0 && hs < G::NS, "dim %d: halo slot %d out of range", DIM, hs);
          if (slot_cell<DIM>(A, hgx, hgy, cell))
            CHECK(cell < ncells, "dim %d %dx%d per %d%d: halo load cell %zu >= %zu (t %d block %d,%d)", DIM, nx,
                  ny, per_x, per_y, cell, ncells, t, bx, by);
        }
        // the face-neighbour slots a cell reads stay inside the tile
        const int W = G::W;
        const int offs[4] = {-1, 1, -W, W};
        for (int f = 0; f < 2 * DIM; ++f)
          CHECK(sc + offs[f] >= 0 && sc + offs[f] < G::NS, "neighbour slot out of range");
        // active cells: own output and the adjoint's neighbour records
        const bool active = gx < nx && gy < (DIM == 2 ? ny : 1);
        if (active) {
          CHECK((size_t)gy * nx + gx < ncells, "output cell out of range");
          for (int f = 0; f < 2 * DIM; ++f) {
            const bool has = f < 2 ? (per_x || (f == 0 ? gx > 0 : gx < nx - 1))
                                   : (per_y || (f == 2 ? gy > 0 : gy < ny - 1));
            if (has)
              CHECK(neighbour_cell(gx, gy, f, nx, DIM == 2 ? ny : 1) < ncells, "neighbour record out of range");
          }
        }
      }
}

template <int DIM, int TX, int TY>
void sweep() {
  const int sizes[] = {1, 2, 3, 7, 8, 9, 15, 16, 17, 31, 63, 64, 65, 100, 255, 256, 257, 300, 513};
  for (int nx : sizes)
    for (int ny : (DIM == 2 ? sizes : sizes))
      for (int px = 0; px < 2; ++px)
        for (int py = 0; py < (DIM == 2 ? 2 : 1); ++py) {
          check<DIM, TX, TY>(nx, ny, px, py);
          if (DIM == 1) break;
        }
}

int main() {
  sweep<1, 256, 1>();
  sweep<1, 64, 1>();
  sweep<2, 16, 16>();
  sweep<2, 8, 8>();
  std::printf("%s (%d failures)\n", failures ? "FAIL" : "ok", failures);
  return failures ? 1 : 0;
}
