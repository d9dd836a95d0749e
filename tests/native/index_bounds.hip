// Host-only check of the tile kernels' global and LDS indexing: for every
// workgroup and thread of a launch, the slots a thread loads, the cells it
// reads or writes and the neighbour records the adjoint gathers must lie
// inside their buffers.  Runs the same __host__ __device__ index functions the
// kernels use; no device code is executed.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2309_12019_amd/csrc/dg_batch_plan.hpp"
#include "../../paper_2309_12019_amd/csrc/dg_euler.hpp"
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

// The shared faces of a 2D tile (shares_faces): for every rotation of the
// leftover waves each face is evaluated by exactly one thread of the face
// phase; the slots below and above each face lie inside the tile and are no
// corner slots (those hold no loaded state); the face's lower cell and its
// slot agree; the face moments stay inside the LDS the launch allocates; and
// each tile cell's four faces are the faces whose upper (-x, -y) or lower
// (+x, +y) slot is the cell's own slot.
template <int TX, int TY>
void check_faces(int nl, int flux) {
  using G = TileGeom<2, TX, TY>;
  using FG = FaceGeom<TX, TY>;
  constexpr int NT = TX * TY, NW = NT / 64;
  int n = 1;
  while (n * n < nl) ++n;
  if (!shares_faces(2, n - 1, flux, TX, TY)) return;
  const long long lds = stage_lds_doubles(2, nl, flux, TX, TY);
  CHECK(lds == tile_lds_doubles(2, nl, TX, TY) + (long long)n * (FG::XS + FG::YS), "faces: LDS size");
  auto corner = [&](int s) {
    const int x = s % G::W, y = s / G::W;
    return (x == 0 || x == G::W - 1) && (y == 0 || y == G::H - 1);
  };
  for (int rot = 0; rot < NW; ++rot) {
    std::vector<int> cx(FG::NXF, 0), cy(FG::NYF, 0);
    for (int t = 0; t < NT; ++t)
      for (int k = 0; k < 4; ++k) {
        int e;
        if (!face_task<TX, TY>(t, rot, k, e)) continue;
        if (k & 1) {
          CHECK(e >= 0 && e < FG::NYF, "faces: y face %d out of range", e);
          if (e >= 0 && e < FG::NYF) cy[e]++;
        } else {
          CHECK(e >= 0 && e < FG::NXF, "faces: x face %d out of range", e);
          if (e >= 0 && e < FG::NXF) cx[e]++;
        }
      }
    for (int e = 0; e < FG::NXF; ++e) CHECK(cx[e] == 1, "faces: x face %d evaluated %d times (rot %d)", e, cx[e], rot);
    for (int e = 0; e < FG::NYF; ++e) CHECK(cy[e] == 1, "faces: y face %d evaluated %d times (rot %d)", e, cy[e], rot);
    // the leftover rounds: whole waves (one wave each), never wave-divergent
    for (int k = 2; k < 4; ++k)
      for (int w = 0; w < NW; ++w) {
        int any = 0, e;
        for (int l = 0; l < 64; ++l) any += (face_task<TX, TY>(w * 64 + l, rot, k, e) ? 1 : 0);
        CHECK(any == 0 || w == (k == 2 ? rot : (rot + NW / 2) % NW), "faces: round %d on wave %d", k, w);
      }
  }
  const int ix0 = 3 * TX, iy0 = 5 * TY;
  for (int axis = 0; axis < 2; ++axis)
    for (int e = 0; e < (axis ? FG::NYF : FG::NXF); ++e) {
      int gx, gy;
      const int lo = face_slot<TX, TY>(axis, e, ix0, iy0, gx, gy);
      const int hi = lo + (axis ? G::W : 1);
      CHECK(lo >= 0 && hi < G::NS && !corner(lo) && !corner(hi), "faces: axis %d face %d slots %d %d", axis, e, lo, hi);
      CHECK(gx == ix0 - 1 + lo % G::W && gy == iy0 - 1 + lo / G::W, "faces: lower cell of face %d", e);
      const long long base = (long long)nl * G::S + (axis ? (long long)n * FG::XS : 0);
      const int st = axis ? FG::YS : FG::XS;
      CHECK(base + (long long)(n - 1) * st + e < lds, "faces: moments of face %d outside LDS", e);
    }
  for (int t = 0; t < NT; ++t) {
    int sc, gx, gy, hs, hgx, hgy;
    tile_slots<2, TX, TY>(t, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
    const int lx = t % TX, ly = t / TX, ex = ly * (TX + 1) + lx, ey = ly * TX + lx;
    int fx, fy, s;
    s = face_slot<TX, TY>(0, ex, ix0, iy0, fx, fy);
    CHECK(s + 1 == sc, "faces: -x face of cell %d", t);
    s = face_slot<TX, TY>(0, ex + 1, ix0, iy0, fx, fy);
    CHECK(s == sc && fx == gx && fy == gy, "faces: +x face of cell %d", t);
    s = face_slot<TX, TY>(1, ey, ix0, iy0, fx, fy);
    CHECK(s + G::W == sc, "faces: -y face of cell %d", t);
    s = face_slot<TX, TY>(1, ey + TX, ix0, iy0, fx, fy);
    CHECK(s == sc && fx == gx && fy == gy, "faces: +y face of cell %d", t);
  }
}

// The fused step kernel: tile A loads U^n on the tile and three rings (each
// slot from the cell it stands for, wrapped or exterior); every stage's
// output slot maps to the same mesh cell in its input tile and in tile A, its
// face neighbours lie inside the input tile, and the last stage writes each
// mesh cell of the tile exactly once.
template <int DIM, int TX, int TY, int KO>
void check_step_stage(const StageArgs& A, int ix0, int iy0, size_t ncells, int nl, int* written) {
  using G = StepGeom<DIM, TX, TY>;
  using TO = typename G::template T<KO>;
  using TI = typename G::template T<KO + 1>;
  for (int o = 0; o < TO::N; ++o) {
    int islot, aslot, gx, gy, wx, wy;
    step_slot<DIM, TX, TY, KO>(o, ix0, iy0, islot, aslot, gx, gy);
    CHECK(islot >= 0 && islot < TI::N && aslot >= 0 && aslot < G::A::N, "step stage %d: slot out of range", KO);
    // same mesh cell in the input tile and in tile A
    const int ix_in = ix0 - (KO + 1) + islot % TI::W, iy_in = DIM == 2 ? iy0 - (KO + 1) + islot / TI::W : 0;
    const int ix_a = ix0 - 3 + aslot % G::A::W, iy_a = DIM == 2 ? iy0 - 3 + aslot / G::A::W : 0;
    CHECK(ix_in == gx && iy_in == gy && ix_a == gx && iy_a == gy, "step stage %d: slot maps to another cell", KO);
    const int offs[4] = {-1, 1, -TI::W, TI::W};
    for (int f = 0; f < 2 * DIM; ++f) {
      const int nb = islot + offs[f];
      CHECK(nb >= 0 && nb < TI::N, "step stage %d: neighbour slot out of the input tile", KO);
      const int nx_ = nb % TI::W;
      CHECK(DIM == 2 || (nx_ == islot % TI::W + (f ? 1 : -1)), "1D neighbour wraps a row");
      if (DIM == 2 && f < 2) CHECK(nb / TI::W == islot / TI::W, "x neighbour in another row");
    }
    if (KO == 0 && (gx >= A.nx || gy >= (DIM == 2 ? A.ny : 1))) continue;
    if (step_cell<DIM>(A, gx, gy, wx, wy)) {
      CHECK(wx >= 0 && wx < A.nx && wy >= 0 && wy < (DIM == 2 ? A.ny : 1), "step: wrapped cell out of range");
      if (KO == 0) {
        const size_t cell = (size_t)wy * A.nx + wx;
        CHECK(cell < ncells && (cell + 1) * nl <= ncells * nl, "step: output out of range");
        if (cell < ncells) written[cell]++;
      }
    } else {
      CHECK(KO > 0, "step: a tile cell inside the mesh classified as exterior");
    }
  }
}

// The split stages of the fused step: every output cell is evaluated whole
// by exactly one thread, or has exactly one gamma thread and one thread for
// the rest; each wave holds one role; the gamma slots stay inside the
// exchange buffer (nt / 2 doubles).
template <int DIM, int TX, int TY, int KO>
void check_split() {
  using G = StepGeom<DIM, TX, TY>;
  using TO = typename G::template T<KO>;
  constexpr int n = TO::N, nt = G::NT, f = split_full(n, nt);
  if (f >= n) return;  // this stage does not split
  static int whole[4096], gam[4096], rest[4096];
  for (int o = 0; o < n; ++o) whole[o] = gam[o] = rest[o] = 0;
  int wave_role[64];
  for (int w = 0; w < 64; ++w) wave_role[w] = -1;
  for (int t = 0; t < nt; ++t) {
    int role, o;
    split_role(t, n, nt, role, o);
    if (o < n) {
      CHECK(o >= 0, "split: negative cell");
      if (role == 0) whole[o]++;
      if (role == 1) gam[o]++;
      if (role == 2) rest[o]++;
      if (role != 0) CHECK(o - f >= 0 && o - f < nt / 2, "split: gamma slot %d out of range", o - f);
    }
    const int w = t / 64;
    CHECK(wave_role[w] < 0 || wave_role[w] == role, "split: wave %d holds two roles", w);
    wave_role[w] = role;
  }
  for (int o = 0; o < n; ++o)
    CHECK((whole[o] == 1 && gam[o] == 0 && rest[o] == 0) || (whole[o] == 0 && gam[o] == 1 && rest[o] == 1),
          "split: cell %d covered %d/%d/%d times", o, whole[o], gam[o], rest[o]);
}

template <int DIM, int TX, int TY>
void check_step(int nx, int ny, int per_x, int per_y) {
  using G = StepGeom<DIM, TX, TY>;
  StageArgs A{};
  A.nx = nx;
  A.ny = DIM == 2 ? ny : 1;
  A.per_x = per_x;
  A.per_y = DIM == 2 ? per_y : 0;
  const size_t ncells = (size_t)A.nx * A.ny;
  static int written[600 * 600];
  for (size_t e = 0; e < ncells; ++e) written[e] = 0;
  const int gx_blocks = (nx + TX - 1) / TX, gy_blocks = DIM == 2 ? (ny + TY - 1) / TY : 1;
  for (int by = 0; by < gy_blocks; ++by)
    for (int bx = 0; bx < gx_blocks; ++bx) {
      const int ix0 = bx * TX, iy0 = DIM == 2 ? by * TY : 0;
      for (int o = 0; o < G::A::N; ++o) {
        const int ox = o % G::A::W, oy = o / G::A::W;
        int wx, wy;
        if (step_cell<DIM>(A, ix0 - 3 + ox, DIM == 2 ? iy0 - 3 + oy : 0, wx, wy))
          CHECK(wx >= 0 && wx < A.nx && wy >= 0 && wy < A.ny, "step: tile A load out of range (%d, %d)", wx, wy);
      }
      check_step_stage<DIM, TX, TY, 2>(A, ix0, iy0, ncells, 9, written);
      check_step_stage<DIM, TX, TY, 1>(A, ix0, iy0, ncells, 9, written);
      check_step_stage<DIM, TX, TY, 0>(A, ix0, iy0, ncells, 9, written);
    }
  for (size_t e = 0; e < ncells; ++e) CHECK(written[e] == 1, "step: cell %zu written %d times", e, written[e]);
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

void sweep_step() {
  const int sizes[] = {1, 2, 3, 5, 15, 16, 17, 31, 33, 64, 100, 257, 513};
  for (int nx : sizes)
    for (int px = 0; px < 2; ++px) {
      check_step<1, kStepTile1D, 1>(nx, 1, px, 0);
      for (int ny : sizes)
        for (int py = 0; py < 2; ++py)
          if ((size_t)nx * ny <= 600 * 600) {
            check_step<2, kStepTile2D, kStepTile2D>(nx, ny, px, py);
            check_step<2, kStepTile2D, kStepTile2DHalf>(nx, ny, px, py);
          }
    }
}

// ---------------------------------------------------------------------------
// Batched runs: the classes, arena offsets, tile lists and persistent grids
// of the library's plan (dg_batch_plan.hpp) for a list of problems.  For one
// class and tile shape: every order's list holds the same tiles (each
// problem's mesh tiled once) within the class's preallocated capacity; every
// grid size visits each list entry exactly once; and for every tile and
// thread of batch_stage_kernel's loop, the problem index, the LDS planes and
// slots (own, halo and the four face-neighbour reads) and the arena entries
// of the loaded, combined and written cells stay inside their buffers, and
// every mesh cell of every problem is written exactly once per stage.
// ---------------------------------------------------------------------------
struct BatchProblemDesc {
  BatchMesh m;
  int per_x, per_y;
};

template <int DIM, int TX, int TY>
void check_batch_class(const std::vector<BatchProblemDesc>& pd, const std::vector<BatchMesh>& m,
                       const std::vector<long long>& off, const std::vector<int>& probs) {
  using G = TileGeom<DIM, TX, TY>;
  const int nl = m[probs[0]].nl();
  const long long lds = tile_lds_doubles(DIM, nl, TX, TY);
  CHECK(stage_lds_doubles(DIM, nl, m[probs[0]].flux, TX, TY) >= lds, "batch: stage LDS below the tile");
  const long long cap = batch_tile_capacity(m, probs);
  const long long total = off.back();
  std::vector<BatchTile> base, list;
  batch_tile_list(m, probs, TX, TY, 0, base);
  auto key = [](const BatchTile& t) { return ((long long)t.prob << 40) | ((long long)t.iy0 << 20) | t.ix0; };
  std::vector<long long> kb;
  for (auto& t : base) kb.push_back(key(t));
  std::sort(kb.begin(), kb.end());
  for (int order = 0; order < 3; ++order) {
    batch_tile_list(m, probs, TX, TY, order, list);
    CHECK((long long)list.size() <= cap, "batch: %zu tiles exceed the capacity %lld", list.size(), cap);
    std::vector<long long> kl;
    for (auto& t : list) kl.push_back(key(t));
    std::sort(kl.begin(), kl.end());
    CHECK(kl == kb, "batch: order %d lists other tiles than order 0", order);
    for (int g : {0, 1, 2, 4, 8, 64}) {
      const int grid = batch_grid(g, 256, (long long)list.size());
      CHECK(grid >= 1 && grid <= (long long)std::max<size_t>(1, list.size()), "batch: grid %d", grid);
      std::vector<int> seen(list.size(), 0);
      for (int b = 0; b < grid; ++b)
        for (long long k = b; k < (long long)list.size(); k += grid) seen[k]++;
      for (size_t k = 0; k < seen.size(); ++k) CHECK(seen[k] == 1, "batch: tile %zu visited %d times", k, seen[k]);
    }
  }
  // every tile and thread of the loop (the order only permutes the tiles)
  std::vector<unsigned char> written(total + 1, 0);
  for (const BatchTile& tl : base) {
    CHECK(tl.prob >= 0 && tl.prob < (int)m.size(), "batch: problem index %d", tl.prob);
    if (tl.prob < 0 || tl.prob >= (int)m.size()) continue;
    const BatchMesh& bm = m[tl.prob];
    CHECK(bm.dim == DIM && bm.nl() == nl, "batch: tile of another class");
    CHECK(tl.ix0 >= 0 && tl.ix0 < bm.nx && tl.iy0 >= 0 && tl.iy0 < bm.ny, "batch: tile origin outside the mesh");
    StageArgs A{};
    A.nx = bm.nx;
    A.ny = DIM == 2 ? bm.ny : 1;
    A.per_x = pd[tl.prob].per_x;
    A.per_y = DIM == 2 ? pd[tl.prob].per_y : 0;
    const long long o = off[tl.prob], ncells = bm.cells();
    const int offs[4] = {-1, 1, -G::W, G::W};
    for (int t = 0; t < G::NT; ++t) {
      int sc, gx, gy, hs, hgx, hgy;
      const bool halo = tile_slots<DIM, TX, TY>(t, tl.ix0, tl.iy0, sc, gx, gy, hs, hgx, hgy);
      CHECK(sc >= 0 && sc < G::NS && (long long)(nl - 1) * G::S + sc < lds, "batch: own LDS slot %d", sc);
      for (int f = 0; f < 2 * DIM; ++f)
        CHECK(sc + offs[f] >= 0 && sc + offs[f] < G::NS && (long long)(nl - 1) * G::S + sc + offs[f] < lds,
              "batch: neighbour LDS slot %d", sc + offs[f]);
      size_t cell;
      if (slot_cell<DIM>(A, gx, gy, cell))
        CHECK((long long)cell < ncells && o + ((long long)cell + 1) * nl <= off[tl.prob + 1],
              "batch: own load outside problem %d", tl.prob);
      if (halo) {
        CHECK(hs >= 0 && hs < G::NS && (long long)(nl - 1) * G::S + hs < lds, "batch: halo LDS slot %d", hs);
        if (slot_cell<DIM>(A, hgx, hgy, cell))
          CHECK((long long)cell < ncells && o + ((long long)cell + 1) * nl <= off[tl.prob + 1],
                "batch: halo load outside problem %d", tl.prob);
      }
      if (gx < A.nx && gy < A.ny) {
        const long long c = (long long)gy * A.nx + gx;
        CHECK(c < ncells && o + (c + 1) * nl <= total, "batch: output outside the arena");
        if (c < ncells) written[o + c * nl]++;
      }
    }
  }
  for (int i : probs)
    for (long long c = 0; c < m[i].cells(); ++c)
      CHECK(written[off[i] + c * m[i].nl()] == 1, "batch: cell %lld of problem %d written %d times", c, i,
            written[off[i] + c * m[i].nl()]);
}

// problems: one line each, "dim nx ny p flux mode per_x per_y"
int check_batch(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) {
    std::printf("cannot open %s\n", path);
    return 1;
  }
  std::vector<BatchProblemDesc> pd;
  BatchProblemDesc d{};
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d", &d.m.dim, &d.m.nx, &d.m.ny, &d.m.p, &d.m.flux, &d.m.mode,
                     &d.per_x, &d.per_y) == 8) {
    if (d.m.dim == 1) d.m.ny = 1;
    pd.push_back(d);
  }
  std::fclose(f);
  std::vector<BatchMesh> m;
  for (auto& x : pd) m.push_back(x.m);
  const std::vector<long long> off = batch_offsets(m);
  for (size_t i = 0; i < m.size(); ++i) CHECK(off[i + 1] - off[i] == m[i].cells() * m[i].nl(), "batch: offsets");
  const auto classes = batch_classes(m);
  size_t members = 0;
  for (const auto& probs : classes) {
    members += probs.size();
    const BatchMesh& c0 = m[probs[0]];
    for (int i : probs)
      CHECK(m[i].dim == c0.dim && m[i].p == c0.p && m[i].flux == c0.flux && m[i].mode == c0.mode,
            "batch: class with mixed kernels");
    const int nl = c0.nl();
    if (c0.dim == 1) {
      check_batch_class<1, 256, 1>(pd, m, off, probs);
      check_batch_class<1, 64, 1>(pd, m, off, probs);
    } else {
      // the 16x16 tile where its LDS fits the 64 KB a workgroup gets by default
      if (stage_lds_doubles(2, nl, c0.flux, 16, 16) * 8 <= 65536) check_batch_class<2, 16, 16>(pd, m, off, probs);
      check_batch_class<2, 8, 8>(pd, m, off, probs);
    }
  }
  CHECK(members == m.size(), "batch: %zu problems in classes, %zu given", members, m.size());
  std::printf("batch: %zu problems, %zu classes, %lld doubles\n", m.size(), classes.size(), off.back());
  return 0;
}

// The KPP 8x8 kernel of four waves (kpp_split_tile) at degree p: every
// volume node and face node task reads slots inside the tile (no corner),
// writes its own entry of the node planes exactly once, inside LDS, and the
// cells read back exactly the entries of their own nodes and faces.
void check_kpp_split(int p) {
  using G = TileGeom<2, 8, 8>;
  const int q = quad_points(2, p, FLUX_KPP), nl = (p + 1) * (p + 1);
  const long long tile = tile_lds_doubles(2, nl, 8, 8), lds = split_lds_doubles(nl, q);
  CHECK(stage_kernel_lds_doubles(2, nl, p, FLUX_KPP, 8, 8) == lds &&
            stage_kernel_lds_doubles(2, nl, p, FLUX_KPP, 16, 16) == stage_lds_doubles(2, nl, FLUX_KPP, 16, 16) &&
            stage_kernel_lds_doubles(2, nl, p, FLUX_BURGERS, 16, 16) == stage_lds_doubles(2, nl, FLUX_BURGERS, 16, 16) &&
            stage_kernel_lds_doubles(2, nl, p, FLUX_BURGERS, 8, 8) >= stage_lds_doubles(2, nl, FLUX_BURGERS, 8, 8),
        "kpp split: LDS size");
  auto corner = [&](int s) {
    const int x = s % G::W, y = s / G::W;
    return (x == 0 || x == G::W - 1) && (y == 0 || y == G::H - 1);
  };
  const int nv = 64 * q * q, nfn = 144 * q;
  std::vector<int> vw(nv, 0), fw(nfn, 0);
  for (int v = 0; v < nv; ++v) {
    int slot, qx, qy;
    const int o = split_vol_task(v, q, slot, qx, qy);
    CHECK(slot >= 0 && slot < G::NS && !corner(slot) && slot % G::W > 0 && slot % G::W <= 8 && slot / G::W > 0 &&
              slot / G::W <= 8,
          "kpp split: volume task %d reads slot %d outside the tile cells", v, slot);
    CHECK(qx >= 0 && qx < q && qy >= 0 && qy < q, "kpp split: volume task %d node", v);
    CHECK(o >= 0 && o < nv && tile + nv + o < lds, "kpp split: volume task %d entry %d", v, o);
    if (o >= 0 && o < nv) vw[o]++;
    // tile cell lc reads its node (qx, qy) at (qx q + qy) 64 + lc
    const int lc = v & 63;
    CHECK(o == (qx * q + qy) * 64 + lc && slot == ((lc / 8) + 1) * G::W + lc % 8 + 1,
          "kpp split: volume task %d is not cell %d's node", v, lc);
  }
  for (int o = 0; o < nv; ++o) CHECK(vw[o] == 1, "kpp split: volume entry %d written %d times", o, vw[o]);
  const int ix0 = 5 * 8, iy0 = 2 * 8;
  for (int i = 0; i < nfn; ++i) {
    int axis, r, e;
    const int o = split_face_task(i, q, axis, r, e);
    CHECK(axis >= 0 && axis < 2 && r >= 0 && r < q && e >= 0 && e < 72, "kpp split: face task %d", i);
    CHECK(o >= 0 && o < nfn && tile + 2LL * nv + o < lds, "kpp split: face task %d entry %d", i, o);
    if (o >= 0 && o < nfn) fw[o]++;
    int gx, gy;
    const int lo = face_slot<8, 8>(axis, e, ix0, iy0, gx, gy), hi = lo + (axis ? G::W : 1);
    CHECK(lo >= 0 && hi < G::NS && !corner(lo) && !corner(hi), "kpp split: face %d slots %d %d", e, lo, hi);
  }
  for (int o = 0; o < nfn; ++o) CHECK(fw[o] == 1, "kpp split: face entry %d written %d times", o, fw[o]);
  for (int lc = 0; lc < 64; ++lc) {
    int sc, gx, gy, hs, hgx, hgy;
    tile_slots<2, 8, 8>(lc, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
    for (int f = 0; f < 4; ++f) {
      const int axis = f >> 1, e = split_cell_face(lc, f);
      CHECK(e >= 0 && e < 72, "kpp split: face %d of cell %d", f, lc);
      int fx, fy;
      const int lo = face_slot<8, 8>(axis, e, ix0, iy0, fx, fy);
      const int want = f == 0 ? sc - 1 : f == 1 ? sc : f == 2 ? sc - G::W : sc;
      CHECK(lo == want, "kpp split: face %d of cell %d has lower slot %d, not %d", f, lc, lo, want);
      for (int r = 0; r < q; ++r) CHECK((axis * q + r) * 72 + e < nfn, "kpp split: face read outside its planes");
    }
  }
  // wave 0's volume rounds: whole rounds within the node count
  for (int nth : {256, 512, 1024}) CHECK(split_v0(p, nth) >= 0 && split_v0(p, nth) <= q * q, "kpp split: v0");
}

// The four-wave 8x8 kernel (roles_tile) at nl coefficients: its face tasks
// cover each of the tile's 144 faces once, read slots inside the tile (no
// corner) and write moments inside LDS; each cell reads back the moments of
// its own four faces; the gamma exchange fits after the faces.
void check_roles(int nl) {
  using G = TileGeom<2, 8, 8>;
  using FG = FaceGeom<8, 8>;
  int n = 1;
  while (n * n < nl) ++n;
  const long long lds = roles_lds_doubles(nl, n);
  CHECK(lds == tile_lds_doubles(2, nl, 8, 8) + (long long)n * (FG::XS + FG::YS) + 64, "roles: LDS size");
  for (int flux : {FLUX_LINADV, FLUX_BURGERS})
    CHECK(stage_kernel_lds_doubles(2, nl, n - 1, flux, 8, 8) >= lds, "roles: the API's LDS bound");
  auto corner = [&](int s) {
    const int x = s % G::W, y = s / G::W;
    return (x == 0 || x == G::W - 1) && (y == 0 || y == G::H - 1);
  };
  std::vector<int> cx(FG::NXF, 0), cy(FG::NYF, 0);
  const int ix0 = 2 * 8, iy0 = 7 * 8;
  for (int t = 128; t < kRoleThreads; ++t)
    for (int i = t - 128; i < FG::NXF + FG::NYF; i += kRoleThreads - 128) {
      int axis, e;
      roles_face_task(i, axis, e);
      CHECK(axis >= 0 && axis < 2 && e >= 0 && e < (axis ? FG::NYF : FG::NXF), "roles: face task %d", i);
      if (axis == 0 && e >= 0 && e < FG::NXF) cx[e]++;
      if (axis == 1 && e >= 0 && e < FG::NYF) cy[e]++;
      int gx, gy;
      const int lo = face_slot<8, 8>(axis, e, ix0, iy0, gx, gy), hi = lo + (axis ? G::W : 1);
      CHECK(lo >= 0 && hi < G::NS && !corner(lo) && !corner(hi), "roles: face %d slots %d %d", e, lo, hi);
      const long long base = (long long)nl * G::S + (axis ? (long long)n * FG::XS : 0);
      CHECK(base + (long long)(n - 1) * (axis ? FG::YS : FG::XS) + e < lds - 64, "roles: moments of face %d", e);
    }
  for (int e = 0; e < FG::NXF; ++e) CHECK(cx[e] == 1, "roles: x face %d evaluated %d times", e, cx[e]);
  for (int e = 0; e < FG::NYF; ++e) CHECK(cy[e] == 1, "roles: y face %d evaluated %d times", e, cy[e]);
  for (int lc = 0; lc < 64; ++lc) {
    int sc, gx, gy, hs, hgx, hgy;
    tile_slots<2, 8, 8>(lc, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
    const int lx = lc % 8, ly = lc / 8, ex = ly * 9 + lx, ey = ly * 8 + lx;
    int fx, fy;
    const int s0 = face_slot<8, 8>(0, ex, ix0, iy0, fx, fy), s1 = face_slot<8, 8>(0, ex + 1, ix0, iy0, fx, fy);
    const int s2 = face_slot<8, 8>(1, ey, ix0, iy0, fx, fy), s3 = face_slot<8, 8>(1, ey + 8, ix0, iy0, fx, fy);
    CHECK(s0 + 1 == sc && s1 == sc && s2 + G::W == sc && s3 == sc, "roles: faces of cell %d", lc);
    CHECK((long long)nl * G::S + (long long)n * (FG::XS + FG::YS) + lc < lds, "roles: gamma slot of cell %d", lc);
  }
}

// The fused Euler step (euler_step_kernel) on an nx-cell mesh: the loads of
// tile A read cells inside the mesh, every stage reads its input slots and
// U^n slots inside their tiles and writes inside its output tile, the three
// tiles fit the LDS size, and the last stage writes each mesh cell once.
void check_euler_step(int nx, int per, int p) {
  constexpr int T = kEulerStepTile;
  const int nle = 3 * (p + 1);
  const long long sa = (T + 6) | 1, sb = (T + 4) | 1, sc = (T + 2) | 1;
  CHECK(euler_step_lds_doubles(p) == nle * (sa + sb + sc), "euler step: LDS size");
  StageArgs A{};
  A.nx = nx;
  A.ny = 1;
  A.per_x = per;
  std::vector<int> written(nx, 0);
  const int tiles = (nx + T - 1) / T;
  for (int k = 0; k < tiles; ++k) {
    const int ix0 = xcd_tile(k, tiles) * T;
    for (int o = 0; o < T + 6; ++o) {
      int wx, wy;
      if (step_cell<1>(A, ix0 - 3 + o, 0, wx, wy)) CHECK(wx >= 0 && wx < nx, "euler step: load of cell %d", wx);
    }
    // stages: (input interior width, output cells, first x, U^n offset)
    const int txi[3] = {T + 4, T + 2, T}, gx0[3] = {ix0 - 2, ix0 - 1, ix0}, aoff[3] = {1, 2, 3};
    for (int st = 0; st < 3; ++st) {
      const int nout = txi[st];
      for (int t = 0; t < kEulerStepThreads; ++t)
        for (int o = t; o < nout; o += kEulerStepThreads) {
          const int gx = gx0[st] + o;
          CHECK(o + 2 < txi[st] + 2, "euler step: stage %d input slots of cell %d", st, o);  // o - 1 + 1 .. o + 1 + 1
          CHECK(o + aoff[st] < T + 6, "euler step: U^n slot of cell %d", o);
          if (st < 2) CHECK(o < ((txi[st]) | 1), "euler step: output slot %d", o);
          int wx, wy;
          const bool in = step_cell<1>(A, gx, 0, wx, wy);
          if (st == 2 && in && gx < nx) {
            CHECK(wx == gx, "euler step: last stage cell %d wrapped", gx);
            if (wx >= 0 && wx < nx) written[wx]++;
          }
        }
    }
  }
  for (int e = 0; e < nx; ++e) CHECK(written[e] == 1, "euler step: cell %d written %d times (nx %d)", e, written[e], nx);
}

// xcd_tile is a bijection of [0, g) for every grid size, and each XCD's
// workgroups take one contiguous, increasing run of tiles.
void check_xcd_order() {
  for (int g = 1; g <= 5000; g += (g < 300 ? 1 : 37)) {
    std::vector<int> seen(g, 0), last(kXcds, -1);
    for (int k = 0; k < g; ++k) {
      const int t = xcd_tile(k, g);
      CHECK(t >= 0 && t < g, "xcd order: tile %d of %d", t, g);
      if (t < 0 || t >= g) continue;
      seen[t]++;
      const int x = k % kXcds;
      CHECK(last[x] < 0 || t == last[x] + 1, "xcd order: XCD %d jumps from tile %d to %d (g %d)", x, last[x], t, g);
      last[x] = t;
    }
    for (int t = 0; t < g; ++t) CHECK(seen[t] == 1, "xcd order: tile %d taken %d times (g %d)", t, seen[t], g);
  }
}

int main(int argc, char** argv) {
  if (argc > 1) {
    if (check_batch(argv[1])) return 1;
    std::printf("%s (%d failures)\n", failures ? "FAIL" : "ok", failures);
    return failures ? 1 : 0;
  }
  check_split<2, kStepTile2D, kStepTile2D, 2>();
  check_split<2, kStepTile2D, kStepTile2D, 1>();
  check_split<2, kStepTile2D, kStepTile2D, 0>();
  check_split<2, kStepTile2D, kStepTile2DHalf, 2>();
  check_split<2, kStepTile2D, kStepTile2DHalf, 1>();
  check_split<2, kStepTile2D, kStepTile2DHalf, 0>();
  check_split<1, kStepTile1D, 1, 2>();
  check_split<1, kStepTile1D, 1, 1>();
  check_split<1, kStepTile1D, 1, 0>();
  static_assert(split_full(256, 512) == 0 && split_full(324, 512) == 256 && split_full(400, 512) == 400,
                "16x16 fused step: stage 3 splits every cell, stage 2 the cells past 256, stage 1 none");
  static_assert(split_full(128, 256) == 0 && split_full(180, 256) == 128 && split_full(240, 256) == 240,
                "16x8 fused step: stage 3 splits every cell, stage 2 the cells past 128, stage 1 none");
  check_xcd_order();
  sweep_step();
  sweep<1, 256, 1>();
  sweep<1, 64, 1>();
  sweep<2, 16, 16>();
  sweep<2, 8, 8>();
  sweep<2, kAdjTileX, kAdjTileY>();  // the adjoint kernels' 2D tile
  for (int nl : {4, 9, 16, 25})
    for (int flux : {FLUX_LINADV, FLUX_BURGERS, FLUX_KPP}) {
      check_faces<16, 16>(nl, flux);
      check_faces<8, 8>(nl, flux);
    }
  for (int p = 1; p <= 4; ++p) check_kpp_split(p);
  for (int nl : {4, 9, 16, 25}) check_roles(nl);
  for (int nx : {1, 2, 3, 128, 255, 256, 257, 600, 4096 + 17})
    for (int per : {0, 1})
      for (int p = 1; p <= 4; ++p) check_euler_step(nx, per, p);
  static_assert(splits_nodes(2, FLUX_KPP, 8, 8) && !splits_nodes(2, FLUX_KPP, 16, 16) &&
                    !splits_nodes(2, FLUX_BURGERS, 8, 8),
                "the node split: 2D KPP on 8x8 tiles only");
  static_assert(split_waves(256, 256, 2) == 16 && split_waves(257, 256, 2) == 8 && split_waves(512, 256, 2) == 8 &&
                    split_waves(513, 256, 2) == 4 && split_waves(256, 256, 1) == 16 &&
                    split_waves(256, 256, 3) == 8 && split_waves(256, 256, 4) == 4 && split_v0(2, 256) == 8 &&
                    split_v0(2, 512) == 2 && split_v0(2, 1024) == 1,
                "KPP split: waves per tile and wave 0's volume rounds");
  static_assert(shares_faces(2, 2, FLUX_BURGERS, 16, 16) && shares_faces(2, 2, FLUX_KPP, 16, 16) &&
                    !shares_faces(2, 2, FLUX_LINADV, 16, 16) && !shares_faces(2, 3, FLUX_BURGERS, 16, 16) &&
                    !shares_faces(2, 2, FLUX_BURGERS, 8, 8) && !shares_faces(1, 2, FLUX_BURGERS, 256, 1),
                "shared faces: 2D 16x16 tiles, p = 2, Burgers and KPP");
  std::printf("%s (%d failures)\n", failures ? "FAIL" : "ok", failures);
  return failures ? 1 : 0;
}
