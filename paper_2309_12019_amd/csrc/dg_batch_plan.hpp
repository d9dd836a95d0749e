// Host-side plan of a batched run: kernel classes, arena offsets, per-class
// tile lists and the persistent grid.  The library (dg_batch.hip) and the
// host bounds harness (tests/native/index_bounds.hip) run these same
// functions, so the harness checks the lists the kernels actually walk.
#pragma once

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "dg_kernels.hpp"

namespace dgk {

// What the plan needs of one problem: mesh shape, coefficients per cell and
// its kernel class (dimension, degree, flux, mode).  ny = 1 in 1D.
struct BatchMesh {
  int dim, nx, ny, p, flux, mode;
  int nl() const { return dim == 1 ? p + 1 : (p + 1) * (p + 1); }
  long long cells() const { return (long long)nx * ny; }
};

// Arena layout: problem i's state is double[cells_i][nl_i] starting at
// offsets[i]; offsets[n] is the arena's size in doubles.
inline std::vector<long long> batch_offsets(const std::vector<BatchMesh>& m) {
  std::vector<long long> off(m.size() + 1, 0);
  for (size_t i = 0; i < m.size(); ++i) off[i + 1] = off[i] + m[i].cells() * m[i].nl();
  return off;
}

// Problems grouped by kernel class, classes in the order their first problem
// appears; problems in a class in batch order.
inline std::vector<std::vector<int>> batch_classes(const std::vector<BatchMesh>& m) {
  std::map<std::tuple<int, int, int, int>, int> key;
  std::vector<std::vector<int>> out;
  for (int i = 0; i < (int)m.size(); ++i) {
    const auto k = std::make_tuple(m[i].dim, m[i].p, m[i].flux, m[i].mode);
    auto it = key.find(k);
    if (it == key.end()) {
      it = key.emplace(k, (int)out.size()).first;
      out.emplace_back();
    }
    out[it->second].push_back(i);
  }
  return out;
}

// Tiles of one problem for a tile of tx x ty cells (ty ignored in 1D)
inline long long batch_tiles_of(const BatchMesh& m, int tx, int ty) {
  const long long nxt = (m.nx + tx - 1) / tx;
  return m.dim == 2 ? nxt * ((m.ny + ty - 1) / ty) : nxt;
}

// The tile list of one class: every problem's tiles, tile origins row by row
// within a problem; problems largest-first (order 0), smallest-first (order
// 1), or round robin over the problems taken largest-first (order 2, one
// tile of each problem in turn).
inline void batch_tile_list(const std::vector<BatchMesh>& m, const std::vector<int>& probs, int tx, int ty,
                            int order, std::vector<BatchTile>& all) {
  std::vector<int> seq = probs;
  auto cells = [&](int i) { return m[i].cells(); };
  if (order == 1)
    std::stable_sort(seq.begin(), seq.end(), [&](int x, int y) { return cells(x) < cells(y); });
  else
    std::stable_sort(seq.begin(), seq.end(), [&](int x, int y) { return cells(x) > cells(y); });
  std::vector<std::vector<BatchTile>> per;
  for (int i : seq) {
    const BatchMesh& d = m[i];
    std::vector<BatchTile> t;
    for (int y = 0; y < d.ny; y += (d.dim == 2 ? ty : 1))
      for (int x = 0; x < d.nx; x += tx) t.push_back(BatchTile{i, x, y, 0});
    per.push_back(std::move(t));
  }
  all.clear();
  if (order == 2) {
    size_t k = 0;
    bool more = true;
    while (more) {
      more = false;
      for (auto& t : per)
        if (k < t.size()) {
          all.push_back(t[k]);
          more = true;
        }
      ++k;
    }
  } else {
    for (auto& t : per) all.insert(all.end(), t.begin(), t.end());
  }
}

// Longest tile list any supported tile shape gives for a class: the capacity
// of its device list, allocated once when the batch is created.
inline long long batch_tile_capacity(const std::vector<BatchMesh>& m, const std::vector<int>& probs) {
  long long cap = 0;
  if (probs.empty()) return 0;
  if (m[probs[0]].dim == 1) {
    for (int t : kTiles1D) {
      long long n = 0;
      for (int i : probs) n += batch_tiles_of(m[i], t, 1);
      cap = std::max(cap, n);
    }
  } else {
    for (auto& t : kTiles2D) {
      long long n = 0;
      for (int i : probs) n += batch_tiles_of(m[i], t[0], t[1]);
      cap = std::max(cap, n);
    }
  }
  return cap;
}

// Workgroups of a class launch: grid_per_cu per compute unit, at most one
// per tile, at least one.  Workgroup g walks tiles g, g + grid, g + 2 grid, ...
// grid_per_cu = 0: one workgroup per tile (the kernel without the tile loop).
inline int batch_grid(int grid_per_cu, int cus, long long ntiles) {
  const long long g = grid_per_cu == 0 ? ntiles : (long long)grid_per_cu * cus;
  return (int)std::max<long long>(1, std::min<long long>(g, ntiles));
}

}  // namespace dgk
