// face_groups.hip -- face groups and planes of a triangle scene (host code).
//
// Triangles whose planes agree (|n_a . n_b| >= 1 - 1e-12 and offsets within
// 1e-9 of the scene diagonal) share a plane id; with equal materials also a
// group id, the unit a path key records per bounce.  Both relations are
// closed transitively, and ids are numbered in order of each class's lowest
// triangle.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

struct Key4 {
  int64_t a, b, c, d;
  bool operator==(const Key4& o) const { return a == o.a && b == o.b && c == o.c && d == o.d; }
};
struct Key4Hash {
  size_t operator()(const Key4& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int64_t v : {k.a, k.b, k.c, k.d}) h = (h ^ (uint64_t)v) * 1099511628211ull;
    return (size_t)h;
  }
};

// Open-addressing map from Key4 to an int (linear probing, power-of-two
// capacity of at least twice the entries); -1 marks an empty slot's value.
// The storage is kept by the caller across calls (reset() only grows it and
// clears the value slots in use), so repeated scene builds neither allocate
// nor touch fresh pages.
struct FlatMap4 {
  std::vector<Key4> keys;
  std::vector<int> vals;
  size_t mask = 0;
  void reset(size_t n) {
    size_t cap = 16;
    while (cap < 2 * n + 16) cap <<= 1;
    if (keys.size() < cap) keys.resize(cap), vals.resize(cap);
    std::fill(vals.begin(), vals.begin() + cap, -1);
    mask = cap - 1;
  }
  size_t slot(const Key4& k) const {
    uint64_t h = (uint64_t)Key4Hash{}(k);
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    size_t i = (size_t)h & mask;
    while (vals[i] >= 0 && !(keys[i] == k)) i = (i + 1) & mask;
    return i;
  }
  // value stored for k, or -1
  int get(const Key4& k) const { return vals[slot(k)]; }
  // value stored for k; stores v first when k is absent
  int get_or_put(const Key4& k, int v) {
    const size_t i = slot(k);
    if (vals[i] < 0) keys[i] = k, vals[i] = v;
    return vals[i];
  }
  void put(const Key4& k, int v) {
    const size_t i = slot(k);
    keys[i] = k, vals[i] = v;
  }
};

int uf_find(std::vector<int>& p, int x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}
void uf_join(std::vector<int>& p, int a, int b) {
  a = uf_find(p, a), b = uf_find(p, b);
  if (a < b) p[b] = a;
  else if (b < a) p[a] = b;
}

}  // namespace

// Pairs with |n_a . n_b| >= 1 - 1e-12 and matching offsets (1e-9 diag) share a
// plane; with equal materials also a group (transitive closure, ids in order
// of the lowest triangle).  Candidate pairs come from a hash grid over the
// sign-canonical (n, c) with cells far wider than the tolerances; a triangle
// probes a neighbouring cell only along a dimension where it lies within the
// tolerance of the cell border, and also probes (-n, -c) when its largest
// normal component is not clearly the largest.
void face_groups(const std::vector<Plane>& pl, const float* eps, const float* sig, const float* rough, double diag,
                 std::vector<int32_t>& group, std::vector<int32_t>& plane, int& ngroups, int& nplanes) {
  const int T = (int)pl.size();
  const double tol_n = 2e-6;  // |n_a - n_b| <= 1.42e-6 when n_a . n_b >= 1 - 1e-12
  const double tol_c = 1e-9 * diag * (1.0 + 1e-9) + 1e-300;
  const double hn = 1.0 / 1024.0, hc = std::max(1e-3 * diag, 1e-300);
  struct Canon {
    double v[4];
    bool ambiguous;
  };
  std::vector<Canon> cn(T);
  for (int t = 0; t < T; ++t) {
    const double* n = pl[t].n;
    int imax = 0;
    for (int k = 1; k < 3; ++k)
      if (std::fabs(n[k]) > std::fabs(n[imax])) imax = k;
    double second = 0.0;
    for (int k = 0; k < 3; ++k)
      if (k != imax) second = std::max(second, std::fabs(n[k]));
    const double sgn = n[imax] < 0 ? -1.0 : 1.0;
    cn[t] = Canon{{sgn * n[0], sgn * n[1], sgn * n[2], sgn * pl[t].c}, std::fabs(n[imax]) - second < 4 * tol_n};
  }
  // cell coordinates by multiplication with the inverse cell sizes and an
  // inline floor (the same function serves insertion and probing)
  const double ihn = 1.0 / hn, ihc = 1.0 / hc;
  auto ifloor = [](double x) {
    const int64_t i = (int64_t)x;
    return i - (int64_t)(x < (double)i);
  };
  auto cell = [&](const double* v, int k) { return ifloor(v[k] * (k < 3 ? ihn : ihc)); };
  // Triangles whose canonical (n, c) are bitwise equal form one class (many
  // box bottoms lie exactly on a floor): they are joined directly, and only
  // one representative per class enters the pairwise tolerance tests, which
  // gives the same transitive closure as testing every pair.  Within a
  // class, members of equal material are joined into one group; across
  // classes, the per-material representatives of matching materials are.
  auto bits = [](double x) {
    int64_t b;
    std::memcpy(&b, &x, 8);
    return b;
  };
  std::vector<int> pp(T), pg(T);
  for (int t = 0; t < T; ++t) pp[t] = pg[t] = t;
  // A material as a key: the bit patterns of (eps, sigma, roughness) with -0
  // read as +0, so that equal keys mean equal values (inputs are finite).
  auto mat_key = [&](int q, int t) {
    auto fb = [](float x) {
      x += 0.0f;
      int32_t b;
      std::memcpy(&b, &x, 4);
      return (int64_t)b;
    };
    return Key4{(int64_t)q, fb(eps[t]), fb(sig[t]), fb(rough[t])};
  };
  // classes in flat arrays: representative, number of distinct materials and
  // the first material representative; each class's material
  // representatives are listed through mat_next (by triangle)
  std::vector<int> cls_rep, cls_nmat, cls_mat, mat_next((size_t)T, -1);
  cls_rep.reserve(T), cls_nmat.reserve(T), cls_mat.reserve(T);
  static thread_local FlatMap4 clsmat, cls, grid;
  clsmat.reset((size_t)T);  // (class, material) -> representative triangle
  {
    cls.reset((size_t)T);  // canonical plane -> class
    for (int t = 0; t < T; ++t) {
      const Key4 k{bits(cn[t].v[0]), bits(cn[t].v[1]), bits(cn[t].v[2]), bits(cn[t].v[3])};
      const int q = cls.get_or_put(k, (int)cls_rep.size());
      if (q == (int)cls_rep.size()) {
        cls_rep.push_back(t), cls_nmat.push_back(1), cls_mat.push_back(t);
        clsmat.put(mat_key(q, t), t);
        continue;
      }
      uf_join(pp, cls_rep[q], t);
      const int r = clsmat.get_or_put(mat_key(q, t), t);
      if (r == t) {
        mat_next[t] = cls_mat[q];
        cls_mat[q] = t;
        ++cls_nmat[q];
      } else {
        uf_join(pg, r, t);
      }
    }
  }
  const int NC = (int)cls_rep.size();
  // cell -> classes, as a list threaded through next_in_cell
  grid.reset((size_t)NC);
  std::vector<int> next_in_cell(NC, -1);
  for (int q = 0; q < NC; ++q) {
    const double* v = cn[cls_rep[q]].v;
    const Key4 k{cell(v, 0), cell(v, 1), cell(v, 2), cell(v, 3)};
    next_in_cell[q] = grid.get(k);
    grid.put(k, q);
  }
  for (int qa = 0; qa < NC; ++qa) {
    const int a = cls_rep[qa];
    for (int flip = 0; flip < (cn[a].ambiguous ? 2 : 1); ++flip) {
      double v[4];
      for (int k = 0; k < 4; ++k) v[k] = flip ? -cn[a].v[k] : cn[a].v[k];
      int64_t base[4];
      int lo[4], hi[4];
      for (int k = 0; k < 4; ++k) {
        const double h = k < 3 ? hn : hc, tol = k < 3 ? tol_n : tol_c;
        base[k] = cell(v, k);
        const double f = v[k] * (k < 3 ? ihn : ihc) - (double)base[k];
        lo[k] = f * h <= tol ? -1 : 0;
        hi[k] = (1.0 - f) * h <= tol ? 1 : 0;
      }
      for (int dx = lo[0]; dx <= hi[0]; ++dx)
        for (int dy = lo[1]; dy <= hi[1]; ++dy)
          for (int dz = lo[2]; dz <= hi[2]; ++dz)
            for (int dc = lo[3]; dc <= hi[3]; ++dc) {
              for (int qb = grid.get(Key4{base[0] + dx, base[1] + dy, base[2] + dz, base[3] + dc}); qb >= 0;
                   qb = next_in_cell[qb]) {
                if (qb == qa) continue;
                const int b = cls_rep[qb];
                const double nd = pl[a].n[0] * pl[b].n[0] + pl[a].n[1] * pl[b].n[1] + pl[a].n[2] * pl[b].n[2];
                if (std::fabs(nd) < 1.0 - 1e-12) continue;
                const double sg = nd > 0 ? 1.0 : -1.0;
                if (std::fabs(pl[a].c - sg * pl[b].c) > 1e-9 * diag) continue;
                uf_join(pp, a, b);
                // equal materials of the two classes: look the smaller list up in the other class
                const bool a_small = cls_nmat[qa] <= cls_nmat[qb];
                const int qs = a_small ? qa : qb, ql = a_small ? qb : qa;
                for (int ms = cls_mat[qs]; ms >= 0; ms = mat_next[ms]) {
                  const int ml = clsmat.get(mat_key(ql, ms));
                  if (ml >= 0) uf_join(pg, ms, ml);
                }
              }
            }
    }
  }
  std::vector<int> gid(T, -1), pid(T, -1);
  ngroups = nplanes = 0;
  group.assign(T, 0);
  plane.assign(T, 0);
  for (int t = 0; t < T; ++t) {
    const int rg = uf_find(pg, t), rp = uf_find(pp, t);
    if (gid[rg] < 0) gid[rg] = ngroups++;
    if (pid[rp] < 0) pid[rp] = nplanes++;
    group[t] = gid[rg];
    plane[t] = pid[rp];
  }
}

}  // namespace sbr
