// P1 meshes on the host: red refinement, boundary faces, interior numbering,
// element-by-element assembly of M_h and K_h, nested interpolation.
#include "stmg_mesh.h"

#include <algorithm>
#include <array>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <limits>
#include <unordered_map>

namespace stmg {

namespace {

// local edges of a cell, in sweep order
const int EDGES3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int EDGES2[3][2] = {{0, 1}, {0, 2}, {1, 2}};

long long edge_key(int a, int b) {
  const long long lo = std::min(a, b), hi = std::max(a, b);
  return (lo << 32) | hi;
}

// Signed d x d determinant of the edge vectors of cell c and, optionally, the
// inverse of the edge matrix B (columns x_i - x_0), row-major.
double edge_matrix(const MeshLevel& L, const int* c, double* Binv) {
  const int d = L.d;
  double B[9];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) B[i * d + j] = L.xyz[(size_t)c[j + 1] * d + i] - L.xyz[(size_t)c[0] * d + i];
  double det;
  if (d == 2) {
    det = B[0] * B[3] - B[1] * B[2];
    if (Binv && det != 0.0) {
      Binv[0] = B[3] / det;
      Binv[1] = -B[1] / det;
      Binv[2] = -B[2] / det;
      Binv[3] = B[0] / det;
    }
    return det;
  }
  const double c00 = B[4] * B[8] - B[5] * B[7];
  const double c01 = B[5] * B[6] - B[3] * B[8];
  const double c02 = B[3] * B[7] - B[4] * B[6];
  det = B[0] * c00 + B[1] * c01 + B[2] * c02;
  if (Binv && det != 0.0) {
    Binv[0] = c00 / det;
    Binv[3] = c01 / det;
    Binv[6] = c02 / det;
    Binv[1] = (B[2] * B[7] - B[1] * B[8]) / det;
    Binv[4] = (B[0] * B[8] - B[2] * B[6]) / det;
    Binv[7] = (B[1] * B[6] - B[0] * B[7]) / det;
    Binv[2] = (B[1] * B[5] - B[2] * B[4]) / det;
    Binv[5] = (B[2] * B[3] - B[0] * B[5]) / det;
    Binv[8] = (B[0] * B[4] - B[1] * B[3]) / det;
  }
  return det;
}

// Lexicographic comparison of two nodes' coordinates.
int coord_cmp(const MeshLevel& L, int p, int q) {
  for (int i = 0; i < L.d; ++i) {
    const double a = L.xyz[(size_t)p * L.d + i], b = L.xyz[(size_t)q * L.d + i];
    if (a < b) return -1;
    if (a > b) return 1;
  }
  return 0;
}

MeshLevel refine(const MeshLevel& C) {
  const int d = C.d, nv = d + 1;
  MeshLevel F;
  F.d = d;
  F.xyz = C.xyz;
  F.par.assign((size_t)C.nodes() * 2, -1);
  std::unordered_map<long long, int> mid;
  mid.reserve((size_t)C.cells() * (d == 3 ? 2 : 2));
  const int ne = d == 3 ? 6 : 3;
  const int(*E)[2] = d == 3 ? EDGES3 : EDGES2;
  for (long long t = 0; t < C.cells(); ++t) {
    const int* c = &C.cell[(size_t)t * nv];
    for (int e = 0; e < ne; ++e) {
      const int a = c[E[e][0]], b = c[E[e][1]];
      const long long k = edge_key(a, b);
      if (mid.find(k) != mid.end()) continue;
      const int id = (int)(F.xyz.size() / d);
      mid.emplace(k, id);
      const int lo = std::min(a, b), hi = std::max(a, b);
      for (int i = 0; i < d; ++i)
        F.xyz.push_back(0.5 * (C.xyz[(size_t)lo * d + i] + C.xyz[(size_t)hi * d + i]));
      F.par.push_back(lo);
      F.par.push_back(hi);
    }
  }
  F.cell.reserve((size_t)C.cells() * nv * (d == 3 ? 8 : 4));
  auto put = [&](std::initializer_list<int> v) { F.cell.insert(F.cell.end(), v); };
  for (long long t = 0; t < C.cells(); ++t) {
    const int* c = &C.cell[(size_t)t * nv];
    int m[4][4];
    for (int e = 0; e < ne; ++e) {
      const int i = E[e][0], j = E[e][1];
      m[i][j] = m[j][i] = mid.at(edge_key(c[i], c[j]));
    }
    if (d == 2) {
      put({c[0], m[0][1], m[0][2]});
      put({m[0][1], c[1], m[1][2]});
      put({m[0][2], m[1][2], c[2]});
      put({m[0][1], m[1][2], m[0][2]});
      continue;
    }
    put({c[0], m[0][1], m[0][2], m[0][3]});
    put({m[0][1], c[1], m[1][2], m[1][3]});
    put({m[0][2], m[1][2], c[2], m[2][3]});
    put({m[0][3], m[1][3], m[2][3], c[3]});
    // inner octahedron: cut along the shortest of the three diagonals joining
    // midpoints of opposite edges; ties go to the smaller (lower endpoint,
    // higher endpoint) in lexicographic coordinate order
    const int opp[3][4] = {{0, 1, 2, 3}, {0, 2, 1, 3}, {0, 3, 1, 2}};
    int best = -1;
    double bl = 0;
    int blo = -1, bhi = -1;
    for (int k = 0; k < 3; ++k) {
      const int p = m[opp[k][0]][opp[k][1]], q = m[opp[k][2]][opp[k][3]];
      double l2 = 0;
      for (int i = 0; i < d; ++i) {
        const double dx = F.xyz[(size_t)p * d + i] - F.xyz[(size_t)q * d + i];
        l2 += dx * dx;
      }
      const int lo = coord_cmp(F, p, q) <= 0 ? p : q, hi = lo == p ? q : p;
      bool better = best < 0 || l2 < bl;
      if (!better && l2 == bl) {
        const int c1 = coord_cmp(F, lo, blo);
        better = c1 < 0 || (c1 == 0 && coord_cmp(F, hi, bhi) < 0);
      }
      if (better) {
        best = k;
        bl = l2;
        blo = lo;
        bhi = hi;
      }
    }
    const int a = opp[best][0], b = opp[best][1], cc = opp[best][2], dd = opp[best][3];
    const int ring[4] = {m[a][cc], m[a][dd], m[b][dd], m[b][cc]};   // neighbours share an old vertex
    const int p = m[a][b], q = m[cc][dd];
    for (int i = 0; i < 4; ++i) put({p, q, ring[i], ring[(i + 1) & 3]});
  }
  return F;
}

// Z-order (Morton) key of a point: each coordinate scaled to the box [lo, hi]
// and quantised to 21 bits (d = 3) or 31 bits (d = 2), bits interleaved with
// the first coordinate lowest.
uint64_t morton_key(const double* x, int d, const double* lo, const double* hi) {
  const int bits = d == 3 ? 21 : 31;
  const double top = (double)((1ull << bits) - 1);
  uint64_t q[3] = {0, 0, 0};
  for (int i = 0; i < d; ++i) {
    const double w = hi[i] > lo[i] ? (x[i] - lo[i]) / (hi[i] - lo[i]) : 0.0;
    q[i] = (uint64_t)std::llround(std::min(std::max(w, 0.0), 1.0) * top);
  }
  uint64_t key = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int i = d - 1; i >= 0; --i) key = (key << 1) | ((q[i] >> b) & 1ull);
  return key;
}

// Boundary faces are faces of exactly one cell; their vertices are Dirichlet
// nodes.  The interior nodes are numbered along the Z-order curve of their
// coordinates (ties by node number), so that a node's matrix row gathers
// from nearby entries of a vector.
void number_interior(MeshLevel& L, const double* lo, const double* hi) {
  const int d = L.d, nv = d + 1;
  std::vector<std::array<int, 3>> faces;
  faces.reserve((size_t)L.cells() * nv);
  for (long long t = 0; t < L.cells(); ++t) {
    const int* c = &L.cell[(size_t)t * nv];
    for (int skip = 0; skip < nv; ++skip) {
      std::array<int, 3> f = {-1, -1, -1};
      int k = 0;
      for (int i = 0; i < nv; ++i)
        if (i != skip) f[k++] = c[i];
      std::sort(f.begin(), f.begin() + d);
      faces.push_back(f);
    }
  }
  std::sort(faces.begin(), faces.end());
  std::vector<char> bnd((size_t)L.nodes(), 0);
  for (size_t i = 0; i < faces.size();) {
    size_t j = i + 1;
    while (j < faces.size() && faces[j] == faces[i]) ++j;
    if (j - i == 1)
      for (int k = 0; k < d; ++k) bnd[(size_t)faces[i][k]] = 1;
    i = j;
  }
  std::vector<std::pair<uint64_t, int>> order;
  for (long long v = 0; v < L.nodes(); ++v)
    if (!bnd[(size_t)v]) order.push_back({morton_key(&L.xyz[(size_t)v * d], d, lo, hi), (int)v});
  std::sort(order.begin(), order.end());
  L.pos.assign((size_t)L.nodes(), -1);
  L.interior.clear();
  for (const auto& o : order) {
    L.pos[(size_t)o.second] = (int)L.interior.size();
    L.interior.push_back(o.second);
  }
}

// M_e = |T| (1 + delta_ij) / ((d+1)(d+2)), K_e = |T| G G^T with G the
// gradients of the barycentric coordinates (grad lambda_i = row i-1 of B^{-1},
// grad lambda_0 = minus their sum); interior rows and columns only.
void assemble(MeshLevel& L) {
  const int d = L.d, nv = d + 1;
  struct Ent { int r, c; double m, k; };
  std::vector<Ent> ent;
  ent.reserve((size_t)L.cells() * nv * nv);
  const double fact = d == 2 ? 2.0 : 6.0;
  for (long long t = 0; t < L.cells(); ++t) {
    const int* c = &L.cell[(size_t)t * nv];
    double Binv[9];
    const double vol = std::fabs(edge_matrix(L, c, Binv)) / fact;
    double G[4][3];
    for (int j = 0; j < d; ++j) {
      double s = 0;
      for (int i = 0; i < d; ++i) {
        G[i + 1][j] = Binv[i * d + j];
        s += Binv[i * d + j];
      }
      G[0][j] = -s;
    }
    const double mw = vol / ((d + 1) * (d + 2));
    for (int a = 0; a < nv; ++a) {
      const int ra = L.pos[(size_t)c[a]];
      if (ra < 0) continue;
      for (int b = 0; b < nv; ++b) {
        const int cb = L.pos[(size_t)c[b]];
        if (cb < 0) continue;
        double g = 0;
        for (int j = 0; j < d; ++j) g += G[a][j] * G[b][j];
        ent.push_back({ra, cb, mw * (a == b ? 2.0 : 1.0), vol * g});
      }
    }
  }
  std::sort(ent.begin(), ent.end(), [](const Ent& x, const Ent& y) { return x.r != y.r ? x.r < y.r : x.c < y.c; });
  const long long nx = L.nx();
  L.rowptr.assign((size_t)nx + 1, 0);
  L.col.clear();
  L.mval.clear();
  L.kval.clear();
  for (size_t i = 0; i < ent.size();) {
    size_t j = i;
    double m = 0, k = 0;
    while (j < ent.size() && ent[j].r == ent[i].r && ent[j].c == ent[i].c) {
      m += ent[j].m;
      k += ent[j].k;
      ++j;
    }
    L.col.push_back(ent[i].c);
    L.mval.push_back(m);
    L.kval.push_back(k);
    L.rowptr[(size_t)ent[i].r + 1] += 1;
    i = j;
  }
  for (long long r = 0; r < nx; ++r) L.rowptr[(size_t)r + 1] += L.rowptr[(size_t)r];
}

void finish(MeshLevel& L, const double* lo, const double* hi) {
  number_interior(L, lo, hi);
  assemble(L);
}

}  // namespace

int mesh_hierarchy(const st_mesh* m, int refinements, std::vector<MeshLevel>& out, std::string& err) {
  out.clear();
  if (!m || !m->coords || !m->cells) {
    err = "mesh: null pointer";
    return ST_EINVAL;
  }
  const int d = m->dim;
  if (d != 2 && d != 3) {
    err = "mesh: dim must be 2 or 3";
    return ST_EINVAL;
  }
  if (m->nnodes < d + 1 || m->ncells < 1) {
    err = "mesh: needs at least dim + 1 nodes and one cell";
    return ST_EINVAL;
  }
  if (refinements < 0 || refinements > 10) {
    err = "mesh: refinements must be in 0..10";
    return ST_EINVAL;
  }
  // sizes after the refinements: cells x 2^(d R), nodes below cells x (nodes per cell + edges)
  const double grow = std::pow(2.0, (double)d * refinements);
  const double cells_f = (double)m->ncells * grow;
  if (cells_f * (d + 1) > (double)std::numeric_limits<int>::max() ||
      (double)m->nnodes + cells_f * 6.0 > (double)std::numeric_limits<int>::max()) {
    err = "mesh: refined mesh exceeds 32-bit indices";
    return ST_ENOMEM;
  }
  MeshLevel L;
  L.d = d;
  L.xyz.assign(m->coords, m->coords + (size_t)m->nnodes * d);
  for (double v : L.xyz)
    if (!std::isfinite(v)) {
      err = "mesh: non-finite coordinate";
      return ST_EINVAL;
    }
  L.cell.assign(m->cells, m->cells + (size_t)m->ncells * (d + 1));
  for (int v : L.cell)
    if (v < 0 || v >= m->nnodes) {
      err = "mesh: cell vertex index out of range";
      return ST_EINVAL;
    }
  double scale = 0;
  for (double v : L.xyz) scale = std::max(scale, std::fabs(v));
  for (int t = 0; t < m->ncells; ++t) {
    const double det = edge_matrix(L, &L.cell[(size_t)t * (d + 1)], nullptr);
    if (!(std::fabs(det) > 1e-14 * std::pow(std::max(scale, 1e-300), d))) {
      err = "mesh: degenerate cell " + std::to_string(t);
      return ST_EINVAL;
    }
  }
  L.par.assign((size_t)m->nnodes * 2, -1);
  for (int t = 0; t < m->ncells; ++t)
    for (int a = 0; a <= d; ++a)
      for (int b = a + 1; b <= d; ++b) {
        const int p = L.cell[(size_t)t * (d + 1) + a], q = L.cell[(size_t)t * (d + 1) + b];
        double l2 = 0;
        for (int i = 0; i < d; ++i) {
          const double dx = L.xyz[(size_t)p * d + i] - L.xyz[(size_t)q * d + i];
          l2 += dx * dx;
        }
        L.longest_edge = std::max(L.longest_edge, std::sqrt(l2));
      }
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};   // bounding box of the coarse mesh
  for (int i = 0; i < d; ++i) {
    lo[i] = hi[i] = L.xyz[(size_t)i];
    for (long long v = 0; v < L.nodes(); ++v) {
      lo[i] = std::min(lo[i], L.xyz[(size_t)v * d + i]);
      hi[i] = std::max(hi[i], L.xyz[(size_t)v * d + i]);
    }
  }
  finish(L, lo, hi);
  out.push_back(std::move(L));
  for (int r = 0; r < refinements; ++r) {
    MeshLevel F = refine(out.back());
    F.longest_edge = 0.5 * out.back().longest_edge;
    finish(F, lo, hi);
    out.push_back(std::move(F));
  }
  return ST_OK;
}

void mesh_interpolation(const MeshLevel& c, const MeshLevel& f, std::vector<int>& p, std::vector<double>& w,
                        std::vector<int>& rrow, std::vector<int>& rcol) {
  const long long nf = f.nx(), nc = c.nx();
  p.assign((size_t)nf * 2, -1);
  w.assign((size_t)nf, 0.0);
  for (long long i = 0; i < nf; ++i) {
    const int v = f.interior[(size_t)i];
    const int a = f.par[(size_t)v * 2], b = f.par[(size_t)v * 2 + 1];
    if (a < 0) {   // an old node keeps its value
      p[(size_t)i * 2] = c.pos[(size_t)v];
      w[(size_t)i] = 1.0;
    } else {       // an edge node: mean of the edge's ends (boundary ends are zero)
      p[(size_t)i * 2] = c.pos[(size_t)a];
      p[(size_t)i * 2 + 1] = c.pos[(size_t)b];
      w[(size_t)i] = 0.5;
    }
  }
  rrow.assign((size_t)nc + 1, 0);
  for (long long i = 0; i < nf; ++i)
    for (int k = 0; k < 2; ++k)
      if (p[(size_t)i * 2 + k] >= 0) rrow[(size_t)p[(size_t)i * 2 + k] + 1] += 1;
  for (long long r = 0; r < nc; ++r) rrow[(size_t)r + 1] += rrow[(size_t)r];
  rcol.assign((size_t)rrow[(size_t)nc], 0);
  std::vector<int> fill(rrow.begin(), rrow.end() - 1);
  for (long long i = 0; i < nf; ++i)
    for (int k = 0; k < 2; ++k) {
      const int q = p[(size_t)i * 2 + k];
      if (q >= 0) rcol[(size_t)fill[(size_t)q]++] = (int)i;
    }
}

}  // namespace stmg

extern "C" int st_mesh_level(const st_mesh* coarse, int level, long long* nx, long long* nnz, double* points,
                             int* rowptr, int* col, double* mval, double* kval) {
  if (level < 0) return ST_EINVAL;
  std::vector<stmg::MeshLevel> L;
  std::string err;
  const int rc = stmg::mesh_hierarchy(coarse, level, L, err);
  if (rc != ST_OK) return rc;
  const stmg::MeshLevel& M = L.back();
  if (nx) *nx = M.nx();
  if (nnz) *nnz = (long long)M.col.size();
  if (points)
    for (long long i = 0; i < M.nx(); ++i)
      std::memcpy(points + (size_t)i * M.d, &M.xyz[(size_t)M.interior[(size_t)i] * M.d], sizeof(double) * M.d);
  if (rowptr) std::memcpy(rowptr, M.rowptr.data(), sizeof(int) * M.rowptr.size());
  if (col) std::memcpy(col, M.col.data(), sizeof(int) * M.col.size());
  if (mval) std::memcpy(mval, M.mval.data(), sizeof(double) * M.mval.size());
  if (kval) std::memcpy(kval, M.kval.data(), sizeof(double) * M.kval.size());
  return ST_OK;
}
