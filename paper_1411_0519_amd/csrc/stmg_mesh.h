// Host-side P1 simplicial meshes for the numerical examples (Sec. 4): red
// refinement of a coarse triangle/tetrahedron mesh, boundary detection,
// interior numbering, P1 mass and stiffness matrices of the interior nodes and
// the nested interpolation between refinement levels.
#pragma once

#include <string>
#include <vector>

#include "st_mg.h"

namespace stmg {

struct MeshLevel {
  int d = 0;
  std::vector<double> xyz;       // node coordinates, nodes x d
  std::vector<int> cell;         // cells x (d + 1) node indices
  std::vector<int> par;          // 2 per node: the edge an edge node halves; -1, -1 for older nodes
  std::vector<int> pos;          // node -> interior index, -1 on the boundary
  std::vector<int> interior;     // interior index -> node
  std::vector<int> rowptr, col;  // CSR of the interior M_h / K_h (shared pattern, columns ascending)
  std::vector<double> mval, kval;
  double longest_edge = 0;
  long long nodes() const { return (long long)xyz.size() / d; }
  long long cells() const { return (long long)cell.size() / (d + 1); }
  long long nx() const { return (long long)interior.size(); }
};

// Levels 0 (the coarse mesh) .. refinements.  Returns ST_OK, ST_EINVAL (err
// says why) or ST_ENOMEM (sizes beyond 32-bit indices).
int mesh_hierarchy(const st_mesh* coarse, int refinements, std::vector<MeshLevel>& out, std::string& err);

// Interpolation from level c to its refinement f: fine interior node i takes
// w[i] * (e[p[2i]] + e[p[2i+1]]) over the parents that are >= 0 (w = 1 for an
// old node, 1/2 for an edge node).  rrow/rcol: the transpose as CSR over the
// coarse interior nodes (fine indices, ascending).
void mesh_interpolation(const MeshLevel& c, const MeshLevel& f, std::vector<int>& p, std::vector<double>& w,
                        std::vector<int>& rrow, std::vector<int>& rcol);

}  // namespace stmg
