// Host-side mesh topology and dual-cell tables for the PMCHWT library.
//
// Built once per scatterer on the host (integer work, O(F log F)) and uploaded
// as structure-of-arrays tables; every integral is evaluated on the GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pmchwt {

// Primal triangulation with RWG edge structure.
//   Edge e = (lo, hi), lexicographic order.  T+ traverses lo -> hi.
//   Local basis a of triangle t sits on the edge opposite vertex a, with sign
//   +1 on T+ and -1 on T-; unit-flux RWG: s (x - P_a) / (2 A_t).
struct Topo {
  int nv = 0, F = 0, E = 0;
  std::vector<double> v;        // nv*3
  std::vector<int32_t> t;       // F*3
  std::vector<int32_t> edges;   // E*2
  std::vector<int32_t> tplus, tminus;
  std::vector<int32_t> t2e;     // F*3
  std::vector<int8_t> sgn;      // F*3
  std::vector<double> area;     // F
  std::vector<double> normal;   // F*3
};

bool build_topology(const double* v, int nv, const int32_t* t, int F, Topo& out, std::string& err);

// Barycentric refinement and Buffa-Christiansen functions, organised by dual
// cell.  The dual cell of primal vertex v is the ring of 2 N_v barycentric
// triangles that have v as a vertex (N_v = number of primal triangles at v).
// Barycentric vertex ids: primal vertex i -> i, midpoint of edge e -> nv + e,
// centroid of triangle t -> nv + E + t.  Children of parent (a, b, c):
// (a,m_ab,g) (m_ab,b,g) (b,m_bc,g) (m_bc,c,g) (c,m_ca,g) (m_ca,a,g).
//
// BC function of edge e = (v+, v-) restricted to a barycentric triangle is an
// RT0 field  alpha x - w  (div = 2 alpha).  Its outward fluxes follow the
// Buffa-Christiansen construction: in the cell of v+ the children t_1..t_2N
// are numbered around v+ starting next to the half edge v+ m_e; flux
// (k - N)/(2N) crosses from t_k to t_{k+1}; 1/2 leaves through each of the
// two edges m_e g shared with the cell of v-; the cell of v- is the mirror
// image with the signs reversed.
struct DualCells {
  int nbv = 0;                      // barycentric vertices
  std::vector<double> bv;           // nbv*3
  std::vector<int32_t> cell_ptr;    // nv+1, into ring
  std::vector<int32_t> ring;        // child triangle ids (parent*6 + j) in ring order
  std::vector<int32_t> child_vid;   // 6F*3 barycentric vertex ids of each child
  std::vector<int32_t> inc_ptr;     // nv+1, into inc_edges
  std::vector<int32_t> inc_edges;   // edges incident to v
  std::vector<int64_t> coef_ptr;    // nv+1, offsets (in 4-double records) of cell blocks
  std::vector<double> coef;         // per cell: N_v slots x 2N_v ring positions x (alpha, wx, wy, wz)
  std::vector<double> bbox;         // E*6, support bounding box of each BC function
  int max_valence = 0;
};

bool build_dual(const Topo& T, DualCells& D, std::string& err);

}  // namespace pmchwt
