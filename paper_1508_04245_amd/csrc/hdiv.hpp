// H(div)-conforming velocity space W_h on a 2D mesh (host side): BDM degrees of freedom,
// global numbering, orientation signs, and the reference dual basis the transfer kernels read.
//
// W_h (Sec. 2.2: element-wise [P^k]^2 fields with continuous normal components) carries the
// Brezzi-Douglas-Marini degrees of freedom, k >= 1:
//   facet    int_F (v . n_F) q_l(s) ds, l = 0..k, n_F the outward normal of the lower-numbered
//            element sharing F (of its element on a boundary facet), s in [0, 1] along F from
//            its lexicographically first vertex, q_l(s) = sqrt(2l+1) P_l(2s-1);
//   interior sign(det J) int_T v . (J^-T psi_r) dx, psi_r over the first-kind Nedelec space
//            N_{k-1} of the reference triangle: (x^a y^b, 0), (0, x^a y^b) for a+b <= k-2
//            (degree ascending, a descending), then (-y, x) x^a y^b for a+b = k-2.
// Global numbering: the k+1 dofs of each facet (facets in the order of their owner element,
// then local facet), then the k^2-1 interior dofs of each element.  A basis function restricted
// to element T is s * Piola_T(psi^_j) with the signed Piola map v = J v^ / det J, psi^_j the
// reference dual basis, and s = sign(det J) n-sign (l-th facet dof: times (-1)^l when the
// local parameter runs against the canonical one).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "mesh.hpp"

namespace dghdiv {

struct Host {
  int k = 0, np = 0, ndof = 0, nint = 0;   // ndof = (k+1)(k+2) local dofs = 2 np
  int64_t nfacet = 0, N = 0;                // global facets, global dofs
  // [E][3]: facet id << 2 | (facet sign s_f < 0) << 1 | (local parameter reversed)
  std::vector<int32_t> elem_facet;
  // [nfacet][2]: 3 element + local facet of the owner side, then of the other side or -1
  std::vector<int64_t> facet_elem;
  std::vector<double> table;                // [ndof][2][np]: psi^_j on the DG basis e_a phi_m
};

// 2D meshes only, k >= 1; returns 0 or an error code with err set
int build(const dgmesh::Host& H, Host& out, std::string& err);

// the reference dual basis, C[(a np + m) * ndof + j] (long double inverse of the moments)
void reference_dual(int k, std::vector<double>& table);

}  // namespace dghdiv
