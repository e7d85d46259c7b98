// H(div)-conforming velocity space W_h on a 2D or 3D mesh (host side): BDM degrees of
// freedom, global numbering, orientation data, and the reference tables the transfer kernels
// read.
//
// W_h (Sec. 2.2: element-wise [P^k]^d fields with continuous normal components) carries the
// Brezzi-Douglas-Marini degrees of freedom, k >= 1:
//   facet    int_F (v . n_F) q_l ds over an L2-orthonormal basis q_l of P^k(F) in the facet's
//            canonical parameter (its vertices in the mesh's lexicographic order, A + s (B - A)
//            [+ t (C - A)]), n_F the outward normal of the lower-numbered element sharing F (of
//            its element on a boundary facet); 2D: q_l(s) = sqrt(2l+1) P_l(2s-1), l = 0..k;
//            3D: q_l(s, t) = phi^_l(s, t) / sqrt(2), the DG basis of the reference triangle;
//   interior sign(det J) int_T v . (J^-T psi_r) dx, psi_r over the first-kind Nedelec space
//            N_{k-1} of the reference simplex: e_i m for the monomials m of degree <= k-2,
//            then the rotations of the monomials of degree k-2 ((-y, x) m in 2D; x ^ (e_i m) in
//            3D, without i = 0 when x divides m); monomials by degree, a descending, then b
//            descending, and i ascending for each.
// Global numbering: the dofs of each facet (facets in the order of their owner element, then
// local facet), then the interior dofs of each element.  A basis function restricted to
// element T is Piola_T(sum_j P_jJ psi^_j) with the signed Piola map v = J v^ / det J, psi^_j
// the reference dual basis (facet moments in each local facet's ascending-vertex parameter),
// and P the local map: on the dofs of local facet f, sign(det J) times the normal sign times
// the change of facet parameter Q (2D: (-1)^l when the local parameter runs against the
// canonical one; 3D: one of six orthogonal matrices), the identity on the interior dofs.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "mesh.hpp"

namespace dghdiv {

struct Host {
  int dim = 0, k = 0, np = 0, ndof = 0, nfd = 0, nint = 0;  // ndof = dim np local dofs
  int64_t nfacet = 0, N = 0;                // global facets, global dofs
  // [E][dim+1]: 2D: facet id << 2 | (facet sign s_f < 0) << 1 | (local parameter reversed);
  //             3D: facet id << 4 | (facet sign s_f < 0) << 3 | facet permutation code (0..5)
  std::vector<int32_t> elem_facet;
  // [nfacet][2]: (dim+1) element + local facet of the owner side, then of the other side or -1
  std::vector<int64_t> facet_elem;
  // [ndof][dim][np]: psi^_j on the DG basis e_a phi_m; in 3D followed by the six facet
  // parameter changes [6][nfd][nfd] (row l: local basis function, column i: canonical)
  std::vector<double> table;
};

// dim 2 or 3, k >= 1; returns 0 or an error code with err set
int build(const dgmesh::Host& H, Host& out, std::string& err);

// the reference dual basis, table[j * ndof + a np + m] (long double inverse of the moments)
void reference_dual(int dim, int k, std::vector<double>& table);

// the facet parameter changes of 3D facets, table[(p nfd + l) nfd + i]: q_l in the local
// (ascending) parameter = sum_i Q_li q_i in the canonical one, for permutation code p
void orientation_tables(int k, std::vector<double>& table);

inline int facet_dofs(int dim, int k) { return dim == 2 ? k + 1 : (k + 1) * (k + 2) / 2; }

}  // namespace dghdiv
