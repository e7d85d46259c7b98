// Host-side mesh processing: element geometry, facet matching (periodic or bounded per box
// direction), boundary facets, canonical facet orientation, element classes ("types") with
// identical facet tables, and the reference tables the kernels read.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dgmesh {

struct Host {
  int dim = 0, k = 0, np = 0;
  int64_t E = 0;
  std::vector<double> X;          // [E][d+1][d] unwrapped vertex coordinates
  std::vector<double> jinv;       // [E][d][d]  (J^-1)_{row, col}
  std::vector<double> absdet;     // [E]
  std::vector<int32_t> nbr;       // [E][d+1]; boundary facet b is encoded as -1 - b
  std::vector<int32_t> nbr_facet; // [E][d+1]; -1 on boundary facets
  int64_t nbf = 0;                // boundary facets, numbered in (element, local facet) order
  std::vector<int64_t> bf_elem;   // [nbf]
  std::vector<int32_t> bf_facet;  // [nbf]
  std::vector<uint8_t> perm_own;  // [E][d+1] canonical-order permutation code, own side
  std::vector<uint8_t> perm_nbr;  // [E][d+1] same for the neighbour's facet
  double hmin = 0, volume = 0;
  // element classes
  std::vector<int32_t> type_of;   // [E]
  int ntypes = 0;
  std::vector<int32_t> type_tab;  // [ntypes][d+1]: (own table) | (nbr table << 16); the
                                  // neighbour table of a boundary facet is kBoundaryTable
  std::vector<int32_t> elem_tab;  // [E][d+1]: type_tab of each element's class (per-lane mode)
  bool lane_tables = false;       // 64-wide tiles in element order, facet tables per lane
  std::vector<int32_t> elem_list; // [ntiles*64], -1 padded (64-wide tiles, VALU kernels)
  std::vector<int32_t> tile_type; // [ntiles], -1 = empty tile
  int ntiles = 0;
  std::vector<int32_t> elem_list16; // [ntiles16*16] (16-wide tiles, matrix-core kernels)
  std::vector<int32_t> tile_type16;
  int ntiles16 = 0;
};

constexpr int kBoundaryTable = 0x7fff;

void build_tiles(const Host& H, int width, std::vector<int32_t>& elem_list,
                 std::vector<int32_t>& tile_type, int& ntiles, bool by_class = true);

// switch the 64-wide tiles to element order with per-lane facet tables (for meshes whose
// element classes leave the class-grouped tiles mostly empty)
void use_lane_tables(Host& H);

// returns empty string on success, else an error message; code set to a dg_status value
int build(int dim, int k, int64_t nvert, const double* xyz, int64_t nelem, const int64_t* elem,
          const double* period, Host& out, std::string& err);

void box_connectivity(int dim, int n, std::vector<double>& xyz, std::vector<int64_t>& elem);

// physical quadrature points of the boundary facets in canonical order: [nbf][nfq][d]
void boundary_points(const Host& H, std::vector<double>& out);

// Tables (FP64) for the kernels, concatenated:
//   Bv [nq][np]            phi_m at the volume points
//   Dv [nq][np][d]         w_q d phi_m / d xi_j at the volume points
//   Tr [(d+1)*P][nfq][np]  phi_m at the canonical facet points of local facet f with
//                          canonical permutation p (table index f*P + p, P = d!)
//   Lf [(d+1)*P][nfq][np]  facet weight times Tr
// and, apart, the basis values at the ns points of the collapsed rule exact to 3k-1 (the
// points of the speed reduction, independent of the volume rule): spd [ns][np].
struct Tables {
  int nq = 0, nfq = 0, nperm = 0, ns = 0;
  size_t off_bv = 0, off_dv = 0, off_tr = 0, off_lf = 0, total = 0;
  std::vector<double> data, spd;
};
void build_tables(int dim, int k, Tables& t);

int n_perm(int dim);
// the canonical vertex order of local facet f under permutation code p: local vertex ids
void canonical_vertices(int dim, int f, int p, int* out);

}  // namespace dgmesh
