// Host-side mesh processing and reference tables (see mesh.hpp).
#include "mesh.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <unordered_map>

#include "refelem.hpp"

namespace dgmesh {

int n_perm(int dim) { return dim == 2 ? 2 : 6; }

static const int kPerm2[2][2] = {{0, 1}, {1, 0}};
static const int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

void canonical_vertices(int dim, int f, int p, int* out) {
  int lv[3], c = 0;
  for (int a = 0; a <= dim; ++a)
    if (a != f) lv[c++] = a;
  for (int j = 0; j < dim; ++j) out[j] = lv[dim == 2 ? kPerm2[p][j] : kPerm3[p][j]];
}

// lexicographic "a < b" with tolerance
static bool lex_less(const double* a, const double* b, int d, double tol) {
  for (int c = 0; c < d; ++c) {
    if (a[c] < b[c] - tol) return true;
    if (a[c] > b[c] + tol) return false;
  }
  return false;
}

static int perm_code(int dim, const double* V /*[d][d] facet vertices in local order*/,
                     double tol) {
  const int np = n_perm(dim);
  for (int p = 0; p < np; ++p) {
    const int* o = dim == 2 ? kPerm2[p] : kPerm3[p];
    bool ok = true;
    for (int j = 0; j + 1 < dim && ok; ++j)
      ok = lex_less(V + o[j] * dim, V + o[j + 1] * dim, dim, tol);
    if (ok) return p;
  }
  return -1;
}

static void inv_det(int d, const double* J, double* Ji, double* det) {
  if (d == 2) {
    const double a = J[0], b = J[1], c = J[2], e = J[3];
    const double dt = a * e - b * c;
    *det = dt;
    Ji[0] = e / dt; Ji[1] = -b / dt; Ji[2] = -c / dt; Ji[3] = a / dt;
    return;
  }
  const double a = J[0], b = J[1], c = J[2], dd = J[3], e = J[4], f = J[5], g = J[6],
               h = J[7], i = J[8];
  const double A = e * i - f * h, B = -(dd * i - f * g), C = dd * h - e * g;
  const double dt = a * A + b * B + c * C;
  *det = dt;
  Ji[0] = A / dt; Ji[1] = -(b * i - c * h) / dt; Ji[2] = (b * f - c * e) / dt;
  Ji[3] = B / dt; Ji[4] = (a * i - c * g) / dt; Ji[5] = -(a * f - c * dd) / dt;
  Ji[6] = C / dt; Ji[7] = -(a * h - b * g) / dt; Ji[8] = (a * e - b * dd) / dt;
}

int build(int dim, int k, int64_t nvert, const double* xyz, int64_t nelem, const int64_t* elem,
          const double* period, Host& H, std::string& err) {
  const int d = dim, nf = d + 1;
  H = Host();
  H.dim = d; H.k = k; H.np = dgref::n_basis(d, k); H.E = nelem;
  H.X.resize((size_t)nelem * nf * d);
  H.jinv.resize((size_t)nelem * d * d);
  H.absdet.resize(nelem);
  double maxedge = 0.0;
  for (int64_t t = 0; t < nelem; ++t) {
    for (int a = 0; a < nf; ++a) {
      const int64_t v = elem[t * nf + a];
      if (v < 0 || v >= nvert) { err = "vertex id out of range"; return -1; }
      for (int j = 0; j < d; ++j) H.X[(t * nf + a) * d + j] = xyz[v * d + j];
    }
    double J[9];
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j)
        J[i * d + j] = H.X[(t * nf + j + 1) * d + i] - H.X[(t * nf) * d + i];
    for (int j = 0; j < d; ++j) {
      double s = 0;
      for (int i = 0; i < d; ++i) s += J[i * d + j] * J[i * d + j];
      maxedge = std::max(maxedge, std::sqrt(s));
    }
    double det;
    inv_det(d, J, &H.jinv[t * d * d], &det);
    H.absdet[t] = std::fabs(det);
  }
  // degeneracy check relative to the element's own edge scale
  for (int64_t t = 0; t < nelem; ++t) {
    double h = 0;
    for (int a = 1; a < nf; ++a) {
      double s = 0;
      for (int j = 0; j < d; ++j) {
        const double v = H.X[(t * nf + a) * d + j] - H.X[(t * nf) * d + j];
        s += v * v;
      }
      h = std::max(h, std::sqrt(s));
    }
    if (!(H.absdet[t] > 1e-12 * std::pow(h, d))) { err = "degenerate element"; return -6; }
  }
  // facets: centroid, measure, canonical permutation
  const size_t NFT = (size_t)nelem * nf;
  std::vector<double> cen(NFT * d);
  std::vector<uint8_t> perm(NFT);
  double minmeas = 1e300;
  for (int64_t t = 0; t < nelem; ++t) {
    const double tol = 1e-10 * maxedge;
    for (int f = 0; f < nf; ++f) {
      double V[9];
      int c = 0;
      for (int a = 0; a < nf; ++a) {
        if (a == f) continue;
        for (int j = 0; j < d; ++j) V[c * d + j] = H.X[(t * nf + a) * d + j];
        ++c;
      }
      for (int j = 0; j < d; ++j) {
        double s = 0;
        for (int a = 0; a < d; ++a) s += V[a * d + j];
        cen[(t * nf + f) * d + j] = s / d;
      }
      double meas;
      if (d == 2) {
        meas = std::hypot(V[2] - V[0], V[3] - V[1]);
      } else {
        const double u0 = V[3] - V[0], u1 = V[4] - V[1], u2 = V[5] - V[2];
        const double w0 = V[6] - V[0], w1 = V[7] - V[1], w2 = V[8] - V[2];
        const double cx = u1 * w2 - u2 * w1, cy = u2 * w0 - u0 * w2, cz = u0 * w1 - u1 * w0;
        meas = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
      }
      minmeas = std::min(minmeas, meas);
      const int p = perm_code(d, V, tol);
      if (p < 0) { err = "facet with coincident vertices"; return -6; }
      perm[t * nf + f] = (uint8_t)p;
    }
  }
  H.hmin = d == 2 ? minmeas : std::sqrt(minmeas);
  double vol = 0;
  for (int64_t t = 0; t < nelem; ++t) vol += H.absdet[t] / (d == 2 ? 2.0 : 6.0);
  H.volume = vol;
  // matching of centroids via a hash grid: periodic directions (period > 0) wrap, bounded
  // directions (period <= 0) do not, and facets left unmatched there are boundary facets
  double L[3] = {0, 0, 0}, lo[3] = {0, 0, 0};
  bool wrap[3] = {false, false, false}, any_bounded = false;
  if (!period) { err = "period is required (entries <= 0 mark bounded directions)"; return -1; }
  for (int j = 0; j < d; ++j) {
    wrap[j] = period[j] > 0;
    any_bounded |= !wrap[j];
    if (wrap[j]) {
      L[j] = period[j];
    } else {
      double mn = 1e300, mx = -1e300;
      for (size_t i = 0; i < NFT; ++i) { mn = std::min(mn, cen[i * d + j]); mx = std::max(mx, cen[i * d + j]); }
      lo[j] = mn;
      L[j] = (mx - mn) + 4.0 * H.hmin;  // extent of the grid only: never wrapped
    }
  }
  const double quantum = 1e-3 * H.hmin;
  const double mtol = 1e-7 * H.hmin;
  int64_t ncell[3];
  for (int j = 0; j < d; ++j) ncell[j] = (int64_t)std::ceil(L[j] / quantum) + 3;
  std::vector<double> wc(NFT * d);
  std::vector<int64_t> cell(NFT * d);
  for (size_t i = 0; i < NFT; ++i)
    for (int j = 0; j < d; ++j) {
      double v = cen[i * d + j];
      if (wrap[j]) {
        v -= L[j] * std::floor(v / L[j]);
        if (v > L[j] - 0.5 * quantum) v -= L[j];
      } else {
        v -= lo[j];
      }
      wc[i * d + j] = v;
      cell[i * d + j] = (int64_t)std::floor(v / quantum);
    }
  auto key = [&](const int64_t* c) {
    int64_t kk = 0;
    for (int j = 0; j < d; ++j) {
      int64_t cj = ((c[j] % ncell[j]) + ncell[j]) % ncell[j];
      kk = kk * ncell[j] + cj;
    }
    return kk;
  };
  std::unordered_map<int64_t, std::vector<int64_t>> grid;
  grid.reserve(NFT * 2);
  for (size_t i = 0; i < NFT; ++i) grid[key(&cell[i * d])].push_back((int64_t)i);
  H.nbr.assign(NFT, -1);
  H.nbr_facet.assign(NFT, -1);
  for (size_t i = 0; i < NFT; ++i) {
    int64_t found = -1;
    int nfound = 0;
    const int span = d == 2 ? 9 : 27;
    for (int s = 0; s < span; ++s) {
      int64_t c[3];
      int ss = s;
      for (int j = 0; j < d; ++j) { c[j] = cell[i * d + j] + (ss % 3) - 1; ss /= 3; }
      auto it = grid.find(key(c));
      if (it == grid.end()) continue;
      for (int64_t o : it->second) {
        if ((size_t)o == i || o / nf == (int64_t)(i / nf)) continue;
        double dist2 = 0;
        for (int j = 0; j < d; ++j) {
          double dd = wc[i * d + j] - wc[o * d + j];
          if (wrap[j]) dd -= L[j] * std::nearbyint(dd / L[j]);
          dist2 += dd * dd;
        }
        if (dist2 < mtol * mtol) {
          if (o != found) { found = o; ++nfound; }
        }
      }
    }
    if (nfound > 1) { err = "non-manifold facet"; return -6; }
    if (nfound == 0) {
      if (!any_bounded) { err = "unmatched facet"; return -6; }
      continue;  // a boundary facet, numbered below
    }
    H.nbr[i] = (int32_t)(found / nf);
    H.nbr_facet[i] = (int32_t)(found % nf);
  }
  for (size_t i = 0; i < NFT; ++i) {
    if (H.nbr[i] < 0) continue;
    const size_t o = (size_t)H.nbr[i] * nf + H.nbr_facet[i];
    if ((size_t)H.nbr[o] * nf + H.nbr_facet[o] != i) { err = "non-manifold facet"; return -6; }
  }
  for (size_t i = 0; i < NFT; ++i) {
    if (H.nbr[i] >= 0) continue;
    H.nbr[i] = (int32_t)(-1 - H.nbf);
    H.bf_elem.push_back((int64_t)(i / nf));
    H.bf_facet.push_back((int32_t)(i % nf));
    ++H.nbf;
  }
  H.perm_own = perm;
  H.perm_nbr.resize(NFT);
  for (size_t i = 0; i < NFT; ++i)
    H.perm_nbr[i] = H.nbr[i] < 0 ? 0 : perm[(size_t)H.nbr[i] * nf + H.nbr_facet[i]];
  // element classes: identical (own table, neighbour table) for every local facet
  const int P = n_perm(d);
  std::map<int64_t, int> type_ids;
  std::vector<int64_t> type_keys;
  H.type_of.resize(nelem);
  for (int64_t t = 0; t < nelem; ++t) {
    int64_t kk = 0;
    for (int f = 0; f < nf; ++f) {
      const size_t i = t * nf + f;
      const int own = f * P + perm[i];
      const int nb = H.nbr[i] < 0 ? 31 : H.nbr_facet[i] * P + H.perm_nbr[i];
      kk = (kk << 10) | (own << 5) | nb;
    }
    auto it = type_ids.find(kk);
    int id;
    if (it == type_ids.end()) {
      id = (int)type_keys.size();
      type_ids[kk] = id;
      type_keys.push_back(kk);
    } else {
      id = it->second;
    }
    H.type_of[t] = id;
  }
  H.ntypes = (int)type_keys.size();
  H.type_tab.resize((size_t)H.ntypes * nf);
  for (int ty = 0; ty < H.ntypes; ++ty) {
    int64_t kk = type_keys[ty];
    for (int f = nf - 1; f >= 0; --f) {
      const int nb = (int)(kk & 31), own = (int)((kk >> 5) & 31);
      kk >>= 10;
      H.type_tab[ty * nf + f] = own | ((nb == 31 ? kBoundaryTable : nb) << 16);
    }
  }
  build_tiles(H, 64, H.elem_list, H.tile_type, H.ntiles);
  build_tiles(H, 16, H.elem_list16, H.tile_type16, H.ntiles16);
  return 0;
}

// Processing order of the blocks of a 3D mesh: eight groups, by the band of the block's
// centroid in y (eight bands), one group per XCD under the kernels' block remap (XCD x works
// on the x-th eighth of the blocks); inside a group the blocks go by their lowest vertex z
// (planes of elements), then in element order.  A group's plane is then small (a band of
// y-rows), so the neighbours across the next plane are read within a few MiB of the XCD's
// L2 traffic and are still there.  The results do not depend on this order (every element is
// computed alone).  2D meshes, and DGCONV_BLOCK_ORDER=0, keep the element order.
static std::vector<int64_t> block_order(const Host& H, int64_t bsz, int64_t nblk) {
  std::vector<int64_t> ord(nblk);
  for (int64_t b = 0; b < nblk; ++b) ord[b] = b;
  const char* env = std::getenv("DGCONV_BLOCK_ORDER");
  if (H.dim != 3 || nblk < 8 || (env && std::string(env) == "0")) return ord;
  const int nv = 4;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (size_t i = 0; i < H.X.size(); ++i) {
    lo[i % 3] = std::min(lo[i % 3], H.X[i]);
    hi[i % 3] = std::max(hi[i % 3], H.X[i]);
  }
  std::vector<int> grp(nblk);
  std::vector<double> zkey(nblk);
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t t0 = b * bsz, t1 = std::min<int64_t>(H.E, t0 + bsz);
    double cy = 0, zmin = 1e300;
    for (int64_t t = t0; t < t1; ++t)
      for (int v = 0; v < nv; ++v) {
        const double* x = &H.X[(t * nv + v) * 3];
        cy += x[1];
        zmin = std::min(zmin, x[2]);
      }
    cy /= (double)(t1 - t0) * nv;
    grp[b] = std::min(7, std::max(0, (int)(8.0 * (cy - lo[1]) / (hi[1] - lo[1]))));
    zkey[b] = zmin;
  }
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    return grp[a] != grp[b] ? grp[a] < grp[b] : zkey[a] < zkey[b];
  });
  return ord;
}

// Tiles of `width` elements: the mesh is cut into blocks of 4*width consecutive elements (one
// workgroup of 4 wavefronts each, taken in block_order); inside a block the elements are
// grouped by class into tiles, and the block's tile count is padded to a multiple of 4 with
// empty tiles (class -1), so every tile of a workgroup covers the same contiguous range of the
// state arrays.
void build_tiles(const Host& H, int width, std::vector<int32_t>& elem_list,
                 std::vector<int32_t>& tile_type, int& ntiles, bool by_class) {
  elem_list.clear();
  tile_type.clear();
  const int64_t bsz = 4 * width;
  const int64_t nblk = (H.E + bsz - 1) / bsz;
  const std::vector<int64_t> ord = block_order(H, bsz, nblk);
  for (int64_t bi = 0; bi < nblk; ++bi) {
    const int64_t b0 = ord[bi] * bsz;
    const int64_t b1 = std::min<int64_t>(H.E, b0 + bsz);
    std::map<int, std::vector<int32_t>> by_type;
    for (int64_t t = b0; t < b1; ++t) by_type[by_class ? H.type_of[t] : 0].push_back((int32_t)t);
    int ntile_block = 0;
    for (auto& kv : by_type) {
      const auto& mm = kv.second;
      for (size_t s0 = 0; s0 < mm.size(); s0 += width) {
        for (size_t l = 0; l < (size_t)width; ++l)
          elem_list.push_back(s0 + l < mm.size() ? mm[s0 + l] : -1);
        tile_type.push_back(kv.first);
        ++ntile_block;
      }
    }
    while (ntile_block % 4) {
      for (int l = 0; l < width; ++l) elem_list.push_back(-1);
      tile_type.push_back(-1);
      ++ntile_block;
    }
  }
  ntiles = (int)tile_type.size();
}

void use_lane_tables(Host& H) {
  const int nf = H.dim + 1;
  H.elem_tab.resize((size_t)H.E * nf);
  for (int64_t t = 0; t < H.E; ++t)
    for (int f = 0; f < nf; ++f) H.elem_tab[t * nf + f] = H.type_tab[(size_t)H.type_of[t] * nf + f];
  build_tiles(H, 64, H.elem_list, H.tile_type, H.ntiles, false);
  H.lane_tables = true;
}

void box_connectivity(int dim, int n, std::vector<double>& xyz, std::vector<int64_t>& elem) {
  const int n1 = n + 1;
  xyz.clear(); elem.clear();
  if (dim == 2) {
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i) { xyz.push_back((double)i / n); xyz.push_back((double)j / n); }
    auto V = [&](int i, int j) { return (int64_t)(j * n1 + i); };
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const int64_t v00 = V(i, j), v10 = V(i + 1, j), v11 = V(i + 1, j + 1), v01 = V(i, j + 1);
        elem.insert(elem.end(), {v00, v10, v11});
        elem.insert(elem.end(), {v11, v01, v00});
      }
    return;
  }
  for (int l = 0; l < n1; ++l)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i) {
        xyz.push_back((double)i / n); xyz.push_back((double)j / n); xyz.push_back((double)l / n);
      }
  auto V = [&](int i, int j, int l) { return (int64_t)((l * n1 + j) * n1 + i); };
  for (int l = 0; l < n; ++l)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        for (int p = 0; p < 6; ++p) {
          int e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
          e0[kPerm3[p][0]] = 1;
          e1[kPerm3[p][0]] = 1;
          e1[kPerm3[p][1]] = 1;
          elem.push_back(V(i, j, l));
          elem.push_back(V(i + e0[0], j + e0[1], l + e0[2]));
          elem.push_back(V(i + e1[0], j + e1[1], l + e1[2]));
          elem.push_back(V(i + 1, j + 1, l + 1));
        }
}

void boundary_points(const Host& H, std::vector<double>& out) {
  using dgref::real;
  const int d = H.dim, nf = d + 1;
  std::vector<real> fp, fw;
  dgref::operator_facet_rule<real>(d, H.k, fp, fw);
  const int nfq = (int)fw.size();
  out.assign((size_t)H.nbf * nfq * d, 0.0);
  for (int64_t b = 0; b < H.nbf; ++b) {
    const int64_t t = H.bf_elem[b];
    const int f = H.bf_facet[b];
    int cv[3];
    canonical_vertices(d, f, H.perm_own[t * nf + f], cv);
    const double* X = &H.X[(size_t)t * nf * d];
    for (int q = 0; q < nfq; ++q)
      for (int j = 0; j < d; ++j) {
        real x = X[cv[0] * d + j];
        for (int c = 1; c < d; ++c)
          x += fp[q * (d - 1) + (c - 1)] * ((real)X[cv[c] * d + j] - (real)X[cv[0] * d + j]);
        out[((size_t)b * nfq + q) * d + j] = (double)x;
      }
  }
}

void build_tables(int dim, int k, Tables& T) {
  using dgref::real;
  const int d = dim, np = dgref::n_basis(d, k);
  std::vector<real> vp, vw, fp, fw;
  dgref::volume_rule<real>(d, k, vp, vw);
  dgref::operator_facet_rule<real>(d, k, fp, fw);
  T.nq = (int)vw.size();
  T.nfq = (int)fw.size();
  T.nperm = n_perm(d);
  const int ntab = (d + 1) * T.nperm;
  T.off_bv = 0;
  T.off_dv = T.off_bv + (size_t)T.nq * np;
  T.off_tr = T.off_dv + (size_t)T.nq * np * d;
  T.off_lf = T.off_tr + (size_t)ntab * T.nfq * np;
  T.total = T.off_lf + (size_t)ntab * T.nfq * np;
  T.data.assign(T.total, 0.0);
  std::vector<real> val(np), grad(np * d);
  for (int q = 0; q < T.nq; ++q) {
    dgref::eval_basis_t<real>(d, k, &vp[q * d], val.data(), grad.data());
    for (int m = 0; m < np; ++m) {
      T.data[T.off_bv + q * np + m] = (double)val[m];
      for (int j = 0; j < d; ++j)
        T.data[T.off_dv + (q * np + m) * d + j] = (double)(vw[q] * grad[m * d + j]);
    }
  }
  {
    std::vector<real> sp, sw;
    dgref::collapsed_rule<real>(d, dgref::vol_points_1d(k), sp, sw);
    T.ns = (int)sw.size();
    T.spd.assign((size_t)T.ns * np, 0.0);
    for (int q = 0; q < T.ns; ++q) {
      dgref::eval_basis_t<real>(d, k, &sp[q * d], val.data(), nullptr);
      for (int m = 0; m < np; ++m) T.spd[(size_t)q * np + m] = (double)val[m];
    }
  }
  const real vref[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int f = 0; f <= d; ++f)
    for (int p = 0; p < T.nperm; ++p) {
      int cv[3];
      canonical_vertices(d, f, p, cv);
      const int tab = f * T.nperm + p;
      for (int q = 0; q < T.nfq; ++q) {
        real xi[3];
        for (int j = 0; j < d; ++j) {
          xi[j] = vref[cv[0]][j];
          for (int c = 1; c < d; ++c)
            xi[j] += fp[q * (d - 1) + (c - 1)] * (vref[cv[c]][j] - vref[cv[0]][j]);
        }
        dgref::eval_basis_t<real>(d, k, xi, val.data(), nullptr);
        for (int m = 0; m < np; ++m) {
          T.data[T.off_tr + ((size_t)tab * T.nfq + q) * np + m] = (double)val[m];
          T.data[T.off_lf + ((size_t)tab * T.nfq + q) * np + m] = (double)(fw[q] * val[m]);
        }
      }
    }
}

}  // namespace dgmesh
