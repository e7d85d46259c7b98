// Transfer operators between the H(div) space W_h and the DG space V_h on 2D and 3D meshes
// (Sec. 2.4): I = (M^V)^-1 M^{U,V} (the DG coefficients of a W_h field) and its transpose
// I^T (a functional on V_h, given by its values on the DG basis, to one on W_h).
//
// On element T a W_h field is Piola(sum_j (P u_T)_j psi^_j), P the local map (facet signs and
// parameter changes), so with the signed Piola map v = J v^ / det J its DG coefficients are
//   c[i][m] = sum_a (J / det J)_ia ref[a][m],   ref[a][m] = sum_j (P u_T)_j C_j[a][m],
// and J / det J is the adjugate of J^-1, which the mesh already stores.  One lane per element.
// I reads the reference dual basis C (ndof x d x np doubles) through scalar loads; the local
// pass of I^T reads it from LDS where the tables fit; the 3D facet parameter changes sit in
// LDS.  The transpose runs in two passes: every element writes the contributions
// P^T (C^T G) of its local dofs (G = adj(J^-1)^T F), then every global dof adds its one
// (interior, boundary facet) or two (interior facet) contributions in a fixed order, so the
// result is deterministic and needs no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace {

using dgi::fail;

template <int D, int K>
struct HShape {
  static constexpr int NP = D == 2 ? (K + 1) * (K + 2) / 2 : (K + 1) * (K + 2) * (K + 3) / 6;
  static constexpr int ND = D * NP;
  static constexpr int NFD = D == 2 ? K + 1 : (K + 1) * (K + 2) / 2;
  static constexpr int NI = ND - (D + 1) * NFD;
  static constexpr int NQ = D == 3 ? 6 * NFD * NFD : 0;  // facet parameter changes (3D)
  static constexpr int TAB = ND * ND + NQ;
};

typedef const double __attribute__((address_space(4)))* cdptr;

// The reference dual basis is read with wave-uniform indices: scalar loads into SGPRs, which
// the FMAs take as operands (an LDS copy would cost LDS bandwidth per lane and was slower).
// The 3D facet parameter changes are read per lane (each element has its own facet
// orientations) and are staged in LDS; all threads of the block take part.  Returns the LDS
// copy of the parameter changes (3D) or nullptr.
template <int D, int K>
__device__ __forceinline__ const double* stage_orientations(const double* tab) {
  using S = HShape<D, K>;
  if constexpr (S::NQ > 0) {
    __shared__ double sq[S::NQ > 0 ? S::NQ : 1];
    for (int i = threadIdx.x; i < S::NQ; i += 256) sq[i] = tab[S::ND * S::ND + i];
    __syncthreads();
    return sq;
  } else {
    return nullptr;
  }
}

// entry i of the reference dual basis (wave-uniform i)
__device__ __forceinline__ double dual_entry(const double* tab, int i) { return ((cdptr)tab)[i]; }

// The transpose's local pass reads the dual basis column by column into short FMA chains;
// there the whole table block staged in LDS (when it fits in 64 KiB) is faster than scalar
// loads (3D P3: 67 against 107 us per pass).  Returns the LDS copy of the table block, or
// (tables beyond 64 KiB) that of the parameter changes alone.
template <int D, int K>
__device__ __forceinline__ const double* stage_all(const double* tab) {
  using S = HShape<D, K>;
  if constexpr (S::TAB * 8 <= 65536) {
    __shared__ double st[S::TAB * 8 <= 65536 ? S::TAB : 1];
    for (int i = threadIdx.x; i < S::TAB; i += 256) st[i] = tab[i];
    __syncthreads();
    return st;
  } else {
    return stage_orientations<D, K>(tab);
  }
}

// facet code of an element's local facet: global facet id, facet sign, 3D permutation code
template <int D>
struct FacetCode {
  int64_t id;
  double sf;  // sign(det J) times the normal sign
  int perm;   // 2D: 1 = local parameter reversed; 3D: permutation code 0..5
  __device__ explicit FacetCode(int c) {
    if constexpr (D == 2) {
      id = c >> 2; sf = (c & 2) ? -1.0 : 1.0; perm = c & 1;
    } else {
      id = c >> 4; sf = (c & 8) ? -1.0 : 1.0; perm = c & 7;
    }
  }
};

// adj(J^-1) = J / det J from the stored J^-1 (row-major)
template <int D>
__device__ __forceinline__ void adjugate(const double* m, double (&A)[D][D]) {
  if constexpr (D == 2) {
    A[0][0] = m[3]; A[0][1] = -m[1]; A[1][0] = -m[2]; A[1][1] = m[0];
  } else {
    A[0][0] = m[4] * m[8] - m[5] * m[7];
    A[0][1] = m[2] * m[7] - m[1] * m[8];
    A[0][2] = m[1] * m[5] - m[2] * m[4];
    A[1][0] = m[5] * m[6] - m[3] * m[8];
    A[1][1] = m[0] * m[8] - m[2] * m[6];
    A[1][2] = m[2] * m[3] - m[0] * m[5];
    A[2][0] = m[3] * m[7] - m[4] * m[6];
    A[2][1] = m[1] * m[6] - m[0] * m[7];
    A[2][2] = m[0] * m[4] - m[1] * m[3];
  }
}

template <int D, int K>
__global__ void __launch_bounds__(256) to_dg_kernel(int64_t E, int64_t nfd, const double* u,
                                                    const int* hf, const double* jinv,
                                                    const double* tab, double* out) {
  using S = HShape<D, K>;
  const double* sq = stage_orientations<D, K>(tab);
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= E) return;
  double ref[D][S::NP];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int m = 0; m < S::NP; ++m) ref[a][m] = 0.0;
  auto accumulate = [&](int j, double uj) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int m = 0; m < S::NP; ++m)
        ref[a][m] = fma(uj, dual_entry(tab, (j * D + a) * S::NP + m), ref[a][m]);
  };
  // facet dofs in local form (reference dof order), then the interior dofs
#pragma unroll
  for (int f = 0; f <= D; ++f) {
    const FacetCode<D> fc(hf[t * (D + 1) + f]);
    const double* uf = u + fc.id * S::NFD;
    if constexpr (D == 2) {
      const double so = fc.perm ? -fc.sf : fc.sf;  // odd l under a reversed parameter
#pragma unroll 1
      for (int l = 0; l < S::NFD; ++l) accumulate(f * S::NFD + l, ((l & 1) ? so : fc.sf) * uf[l]);
    } else {
      double ug[S::NFD];
#pragma unroll
      for (int i = 0; i < S::NFD; ++i) ug[i] = uf[i];
      const double* Q = sq + fc.perm * S::NFD * S::NFD;
#pragma unroll 1
      for (int l = 0; l < S::NFD; ++l) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < S::NFD; ++i) v = fma(Q[l * S::NFD + i], ug[i], v);
        accumulate(f * S::NFD + l, fc.sf * v);
      }
    }
  }
  const double* ui = u + nfd + t * S::NI;
#pragma unroll 1
  for (int r = 0; r < S::NI; ++r) accumulate((D + 1) * S::NFD + r, ui[r]);
  double A[D][D];
  adjugate<D>(jinv + t * D * D, A);
  double* o = out + t * S::ND;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int m = 0; m < S::NP; ++m) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) v = fma(A[i][a], ref[a][m], v);
      o[i * S::NP + m] = v;
    }
}

template <int D, int K>
__global__ void __launch_bounds__(256) transpose_local_kernel(int64_t E, const double* F,
                                                              const int* hf, const double* jinv,
                                                              const double* tab, double* loc) {
  using S = HShape<D, K>;
  // st: the table block (dual basis then parameter changes) in LDS where it fits; sq: the
  // parameter changes
  constexpr bool LDS = S::TAB * 8 <= 65536;
  const double* st = stage_all<D, K>(tab);
  const double* sq = LDS ? st + S::ND * S::ND : st;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= E) return;
  double A[D][D];
  adjugate<D>(jinv + t * D * D, A);
  const double* f = F + t * S::ND;
  double G[D][S::NP];  // G[a][m] = sum_i A[i][a] F[i][m]
#pragma unroll
  for (int m = 0; m < S::NP; ++m) {
    double fi[D];
#pragma unroll
    for (int i = 0; i < D; ++i) fi[i] = f[i * S::NP + m];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) v = fma(A[i][a], fi[i], v);
      G[a][m] = v;
    }
  }
  double* o = loc + t * S::ND;
  auto contract = [&](int j) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int m = 0; m < S::NP; ++m)
        acc = fma(LDS ? st[(j * D + a) * S::NP + m] : dual_entry(tab, (j * D + a) * S::NP + m),
                  G[a][m], acc);
    return acc;
  };
#pragma unroll
  for (int fcn = 0; fcn <= D; ++fcn) {
    const FacetCode<D> fc(hf[t * (D + 1) + fcn]);
    if constexpr (D == 2) {
      const double so = fc.perm ? -fc.sf : fc.sf;  // odd l under a reversed parameter
#pragma unroll 1
      for (int l = 0; l < S::NFD; ++l) {
        const int j = fcn * S::NFD + l;
        o[j] = ((l & 1) ? so : fc.sf) * contract(j);
      }
    } else {
      // local values c_l, then the canonical contributions sf sum_l Q_li c_l
      double cl[S::NFD];
#pragma unroll
      for (int l = 0; l < S::NFD; ++l) cl[l] = contract(fcn * S::NFD + l);
      const double* Q = sq + fc.perm * S::NFD * S::NFD;
#pragma unroll 1
      for (int i = 0; i < S::NFD; ++i) {
        double v = 0.0;
#pragma unroll
        for (int l = 0; l < S::NFD; ++l) v = fma(Q[l * S::NFD + i], cl[l], v);
        o[fcn * S::NFD + i] = fc.sf * v;
      }
    }
  }
#pragma unroll 1
  for (int j = (D + 1) * S::NFD; j < S::ND; ++j) o[j] = contract(j);
}

template <int D, int K>
__global__ void __launch_bounds__(256) transpose_gather_kernel(int64_t N, int64_t nfd,
                                                               const int64_t* fe,
                                                               const double* loc, double* out) {
  using S = HShape<D, K>;
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (d >= N) return;
  if (d < nfd) {
    const int64_t fc = d / S::NFD, l = d % S::NFD;
    const int64_t s0 = fe[2 * fc], s1 = fe[2 * fc + 1];
    double v = loc[(s0 / (D + 1)) * S::ND + (s0 % (D + 1)) * S::NFD + l];
    if (s1 >= 0) v += loc[(s1 / (D + 1)) * S::ND + (s1 % (D + 1)) * S::NFD + l];
    out[d] = v;
  } else {
    const int64_t t = (d - nfd) / S::NI, r = (d - nfd) % S::NI;
    out[d] = loc[t * S::ND + (D + 1) * S::NFD + r];
  }
}

template <typename T>
dg_status upload(const std::vector<T>& v, T** d) {
  HIP_TRY(hipMalloc((void**)d, v.size() * sizeof(T) + 16));
  HIP_TRY(hipMemcpy(*d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return DG_OK;
}

// numbering, tables and device copies on first use (synchronous, under the mesh lock)
dg_status ensure_hdiv(const dg_mesh* cm) {
  dg_mesh* m = const_cast<dg_mesh*>(cm);
  std::lock_guard<std::mutex> lock(m->mu);
  if (m->hd_ready) return DG_OK;
  std::string err;
  const int rc = dghdiv::build(m->h, m->hd, err);
  if (rc != 0) return fail(rc == -4 ? DG_EUNSUPPORTED : rc == -6 ? DG_EMESH : DG_EINVAL, err);
  dg_status s;
  if ((s = upload(m->hd.elem_facet, &m->d_hfacet)) != DG_OK ||
      (s = upload(m->hd.facet_elem, &m->d_hfelem)) != DG_OK ||
      (s = upload(m->hd.table, &m->d_htab)) != DG_OK)
    return s;
  HIP_TRY(hipMalloc((void**)&m->d_hlocal, (size_t)m->h.E * m->hd.ndof * sizeof(double) + 16));
  m->hd_ready = true;
  return DG_OK;
}

template <int D, int K>
dg_status run_to_dg(const dg_mesh* m, const double* u, double* out, hipStream_t s) {
  if (m->hd.table.size() != (size_t)HShape<D, K>::TAB || m->hd.ndof != HShape<D, K>::ND)
    return fail(DG_EINVAL, "H(div) tables do not match the kernel");
  const int64_t E = m->h.E, nfd = m->hd.nfacet * HShape<D, K>::NFD;
  hipLaunchKernelGGL((to_dg_kernel<D, K>), dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s, E,
                     nfd, u, m->d_hfacet, m->d_jinv, m->d_htab, out);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

template <int D, int K>
dg_status run_transpose(const dg_mesh* m, const double* F, double* out, hipStream_t s) {
  if (m->hd.table.size() != (size_t)HShape<D, K>::TAB || m->hd.ndof != HShape<D, K>::ND)
    return fail(DG_EINVAL, "H(div) tables do not match the kernel");
  const int64_t E = m->h.E, nfd = m->hd.nfacet * HShape<D, K>::NFD, N = m->hd.N;
  hipLaunchKernelGGL((transpose_local_kernel<D, K>), dim3((unsigned)((E + 255) / 256)), dim3(256), 0,
                     s, E, F, m->d_hfacet, m->d_jinv, m->d_htab, m->d_hlocal);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL((transpose_gather_kernel<D, K>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                     s, N, nfd, m->d_hfelem, m->d_hlocal, out);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

// degrees with kernels: 1..6 in 2D, 1..4 in 3D (the operator kernels' range)
bool hdiv_degree_ok(int dim, int k) { return k >= 1 && k <= (dim == 2 ? 6 : 4); }

dg_status prepare(const dg_mesh* m) {
  if (m->h.dim != 2 && m->h.dim != 3) return fail(DG_EINVAL, "the H(div) transfer needs dim 2 or 3");
  if (!hdiv_degree_ok(m->h.dim, m->h.k))
    return fail(DG_EINVAL, "the H(div) transfer needs 1 <= k <= 6 (2D) or 1 <= k <= 4 (3D)");
  dg_status st = dgi::ensure_device(m);
  if (st != DG_OK) return st;
  return ensure_hdiv(m);
}

}  // namespace

extern "C" {

dg_status dg_hdiv_info(const dg_mesh* m, int64_t* n_dof, int64_t* n_facet) {
  if (!m || !n_dof) return fail(DG_EINVAL, "null pointer");
  if (m->h.dim != 2 && m->h.dim != 3) return fail(DG_EINVAL, "the H(div) transfer needs dim 2 or 3");
  if (!hdiv_degree_ok(m->h.dim, m->h.k))
    return fail(DG_EINVAL, "the H(div) transfer needs 1 <= k <= 6 (2D) or 1 <= k <= 4 (3D)");
  dghdiv::Host hd;
  std::string err;
  const int rc = dghdiv::build(m->h, hd, err);
  if (rc != 0) return fail(DG_EMESH, err);
  *n_dof = hd.N;
  if (n_facet) *n_facet = hd.nfacet;
  return DG_OK;
}

dg_status dg_hdiv_reference(int dim, int k, double* table_out) {
  if (!table_out) return fail(DG_EINVAL, "null pointer");
  if ((dim != 2 && dim != 3) || !hdiv_degree_ok(dim, k))
    return fail(DG_EINVAL, "need dim 2 with k in 1..6 or dim 3 with k in 1..4");
  std::vector<double> t;
  dghdiv::reference_dual(dim, k, t);
  std::memcpy(table_out, t.data(), t.size() * sizeof(double));
  return DG_OK;
}

dg_status dg_transfer_to_dg(const dg_mesh* m, const double* u, double* w_out, void* stream) {
  if (!m || !u || !w_out) return fail(DG_EINVAL, "null pointer");
  if (u == w_out) return fail(DG_EINVAL, "w_out must not alias u");
  dg_status st = prepare(m);
  if (st != DG_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  if (m->h.dim == 3) {
    switch (m->h.k) {
      case 1: return run_to_dg<3, 1>(m, u, w_out, s);
      case 2: return run_to_dg<3, 2>(m, u, w_out, s);
      case 3: return run_to_dg<3, 3>(m, u, w_out, s);
      default: return run_to_dg<3, 4>(m, u, w_out, s);
    }
  }
  switch (m->h.k) {
    case 1: return run_to_dg<2, 1>(m, u, w_out, s);
    case 2: return run_to_dg<2, 2>(m, u, w_out, s);
    case 3: return run_to_dg<2, 3>(m, u, w_out, s);
    case 4: return run_to_dg<2, 4>(m, u, w_out, s);
    case 5: return run_to_dg<2, 5>(m, u, w_out, s);
    default: return run_to_dg<2, 6>(m, u, w_out, s);
  }
}

dg_status dg_transfer_transpose(const dg_mesh* m, const double* f, double* g_out,
                                void* stream) {
  if (!m || !f || !g_out) return fail(DG_EINVAL, "null pointer");
  if (f == g_out) return fail(DG_EINVAL, "g_out must not alias f");
  dg_status st = prepare(m);
  if (st != DG_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  if (m->h.dim == 3) {
    switch (m->h.k) {
      case 1: return run_transpose<3, 1>(m, f, g_out, s);
      case 2: return run_transpose<3, 2>(m, f, g_out, s);
      case 3: return run_transpose<3, 3>(m, f, g_out, s);
      default: return run_transpose<3, 4>(m, f, g_out, s);
    }
  }
  switch (m->h.k) {
    case 1: return run_transpose<2, 1>(m, f, g_out, s);
    case 2: return run_transpose<2, 2>(m, f, g_out, s);
    case 3: return run_transpose<2, 3>(m, f, g_out, s);
    case 4: return run_transpose<2, 4>(m, f, g_out, s);
    case 5: return run_transpose<2, 5>(m, f, g_out, s);
    default: return run_transpose<2, 6>(m, f, g_out, s);
  }
}

}  // extern "C"
