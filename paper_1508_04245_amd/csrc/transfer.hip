// Transfer operators between the H(div) space W_h and the DG space V_h on 2D meshes
// (Sec. 2.4): I = (M^V)^-1 M^{U,V} (the DG coefficients of a W_h field) and its transpose
// I^T (a functional on V_h, given by its values on the DG basis, to one on W_h).
//
// On element T a W_h field is sum_j s_j u_J(j) Piola(psi^_j), so with the signed Piola map
// v = J v^ / det J its DG coefficients are
//   c[i][m] = sum_a (J / det J)_ia ref[a][m],   ref[a][m] = sum_j s_j u_J(j) C_j[a][m],
// and J / det J is the adjugate of J^-1, which the mesh already stores.  One lane per element;
// the reference dual basis C (ndof x 2 x np doubles) sits in LDS and is read with wave-uniform
// addresses.  The transpose runs in two passes: every element writes the signed contributions
// s_j sum_{a,m} C_j[a][m] G[a][m] (G = adj(J^-1)^T F) of its local dofs, then every global dof
// adds its one (interior, boundary facet) or two (interior facet) contributions in a fixed
// order, so the result is deterministic and needs no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace {

using dgi::fail;

template <int K>
struct HShape {
  static constexpr int NP = (K + 1) * (K + 2) / 2, ND = 2 * NP, NFD = K + 1, NI = K * K - 1;
};

template <int K>
__global__ void __launch_bounds__(256) to_dg_kernel(int64_t E, int64_t nfd, const double* u,
                                                    const int* hf, const double* jinv,
                                                    const double* tab, double* out) {
  using S = HShape<K>;
  __shared__ double st[S::ND * S::ND];
  for (int i = threadIdx.x; i < S::ND * S::ND; i += 256) st[i] = tab[i];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= E) return;
  double ref[2][S::NP];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int m = 0; m < S::NP; ++m) ref[a][m] = 0.0;
  auto accumulate = [&](int j, double uj) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int m = 0; m < S::NP; ++m) ref[a][m] = fma(uj, st[(j * 2 + a) * S::NP + m], ref[a][m]);
  };
  // facet dofs with their signs (reference dof order), then the interior dofs
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int code = hf[t * 3 + f];
    const int64_t id = code >> 2;
    const double sf = (code & 2) ? -1.0 : 1.0;
    const double so = (code & 1) ? -sf : sf;  // odd l under a reversed parameter
#pragma unroll 1
    for (int l = 0; l < S::NFD; ++l) accumulate(f * S::NFD + l, ((l & 1) ? so : sf) * u[id * S::NFD + l]);
  }
  const double* ui = u + nfd + t * S::NI;
#pragma unroll 1
  for (int r = 0; r < S::NI; ++r) accumulate(3 * S::NFD + r, ui[r]);
  // J / det J = adj(J^-1) = [[ji11, -ji01], [-ji10, ji00]]
  const double* ji = jinv + t * 4;
  const double A[2][2] = {{ji[3], -ji[1]}, {-ji[2], ji[0]}};
  double* o = out + t * S::ND;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int m = 0; m < S::NP; ++m) o[i * S::NP + m] = fma(A[i][0], ref[0][m], A[i][1] * ref[1][m]);
}

template <int K>
__global__ void __launch_bounds__(256) transpose_local_kernel(int64_t E, const double* F,
                                                              const int* hf, const double* jinv,
                                                              const double* tab, double* loc) {
  using S = HShape<K>;
  __shared__ double st[S::ND * S::ND];
  for (int i = threadIdx.x; i < S::ND * S::ND; i += 256) st[i] = tab[i];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= E) return;
  const double* ji = jinv + t * 4;
  const double A[2][2] = {{ji[3], -ji[1]}, {-ji[2], ji[0]}};
  const double* f = F + t * S::ND;
  double G[2][S::NP];  // G[a][m] = sum_i A[i][a] F[i][m]
#pragma unroll
  for (int m = 0; m < S::NP; ++m) {
    const double f0 = f[m], f1 = f[S::NP + m];
#pragma unroll
    for (int a = 0; a < 2; ++a) G[a][m] = fma(A[0][a], f0, A[1][a] * f1);
  }
  double* o = loc + t * S::ND;
  auto contract = [&](int j) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int m = 0; m < S::NP; ++m) acc = fma(st[(j * 2 + a) * S::NP + m], G[a][m], acc);
    return acc;
  };
#pragma unroll
  for (int fc = 0; fc < 3; ++fc) {
    const int code = hf[t * 3 + fc];
    const double sf = (code & 2) ? -1.0 : 1.0;
    const double so = (code & 1) ? -sf : sf;  // odd l under a reversed parameter
#pragma unroll 1
    for (int l = 0; l < S::NFD; ++l) {
      const int j = fc * S::NFD + l;
      o[j] = ((l & 1) ? so : sf) * contract(j);
    }
  }
#pragma unroll 1
  for (int j = 3 * S::NFD; j < S::ND; ++j) o[j] = contract(j);
}

template <int K>
__global__ void __launch_bounds__(256) transpose_gather_kernel(int64_t N, int64_t nfd,
                                                               const int64_t* fe,
                                                               const double* loc, double* out) {
  using S = HShape<K>;
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (d >= N) return;
  if (d < nfd) {
    const int64_t fc = d / S::NFD, l = d % S::NFD;
    const int64_t s0 = fe[2 * fc], s1 = fe[2 * fc + 1];
    double v = loc[(s0 / 3) * S::ND + (s0 % 3) * S::NFD + l];
    if (s1 >= 0) v += loc[(s1 / 3) * S::ND + (s1 % 3) * S::NFD + l];
    out[d] = v;
  } else {
    const int64_t t = (d - nfd) / S::NI, r = (d - nfd) % S::NI;
    out[d] = loc[t * S::ND + 3 * S::NFD + r];
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

template <int K>
dg_status run_to_dg(const dg_mesh* m, const double* u, double* out, hipStream_t s) {
  const int64_t E = m->h.E, nfd = m->hd.nfacet * (K + 1);
  hipLaunchKernelGGL(to_dg_kernel<K>, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s, E,
                     nfd, u, m->d_hfacet, m->d_jinv, m->d_htab, out);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

template <int K>
dg_status run_transpose(const dg_mesh* m, const double* F, double* out, hipStream_t s) {
  const int64_t E = m->h.E, nfd = m->hd.nfacet * (K + 1), N = m->hd.N;
  hipLaunchKernelGGL(transpose_local_kernel<K>, dim3((unsigned)((E + 255) / 256)), dim3(256), 0,
                     s, E, F, m->d_hfacet, m->d_jinv, m->d_htab, m->d_hlocal);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(transpose_gather_kernel<K>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                     s, N, nfd, m->d_hfelem, m->d_hlocal, out);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

dg_status prepare(const dg_mesh* m) {
  if (m->h.dim != 2) return fail(DG_EUNSUPPORTED, "the H(div) transfer is built for 2D meshes");
  if (m->h.k < 1 || m->h.k > 6) return fail(DG_EINVAL, "the H(div) transfer needs 1 <= k <= 6");
  dg_status st = dgi::ensure_device(m);
  if (st != DG_OK) return st;
  return ensure_hdiv(m);
}

}  // namespace

extern "C" {

dg_status dg_hdiv_info(const dg_mesh* m, int64_t* n_dof, int64_t* n_facet) {
  if (!m || !n_dof) return fail(DG_EINVAL, "null pointer");
  if (m->h.dim != 2) return fail(DG_EUNSUPPORTED, "the H(div) transfer is built for 2D meshes");
  if (m->h.k < 1) return fail(DG_EINVAL, "the H(div) transfer needs k >= 1");
  dghdiv::Host hd;
  std::string err;
  const int rc = dghdiv::build(m->h, hd, err);
  if (rc != 0) return fail(DG_EMESH, err);
  *n_dof = hd.N;
  if (n_facet) *n_facet = hd.nfacet;
  return DG_OK;
}

dg_status dg_hdiv_reference(int k, double* table_out) {
  if (!table_out) return fail(DG_EINVAL, "null pointer");
  if (k < 1 || k > 6) return fail(DG_EINVAL, "k must be in 1..6");
  std::vector<double> t;
  dghdiv::reference_dual(k, t);
  std::memcpy(table_out, t.data(), t.size() * sizeof(double));
  return DG_OK;
}

dg_status dg_transfer_to_dg(const dg_mesh* m, const double* u, double* w_out, void* stream) {
  if (!m || !u || !w_out) return fail(DG_EINVAL, "null pointer");
  if (u == w_out) return fail(DG_EINVAL, "w_out must not alias u");
  dg_status st = prepare(m);
  if (st != DG_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  switch (m->h.k) {
    case 1: return run_to_dg<1>(m, u, w_out, s);
    case 2: return run_to_dg<2>(m, u, w_out, s);
    case 3: return run_to_dg<3>(m, u, w_out, s);
    case 4: return run_to_dg<4>(m, u, w_out, s);
    case 5: return run_to_dg<5>(m, u, w_out, s);
    default: return run_to_dg<6>(m, u, w_out, s);
  }
}

dg_status dg_transfer_transpose(const dg_mesh* m, const double* f, double* g_out,
                                void* stream) {
  if (!m || !f || !g_out) return fail(DG_EINVAL, "null pointer");
  if (f == g_out) return fail(DG_EINVAL, "g_out must not alias f");
  dg_status st = prepare(m);
  if (st != DG_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  switch (m->h.k) {
    case 1: return run_transpose<1>(m, f, g_out, s);
    case 2: return run_transpose<2>(m, f, g_out, s);
    case 3: return run_transpose<3>(m, f, g_out, s);
    case 4: return run_transpose<4>(m, f, g_out, s);
    case 5: return run_transpose<5>(m, f, g_out, s);
    default: return run_transpose<6>(m, f, g_out, s);
  }
}

}  // extern "C"
