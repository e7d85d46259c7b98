// C ABI of the upwind-DG convection library (see include/dgconv.h): mesh creation and
// device tables, operator application, fused SSP-RK3 substeps, reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dgconv.h"
#include "internal.hpp"
#include "conv_kernels.hpp"
#include "mfma_kernels.hpp"
#include "mesh.hpp"
#include "refelem.hpp"

namespace dgi {
thread_local std::string g_err;
dg_status fail(dg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
}  // namespace dgi

namespace {

using dgi::fail;

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

constexpr int kMaxK2 = 6, kMaxK3 = 4;
constexpr int kRedBlock = 256;

}  // namespace

namespace {

// ------------------------------------------------------------------ reductions
// what: 1 energy, 2 momentum (first dim outputs), 3 l2diff (2 outputs), 4 nonfinite
__global__ void __launch_bounds__(kRedBlock)
elem_reduce_kernel(int what, int dim, int np, int64_t E, const double* __restrict__ a,
                   const double* __restrict__ b, const double* __restrict__ absdet,
                   double phi0_vol, double* __restrict__ partial) {
  __shared__ double sh[kRedBlock][3];
  const int64_t t = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
  double v[3] = {0, 0, 0};
  if (t < E) {
    const double* pa = a + t * dim * np;
    const double J = absdet[t];
    if (what == 1) {
      double s = 0;
      for (int i = 0; i < dim * np; ++i) s = fma(pa[i], pa[i], s);
      v[0] = 0.5 * J * s;
    } else if (what == 2) {
      for (int i = 0; i < dim; ++i) v[i] = J * pa[i * np] * phi0_vol;
    } else if (what == 3) {
      const double* pb = b + t * dim * np;
      double s0 = 0, s1 = 0;
      for (int i = 0; i < dim * np; ++i) {
        const double d = pa[i] - pb[i];
        s0 = fma(d, d, s0);
        s1 = fma(pb[i], pb[i], s1);
      }
      v[0] = J * s0;
      v[1] = J * s1;
    } else {
      double s = 0;
      for (int i = 0; i < dim * np; ++i) s += isfinite(pa[i]) ? 0.0 : 1.0;
      v[0] = s;
    }
  }
  for (int c = 0; c < 3; ++c) sh[threadIdx.x][c] = v[c];
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 3; ++c) sh[threadIdx.x][c] += sh[threadIdx.x + s][c];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) partial[blockIdx.x * 3 + c] = sh[0][c];
}

// max over the points of the collapsed rule exact to 3k-1 of |w|, per block (spd: the basis
// values there, [NS][NP])
template <int D, int K>
__global__ void __launch_bounds__(kRedBlock)
maxvel_kernel(int64_t E, const double* __restrict__ a, const double* __restrict__ spd,
              double* __restrict__ partial) {
  using S = dgk::Shape<D, K>;
  __shared__ double sh[kRedBlock];
  const int64_t t = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
  double mx = 0;
  if (t < E) {
    const double* pa = a + t * D * S::NP;
    for (int q = 0; q < S::NS; ++q) {
      double s = 0;
      for (int i = 0; i < D; ++i) {
        double w = 0;
        for (int m = 0; m < S::NP; ++m) w = fma(spd[q * S::NP + m], pa[i * S::NP + m], w);
        s = fma(w, w, s);
      }
      mx = fmax(mx, s);
    }
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[blockIdx.x * 3] = sqrt(sh[0]);
    partial[blockIdx.x * 3 + 1] = 0;
    partial[blockIdx.x * 3 + 2] = 0;
  }
}

// single block: combine the partials in a fixed order
__global__ void __launch_bounds__(kRedBlock)
final_reduce_kernel(int nblocks, int is_max, int nout, int sqrt_out,
                    const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double sh[kRedBlock][3];
  double v[3] = {0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kRedBlock)
    for (int c = 0; c < 3; ++c)
      v[c] = is_max ? fmax(v[c], partial[b * 3 + c]) : v[c] + partial[b * 3 + c];
  for (int c = 0; c < 3; ++c) sh[threadIdx.x][c] = v[c];
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 3; ++c)
        sh[threadIdx.x][c] = is_max ? fmax(sh[threadIdx.x][c], sh[threadIdx.x + s][c])
                                    : sh[threadIdx.x][c] + sh[threadIdx.x + s][c];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < nout; ++c) out[c] = sqrt_out ? sqrt(sh[0][c]) : sh[0][c];
}

// ------------------------------------------------------------------ dispatch
template <int D, int K>
hipError_t launch_maxvel(const dg_mesh* m, const double* a, double* partial, hipStream_t s) {
  if (dgk::Shape<D, K>::NS != m->t.ns || dgk::Shape<D, K>::NP != m->h.np)
    return hipErrorInvalidValue;
  const int nb = (int)((m->h.E + kRedBlock - 1) / kRedBlock);
  hipLaunchKernelGGL((maxvel_kernel<D, K>), dim3(nb), dim3(kRedBlock), 0, s, m->h.E, a,
                     m->d_spd, partial);
  return hipGetLastError();
}

// default table sources of the VALU kernel (bit t of the mask: table t read through scalar
// loads, else from LDS; t = basis values, gradients, own traces, neighbour traces, lifts),
// from sweeps of the masks on MI355X.  2D P4 FP64 (28 volume points): basis values and lifts
// in LDS, gradients and both trace tables through scalar loads (mask 14: 41.2-41.3 us per
// launch on 256x256x2 triangles, against 41.6-41.7 for 22, 44.1 for 26, 48.2 for 20, 49.1-
// 49.5 for 2, 18 and 30, 52 for 6, 53.5 for 21, 57 for 28, 58 with every table in LDS and 78
// with none).  Smaller elements keep every table in LDS; other tables too large for LDS all
// come through scalar loads.
template <int D, int K, typename T, bool SELF = true, bool BND = false>
constexpr int default_tab_src() {
  // 3D P2 (14 volume and 12 facet points, 49 KiB of tables): the FP64 self kernel with the
  // basis values in LDS and every other table through scalar loads (496 us per launch
  // against 507 with every table through scalar loads, 519 for basis values and gradients in
  // LDS, 526 for 22, 616 with every table in LDS); the frozen and boundary variants keep
  // scalar loads
  if (D == 3 && K == 2 && sizeof(T) == 8) return SELF && !BND ? 30 : dgk::SM_ALL;
  // FP32 self kernels: 3D P2 with basis values and gradients in LDS (285.5 against 289.5 us
  // for 22, 287 with every table through scalar loads, 328 with every table in LDS); 2D P4
  // with the lifts through scalar loads (35.0 against 36.2)
  if (D == 3 && K == 2 && sizeof(T) == 4 && SELF && !BND) return 28;
  if (D == 2 && K == 4 && sizeof(T) == 4 && SELF && !BND) return 16;
  if (!dgk::tables_in_lds<D, K, T>()) return dgk::SM_ALL;
  if (D == 2 && K == 4 && sizeof(T) == 8) return 14;
  return 0;
}

// TS: state type; TC: contraction type (TS = double, TC = float: FP32 contractions around an
// FP64 state, flux, facet sums and update)
template <int D, int K, typename TS, bool SELF, int SM, bool BND = false, bool LANE = false,
          typename TC = TS>
void launch_conv_sm(const dgk::ConvArgs<TS, TC>& a, dim3 grid, hipStream_t s) {
  hipLaunchKernelGGL((dgk::conv_kernel<D, K, TS, SELF, SM, BND, LANE, TC>), grid, dim3(256), 0,
                     s, a);
}

// FP64 self-convection on a periodic mesh, class-grouped tiles: the pipelined kernel, or the
// general one (mesh option)
template <int D, int K, int SM>
void launch_self_fp64(const dg_mesh* m, const dgk::ConvArgs<double>& a, dim3 grid, hipStream_t s) {
  if (m->self_pipe)
    hipLaunchKernelGGL((dgk::conv_self_kernel<D, K, SM>), grid, dim3(256), 0, s, a);
  else
    launch_conv_sm<D, K, double, true, SM>(a, grid, s);
}

// per-lane table mode: the facet tables must come from LDS; the volume tables go through
// scalar loads when the whole set does not fit the 64 KiB a class-tiled kernel stages
template <int D, int K, typename T>
constexpr int lane_tab_src() {
  // 2D P4 FP64: the weighted gradients through scalar loads (jittered 256x256x2: 51.4 against
  // 52.3 us per launch with every table in LDS; the basis values too: 84 us)
  if (D == 2 && K == 4 && sizeof(T) == 8) return 1 << dgk::TB_DV;
  if (D == 3 && K == 2 && sizeof(T) == 8) return (1 << dgk::TB_BV) | (1 << dgk::TB_DV);
  return (size_t)dgk::Shape<D, K>::TOTAL * sizeof(T) <= 65536 ? 0
                                                              : (1 << dgk::TB_BV) | (1 << dgk::TB_DV);
}

template <int D, int K, typename TS, typename T, bool SELF>
hipError_t launch_conv_dk(const dg_mesh* m, const dgk::ConvArgs<TS, T>& a, hipStream_t s) {
  // table sources follow the contraction type (the tables are stored in it)
  constexpr int kDef = default_tab_src<D, K, T, SELF>();
  // the kernel's compile-time table layout must match the host tables it reads
  if ((size_t)dgk::Shape<D, K>::TOTAL != m->t.total || dgk::Shape<D, K>::NP != m->h.np)
    return hipErrorInvalidValue;
  if ((int64_t)m->h.elem_list.size() != (int64_t)m->h.ntiles * 64) return hipErrorInvalidValue;
  const dim3 grid((m->h.ntiles + 3) / 4);
  if (m->h.lane_tables) {
    if constexpr (dgk::lane_tables_ok<D, K, T>()) {
      launch_conv_sm<D, K, TS, SELF, lane_tab_src<D, K, T>(), true, true, T>(a, grid, s);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;  // never chosen at mesh creation for such elements
  }
  if (m->h.nbf > 0) {  // meshes with boundary facets: the variant that handles them
    launch_conv_sm<D, K, TS, SELF, default_tab_src<D, K, T, SELF, true>(), true, false, T>(
        a, grid, s);
    return hipGetLastError();
  }
  // DGCONV_TABLES may pick another split for the FP64 self kernel: every table through
  // scalar loads (31) and, where the whole block fits in LDS, every table in LDS (0), 21
  // (gradients and neighbour traces in LDS) or 22; other values keep the default
  if constexpr (SELF && sizeof(T) == 8 && sizeof(TS) == 8) {
    if constexpr (D == 2 && K >= 2 && K <= 4) {  // two lanes per element (mesh option)
      if (m->pair && a.mode != 2) {
        // table sources at four waves per SIMD: every table in LDS up to P3; for P4 the LDS
        // return bandwidth of the broadcast reads limits, and only the basis values stay there
        constexpr int kPair = K == 4 ? 30 : 0;
        hipLaunchKernelGGL((dgk::conv_pair_kernel<K, kPair>), dim3(m->h.ntiles / 2), dim3(256),
                           0, s, a);
        return hipGetLastError();
      }
    }
    const int src = m->tab_src;
    if (src >= 0 && src != kDef) {
      if (src == dgk::SM_ALL) {
        launch_self_fp64<D, K, dgk::SM_ALL>(m, a, grid, s);
        return hipGetLastError();
      }
      if constexpr (dgk::tables_in_lds<D, K, T>()) {
        switch (src) {
          case 0: launch_self_fp64<D, K, 0>(m, a, grid, s); return hipGetLastError();
          case 21: launch_self_fp64<D, K, 21>(m, a, grid, s); return hipGetLastError();
          case 22: launch_self_fp64<D, K, 22>(m, a, grid, s); return hipGetLastError();
          default: break;
        }
      }
    }
    launch_self_fp64<D, K, kDef>(m, a, grid, s);
    return hipGetLastError();
  }
  launch_conv_sm<D, K, TS, SELF, kDef, false, false, T>(a, grid, s);
  return hipGetLastError();
}

template <typename TS, typename TC, bool SELF>
hipError_t launch_conv(const dg_mesh* m, const dgk::ConvArgs<TS, TC>& a, hipStream_t s) {
  const int d = m->h.dim, k = m->h.k;
#define DG_CASE(D_, K_) \
  if (d == D_ && k == K_) return launch_conv_dk<D_, K_, TS, TC, SELF>(m, a, s);
  DG_CASE(2, 0) DG_CASE(2, 1) DG_CASE(2, 2) DG_CASE(2, 3) DG_CASE(2, 4) DG_CASE(2, 5)
  DG_CASE(2, 6) DG_CASE(3, 0) DG_CASE(3, 1) DG_CASE(3, 2) DG_CASE(3, 3) DG_CASE(3, 4)
#undef DG_CASE
  return hipErrorInvalidValue;
}

template <typename TS, typename TC>
hipError_t launch_conv_any(const dg_mesh* m, const dgk::ConvArgs<TS, TC>& a, hipStream_t s) {
  return a.u ? launch_conv<TS, TC, false>(m, a, s) : launch_conv<TS, TC, true>(m, a, s);
}

template <typename TS, typename TC = TS>
dgk::ConvArgs<TS, TC> base_args(const dg_mesh* m) {
  dgk::ConvArgs<TS, TC> a{};
  if constexpr (sizeof(TC) == 8) a.tab = m->d_tab;
  else a.tab = m->d_tab_f;
  if constexpr (sizeof(TS) == 8) a.jinv = m->d_jinv;
  else a.jinv = m->d_jinv_f;
  a.nbr = m->d_nbr;
  a.elem_list = m->d_elem_list;
  a.tile_type = m->d_tile_type;
  a.type_tab = m->d_type_tab;
  a.elem_tab = m->d_elem_tab;
  a.ntiles = m->h.ntiles;
  return a;
}

// outer values at the boundary facet points (meshes with bounded directions)
struct Bnd {
  const void* wb;
  const void* ub;
};

template <typename T, typename TC = T>
dg_status run_apply(const dg_mesh* m, const void* w, const void* u, void* r, hipStream_t s,
                    const Bnd* bc = nullptr) {
  auto a = base_args<T, TC>(m);
  a.x = (const T*)w;
  a.u = (const T*)u;
  if (bc) { a.wb = (const T*)bc->wb; a.ub = (const T*)bc->ub; }
  a.out = (T*)r;
  a.mode = 0;
  HIP_TRY(launch_conv_any(m, a, s));
  return DG_OK;
}

// Convecting velocity extrapolated linearly in time from two fields (the propagation problem
// of Sec. 3.2): u(s) = ua + (s - ta) / (tb - ta) (ub - ua); substep j starts at t0 + j dt.
struct Extrap {
  const void* ub;
  double t0, ta, tb;
  // time weight of ub at stage time t0 + j dt + c dt (Shu-Osher abscissae c = 0, 1, 1/2)
  double weight(int j, double dt, double c) const {
    const double s = t0 + j * dt;
    return ((c == 0.0 ? s : s + c * dt) - ta) / (tb - ta);
  }
};

template <typename T, typename TC = T>
dg_status run_rk(const dg_mesh* m, void* w, double dt, int n, const void* u, void* work,
                 hipStream_t s, const Extrap* ex = nullptr, const Bnd* bc = nullptr) {
  const size_t n_state = (size_t)m->h.E * m->h.dim * m->h.np;
  T* w0 = (T*)w;
  T* w1 = (T*)work;
  T* w2 = w1 + n_state;
  auto a = base_args<T, TC>(m);
  a.u = (const T*)u;
  a.u2 = ex ? (const T*)ex->ub : nullptr;
  if (bc) { a.wb = (const T*)bc->wb; a.ub = (const T*)bc->ub; }
  a.mode = 1;
  a.dt = (T)dt;
  for (int it = 0; it < n; ++it) {
    a.x = w0; a.w0 = nullptr; a.out = w1; a.a = T(0); a.b = T(1);
    if (ex) a.uth = (T)ex->weight(it, dt, 0.0);
    HIP_TRY(launch_conv_any(m, a, s));
    a.x = w1; a.w0 = w0; a.out = w2; a.a = T(0.75); a.b = T(0.25);
    if (ex) a.uth = (T)ex->weight(it, dt, 1.0);
    HIP_TRY(launch_conv_any(m, a, s));
    a.x = w2; a.w0 = w0; a.out = w0; a.a = T(1.0 / 3.0); a.b = T(2.0 / 3.0);
    if (ex) a.uth = (T)ex->weight(it, dt, 0.5);
    HIP_TRY(launch_conv_any(m, a, s));
  }
  return DG_OK;
}


// ------------------------------------------------------------------ matrix-core tables
// A-operand fragment blocks (see mfma_kernels.hpp) built from the FP64 reference tables.
// Engine 0: f64 blocks, 256 doubles: [j][lane] = A[lane % 16][4 j + lane / 16].
// Engines 1, 2: NS pieces of 16-bit values: [piece][lane][j] = piece(A[lane % 16][4 (lane/16) + j]).
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint16_t f16_bits(double v, double* back) {
  const _Float16 h = (_Float16)(float)v;
  *back = (double)(float)h;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

std::vector<uint8_t> build_frags(const dgmesh::Tables& t, int d, int np, int engine) {
  const int nq = t.nq, nfq = t.nfq, ntab = (d + 1) * t.nperm;
  const int KP = (np + 15) / 16, QT = (nq + 15) / 16, FT = (nfq + 15) / 16;
  const int nblk = QT * KP + d * KP * QT + ntab * FT * KP + ntab * KP * FT;
  const int ns = engine == 0 ? 1 : (engine == 1 ? 2 : 3);
  const size_t blk_bytes = engine == 0 ? 256 * 8 : (size_t)ns * 64 * 4 * 2;
  std::vector<uint8_t> out((size_t)nblk * blk_bytes, 0);
  auto put = [&](int blk, auto&& A /* (row, col) -> double, 16 x 16 block */) {
    uint8_t* base = out.data() + (size_t)blk * blk_bytes;
    for (int lane = 0; lane < 64; ++lane)
      for (int j = 0; j < 4; ++j) {
        if (engine == 0) {
          ((double*)base)[j * 64 + lane] = A(lane % 16, 4 * j + lane / 16);
          continue;
        }
        double rem = A(lane % 16, 4 * (lane / 16) + j);
        for (int p = 0; p < ns; ++p) {
          uint16_t bits;
          double back;
          if (engine == 1) {
            bits = f16_bits(rem, &back);
          } else {
            bits = bf16_bits((float)rem);
            back = (double)bf16_value(bits);
          }
          rem -= back;
          ((uint16_t*)base)[((size_t)p * 64 + lane) * 4 + j] = bits;
        }
      }
  };
  const double* Bv = &t.data[t.off_bv];
  const double* Dv = &t.data[t.off_dv];
  const double* Tr = &t.data[t.off_tr];
  const double* Lf = &t.data[t.off_lf];
  int blk = 0;
  for (int qt = 0; qt < QT; ++qt)
    for (int kc = 0; kc < KP; ++kc, ++blk)
      put(blk, [&](int r, int c) {
        const int q = 16 * qt + r, m = 16 * kc + c;
        return (q < nq && m < np) ? Bv[q * np + m] : 0.0;
      });
  for (int j = 0; j < d; ++j)
    for (int mt = 0; mt < KP; ++mt)
      for (int qt = 0; qt < QT; ++qt, ++blk)
        put(blk, [&](int r, int c) {
          const int m = 16 * mt + r, q = 16 * qt + c;
          return (q < nq && m < np) ? Dv[(q * np + m) * d + j] : 0.0;
        });
  for (int tb = 0; tb < ntab; ++tb)
    for (int ft = 0; ft < FT; ++ft)
      for (int kc = 0; kc < KP; ++kc, ++blk)
        put(blk, [&](int r, int c) {
          const int q = 16 * ft + r, m = 16 * kc + c;
          return (q < nfq && m < np) ? Tr[((size_t)tb * nfq + q) * np + m] : 0.0;
        });
  for (int tb = 0; tb < ntab; ++tb)
    for (int mt = 0; mt < KP; ++mt)
      for (int ft = 0; ft < FT; ++ft, ++blk)
        put(blk, [&](int r, int c) {
          const int m = 16 * mt + r, q = 16 * ft + c;
          return (q < nfq && m < np) ? -Lf[((size_t)tb * nfq + q) * np + m] : 0.0;
        });
  return out;
}

dg_status ensure_frags(const dg_mesh* cm, int engine) {
  dg_mesh* m = const_cast<dg_mesh*>(cm);
  std::lock_guard<std::mutex> lock(m->mu);
  if (m->d_frag[engine]) return DG_OK;
  const auto bytes = build_frags(m->t, m->h.dim, m->h.np, engine);
  HIP_TRY(hipMalloc(&m->d_frag[engine], bytes.size()));
  HIP_TRY(hipMemcpy(m->d_frag[engine], bytes.data(), bytes.size(), hipMemcpyHostToDevice));
  return DG_OK;
}

template <int D, int K, class E, bool SELF>
hipError_t launch_mconv_dk(const dg_mesh* m, const dgm::MArgs<double>& a, hipStream_t s) {
  if ((size_t)m->h.elem_list16.size() != (size_t)m->h.ntiles16 * 16 || m->h.ntiles16 % 4)
    return hipErrorInvalidValue;
  const dim3 grid(m->h.ntiles16 / 4), block(256);
  if (m->h.nbf > 0)  // meshes with boundary facets: the variant that handles them
    hipLaunchKernelGGL((dgm::mconv_kernel<D, K, E, SELF, true>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((dgm::mconv_kernel<D, K, E, SELF, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <class E, bool SELF>
hipError_t launch_mconv(const dg_mesh* m, const dgm::MArgs<double>& a, hipStream_t s) {
  const int d = m->h.dim, k = m->h.k;
#define DG_CASE(D_, K_) \
  if (d == D_ && k == K_) return launch_mconv_dk<D_, K_, E, SELF>(m, a, s);
  DG_CASE(2, 0) DG_CASE(2, 1) DG_CASE(2, 2) DG_CASE(2, 3) DG_CASE(2, 4) DG_CASE(2, 5)
  DG_CASE(2, 6) DG_CASE(3, 0) DG_CASE(3, 1) DG_CASE(3, 2) DG_CASE(3, 3) DG_CASE(3, 4)
#undef DG_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_mconv_any(const dg_mesh* m, int engine, const dgm::MArgs<double>& a,
                            hipStream_t s) {
  const bool self = a.u == nullptr;
  switch (engine) {
    case 0: return self ? launch_mconv<dgm::EngF64, true>(m, a, s) : launch_mconv<dgm::EngF64, false>(m, a, s);
    case 1: return self ? launch_mconv<dgm::EngSplit<true, 2>, true>(m, a, s)
                        : launch_mconv<dgm::EngSplit<true, 2>, false>(m, a, s);
    default: return self ? launch_mconv<dgm::EngSplit<false, 3>, true>(m, a, s)
                         : launch_mconv<dgm::EngSplit<false, 3>, false>(m, a, s);
  }
}

dgm::MArgs<double> mbase_args(const dg_mesh* m, int engine) {
  dgm::MArgs<double> a{};
  a.frag = m->d_frag[engine];
  a.jinv = m->d_jinv;
  a.nbr = m->d_nbr;
  a.elem_list = m->d_elem_list16;
  a.tile_type = m->d_tile_type16;
  a.type_tab = m->d_type_tab;
  a.ntiles = m->h.ntiles16;
  return a;
}

bool known_precision(dg_precision p) {
  return p == DG_FP64 || p == DG_FP32 || p == DG_MIX_F32 || p == DG_MIX_F16x2 ||
         p == DG_MIX_BF16x3;
}

// engine of a precision on the matrix-core path, or -1 for the VALU kernels
int engine_of(const dg_mesh* m, dg_precision prec, bool frozen) {
  if (prec == DG_MIX_F16x2) return 1;
  if (prec == DG_MIX_BF16x3) return 2;
  if (prec == DG_FP64 && (frozen ? m->fp64_mfma_frozen : m->fp64_mfma)) return 0;
  return -1;
}

dg_status run_apply_m(const dg_mesh* m, int engine, const void* w, const void* u, void* r,
                      hipStream_t s, const Bnd* bc = nullptr) {
  dg_status st = ensure_frags(m, engine);
  if (st != DG_OK) return st;
  auto a = mbase_args(m, engine);
  a.x = (const double*)w;
  a.u = (const double*)u;
  if (bc) { a.wb = (const double*)bc->wb; a.ub = (const double*)bc->ub; }
  a.out = (double*)r;
  a.mode = 0;
  HIP_TRY(launch_mconv_any(m, engine, a, s));
  return DG_OK;
}

dg_status run_rk_m(const dg_mesh* m, int engine, void* w, double dt, int n, const void* u,
                   void* work, hipStream_t s, const Extrap* ex = nullptr,
                   const Bnd* bc = nullptr) {
  dg_status st = ensure_frags(m, engine);
  if (st != DG_OK) return st;
  const size_t n_state = (size_t)m->h.E * m->h.dim * m->h.np;
  double* w0 = (double*)w;
  double* w1 = (double*)work;
  double* w2 = w1 + n_state;
  auto a = mbase_args(m, engine);
  a.u = (const double*)u;
  a.u2 = ex ? (const double*)ex->ub : nullptr;
  if (bc) { a.wb = (const double*)bc->wb; a.ub = (const double*)bc->ub; }
  a.mode = 1;
  a.dt = dt;
  for (int it = 0; it < n; ++it) {
    a.x = w0; a.w0 = nullptr; a.out = w1; a.a = 0.0; a.b = 1.0;
    if (ex) a.uth = ex->weight(it, dt, 0.0);
    HIP_TRY(launch_mconv_any(m, engine, a, s));
    a.x = w1; a.w0 = w0; a.out = w2; a.a = 0.75; a.b = 0.25;
    if (ex) a.uth = ex->weight(it, dt, 1.0);
    HIP_TRY(launch_mconv_any(m, engine, a, s));
    a.x = w2; a.w0 = w0; a.out = w0; a.a = 1.0 / 3.0; a.b = 2.0 / 3.0;
    if (ex) a.uth = ex->weight(it, dt, 0.5);
    HIP_TRY(launch_mconv_any(m, engine, a, s));
  }
  return DG_OK;
}

// ------------------------------------------------------------------ pseudo-time iteration
// Device-side control block of the Richardson iteration.  The host enqueues iterations in
// batches; the check kernel sets `done` at the first iterate whose residual meets the
// criterion and every later kernel of the batch returns at once, so the iterates stop exactly
// there without a host round trip per iteration.
struct RichState {
  int done, iters;
  double res0, res_last, unused;
};
static_assert(sizeof(RichState) <= 4 * sizeof(double), "control block size");

__global__ void rich_init_kernel(RichState* st) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->iters = -1;
    st->res0 = 0.0;
    st->res_last = 0.0;
  }
}

// residual norm of iterate `it` from the per-tile sums (fixed summation order), criterion
__global__ void __launch_bounds__(kRedBlock)
rich_check_kernel(int nparts, const double* __restrict__ partial, double rtol, int it,
                  RichState* st) {
  if (st->done) return;
  __shared__ double sh[kRedBlock];
  double v = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kRedBlock) v += partial[b];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double res = sqrt(sh[0]);
    if (it == 0) st->res0 = res;
    st->res_last = res;
    if (res <= rtol * (it == 0 ? res : st->res0)) {
      st->done = 1;
      st->iters = it;
    }
  }
}

// one Richardson update of x into out for every element, with the residual tile sums
template <typename TC>
dg_status rich_update_valu(const dg_mesh* m, const double* x, const double* g, const double* u,
                           double* out, double tau, double ds, const int* stop, hipStream_t s) {
  auto a = base_args<double, TC>(m);
  a.x = x; a.u = u; a.w0 = g; a.out = out; a.mode = 2; a.tau = tau; a.ds = ds;
  a.absdet = m->d_absdet; a.partial = m->d_rich_partial; a.stop = stop;
  HIP_TRY(launch_conv_any(m, a, s));
  return DG_OK;
}

// engine >= 0: the matrix-core kernel; -1: the FP64 VALU kernel; -2: the VALU kernel with
// FP32 contractions (DG_MIX_F32)
dg_status rich_update(const dg_mesh* m, int engine, const double* x, const double* g,
                      const double* u, double* out, double tau, double ds, const int* stop,
                      hipStream_t s, int* nparts) {
  if (engine >= 0) {
    auto a = mbase_args(m, engine);
    a.x = x; a.u = u; a.w0 = g; a.out = out; a.mode = 2; a.tau = tau; a.ds = ds;
    a.absdet = m->d_absdet; a.partial = m->d_rich_partial; a.stop = stop;
    *nparts = m->h.ntiles16;
    HIP_TRY(launch_mconv_any(m, engine, a, s));
  } else {
    *nparts = m->h.ntiles;
    return engine == -2 ? rich_update_valu<float>(m, x, g, u, out, tau, ds, stop, s)
                        : rich_update_valu<double>(m, x, g, u, out, tau, ds, stop, s);
  }
  return DG_OK;
}

dg_status run_richardson(const dg_mesh* m, int engine, double* v, const double* g,
                         const double* u, double tau, double ds, double rtol, int max_it,
                         double* work, hipStream_t s, int* iters_out, double* res_out) {
  RichState* st = (RichState*)m->d_rich_state;
  const int* stop = &st->done;
  double* buf[2] = {v, work};
  hipLaunchKernelGGL(rich_init_kernel, dim3(1), dim3(64), 0, s, st);
  HIP_TRY(hipGetLastError());
  constexpr int kBatch = 8;  // iterations enqueued between host checks
  RichState h{};
  int it = 0;
  while (it < max_it) {
    const int end = std::min(max_it, it + kBatch);
    for (; it < end; ++it) {
      int nparts = 0;
      dg_status rc = rich_update(m, engine, buf[it & 1], g, u, buf[(it + 1) & 1], tau, ds, stop,
                                 s, &nparts);
      if (rc != DG_OK) return rc;
      hipLaunchKernelGGL(rich_check_kernel, dim3(1), dim3(kRedBlock), 0, s, nparts,
                         m->d_rich_partial, rtol, it, st);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(RichState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h.done) break;
  }
  if (max_it == 0) {
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(RichState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  // iterate n is in buf[n & 1]: the first meeting the criterion, else the last computed
  const int n = h.done ? h.iters : max_it;
  if (n & 1) {
    const size_t bytes = (size_t)m->h.E * m->h.dim * m->h.np * sizeof(double);
    HIP_TRY(hipMemcpyAsync(v, work, bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (iters_out) *iters_out = n;
  if (res_out) {
    res_out[0] = h.res0;
    res_out[1] = h.res_last;
  }
  return DG_OK;
}

dg_status check_k(int dim, int k) {
  if (dim != 2 && dim != 3) return fail(DG_EINVAL, "dim must be 2 or 3");
  if (k < 0) return fail(DG_EINVAL, "k must be >= 0");
  if ((dim == 2 && k > kMaxK2) || (dim == 3 && k > kMaxK3))
    return fail(DG_EUNSUPPORTED, "k above the compiled range (2D: 0..6, 3D: 0..4)");
  return DG_OK;
}

template <typename T>
dg_status upload(const std::vector<T>& v, T** d) {
  HIP_TRY(hipMalloc((void**)d, v.size() * sizeof(T) + 16));
  HIP_TRY(hipMemcpy(*d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return DG_OK;
}

}  // namespace

// Device tables are uploaded on the first compute call (synchronously), to the device that
// is current then; later calls must use the same device.
dg_status dgi::ensure_device(const dg_mesh* cm) {
  dg_mesh* m = const_cast<dg_mesh*>(cm);
  std::lock_guard<std::mutex> lock(m->mu);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (m->on_device) {
    if (dev != m->device) return fail(DG_EINVAL, "mesh was uploaded to another device");
    return DG_OK;
  }
  m->device = dev;
  std::vector<float> tabf(m->t.data.begin(), m->t.data.end());
  std::vector<float> jinvf(m->h.jinv.begin(), m->h.jinv.end());
  std::vector<double> zeros((size_t)m->n_partial * 3, 0.0);
  dg_status s = DG_OK;
  if ((s = upload(m->t.data, &m->d_tab)) != DG_OK || (s = upload(tabf, &m->d_tab_f)) != DG_OK ||
      (s = upload(m->t.spd, &m->d_spd)) != DG_OK ||
      (s = upload(m->h.jinv, &m->d_jinv)) != DG_OK || (s = upload(jinvf, &m->d_jinv_f)) != DG_OK ||
      (s = upload(m->h.absdet, &m->d_absdet)) != DG_OK ||
      (s = upload(m->h.nbr, &m->d_nbr)) != DG_OK ||
      (s = upload(m->h.elem_list, &m->d_elem_list)) != DG_OK ||
      (s = upload(m->h.tile_type, &m->d_tile_type)) != DG_OK ||
      (s = upload(m->h.type_tab, &m->d_type_tab)) != DG_OK ||
      (s = upload(m->h.elem_list16, &m->d_elem_list16)) != DG_OK ||
      (s = upload(m->h.tile_type16, &m->d_tile_type16)) != DG_OK ||
      (!m->h.elem_tab.empty() && (s = upload(m->h.elem_tab, &m->d_elem_tab)) != DG_OK) ||
      (s = upload(zeros, &m->d_partial)) != DG_OK)
    return s;
  {
    std::vector<double> rz((size_t)std::max(m->h.ntiles, m->h.ntiles16) + 4, 0.0);
    std::vector<double> st(4, 0.0);
    double* pst = nullptr;
    if ((s = upload(rz, &m->d_rich_partial)) != DG_OK || (s = upload(st, &pst)) != DG_OK)
      return s;
    m->d_rich_state = pst;
  }
  m->on_device = true;
  return DG_OK;
}

namespace {
using dgi::ensure_device;

void free_mesh(dg_mesh* m) {
  if (!m) return;
  void* ptrs[] = {m->d_tab, m->d_spd, m->d_tab_f, m->d_jinv, m->d_jinv_f, m->d_absdet, m->d_nbr,
                  m->d_elem_list, m->d_tile_type, m->d_type_tab, m->d_elem_tab, m->d_work,
                  m->d_partial, m->d_rich_partial, m->d_rich_state, m->d_elem_list16,
                  m->d_tile_type16, m->d_frag[0], m->d_frag[1], m->d_frag[2], m->d_hfacet,
                  m->d_hfelem, m->d_htab, m->d_hlocal};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
}

// Static scratch of dg_reduce_noalloc: the per-block partial results (3 doubles per block of
// kRedBlock elements), one copy per device, held until the process ends.  In host code the
// array's name is no device address: kernels get the address hipGetSymbolAddress returns for
// the current device (kept per device below).  Every call on one device shares it.
constexpr int kScratchBlocks = 32768;  // meshes of up to 8 388 608 elements (768 KiB)
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchBlocks * 3];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// the device address of this device's scratch, looked up once per device (the device is
// current); no memory is allocated
dg_status scratch_of_device(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(DG_EDEVICE, "no device address for the reduction scratch");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

dg_status check_reduce(const dg_mesh* m, int what, const double* a, const double* b,
                       const double* out_dev) {
  if (!m || !a || !out_dev) return fail(DG_EINVAL, "null pointer");
  if (what < DG_RED_MAXVEL || what > DG_RED_NONFINITE) return fail(DG_EINVAL, "unknown reduction");
  if (what == DG_RED_L2DIFF && !b) return fail(DG_EINVAL, "L2DIFF needs b");
  return DG_OK;
}

// the reductions of dg_reduce with the per-block partial results in `partial` (at least
// 3 n_partial doubles; every block writes its own entries before the final pass reads them,
// so nothing needs clearing)
dg_status run_reduce(const dg_mesh* m, int what, const double* a, const double* b,
                     double* out_dev, double* partial, hipStream_t s) {
  const int nb = m->n_partial, d = m->h.dim;
  if (what == DG_RED_MAXVEL) {
    hipError_t e = hipErrorInvalidValue;
    const int k = m->h.k;
#define DG_CASE(D_, K_) \
  if (d == D_ && k == K_) e = launch_maxvel<D_, K_>(m, a, partial, s);
    DG_CASE(2, 0) DG_CASE(2, 1) DG_CASE(2, 2) DG_CASE(2, 3) DG_CASE(2, 4) DG_CASE(2, 5)
    DG_CASE(2, 6) DG_CASE(3, 0) DG_CASE(3, 1) DG_CASE(3, 2) DG_CASE(3, 3) DG_CASE(3, 4)
#undef DG_CASE
    HIP_TRY(e);
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(kRedBlock), 0, s, nb, 1, 1, 0,
                       partial, out_dev);
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
  const double phi0_vol = d == 2 ? std::sqrt(2.0) * 0.5 : std::sqrt(6.0) / 6.0;
  hipLaunchKernelGGL(elem_reduce_kernel, dim3(nb), dim3(kRedBlock), 0, s, what, d, m->h.np,
                     m->h.E, a, b, m->d_absdet, phi0_vol, partial);
  HIP_TRY(hipGetLastError());
  const int nout = what == DG_RED_MOMENTUM ? d : (what == DG_RED_L2DIFF ? 2 : 1);
  hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(kRedBlock), 0, s, nb, 0, nout,
                     what == DG_RED_L2DIFF ? 1 : 0, partial, out_dev);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

}  // namespace

extern "C" {

const char* dg_last_error(void) { return dgi::g_err.c_str(); }
const char* dg_version(void) { return "dgconv 0.1 gfx950"; }

dg_status dg_mesh_create(int dim, int k, int64_t n_vert, const double* xyz, int64_t n_elem,
                         const int64_t* elem, const double* period, dg_mesh** out) {
  if (!out) return fail(DG_EINVAL, "out is NULL");
  dg_status st = check_k(dim, k);
  if (st != DG_OK) return st;
  if (!xyz || !elem || !period || n_vert <= 0 || n_elem <= 0)
    return fail(DG_EINVAL, "null pointer or empty mesh");
  if (n_elem > (int64_t)0x7fffffff / 64) return fail(DG_EINVAL, "too many elements");
  dg_mesh* m = new (std::nothrow) dg_mesh();
  if (!m) return fail(DG_ENOMEM, "host allocation");
  std::string err;
  const int rc = dgmesh::build(dim, k, n_vert, xyz, n_elem, elem, period, m->h, err);
  if (rc != 0) {
    delete m;
    return fail(rc == -6 ? DG_EMESH : DG_EINVAL, err);
  }
  dgmesh::build_tables(dim, k, m->t);
  m->n_partial = (int)((n_elem + kRedBlock - 1) / kRedBlock);
  {
    // VALU kernel table sources: DGCONV_TABLES = lds | smem | <mask> (bit t: table t through
    // scalar loads; t = basis values, gradients, own traces, neighbour traces, lifts)
    const char* tm = std::getenv("DGCONV_TABLES");
    if (tm) m->tab_src = std::string(tm) == "lds" ? 0 : std::string(tm) == "smem" ? 31 : std::atoi(tm);
    // FP64 kernel, from measurements on MI355X (us per stage launch, VALU / matrix cores):
    // 3D P3 1360 / 575, 2D P3 15.5 / 13.5, 2D P4 49 / 54, 3D P2 809 / 1005.  Matrix cores
    // for elements with >= 20 basis functions and for 2D P3, the VALU kernel otherwise;
    // DGCONV_FP64_KERNEL=valu|mfma overrides
    // Per-lane facet tables (64-wide tiles in element order) when the element classes would
    // leave the class-grouped tiles less than 3/4 full, as on meshes with arbitrary vertex
    // orders, and the facet tables fit in LDS; DGCONV_LANE_TABLES=0|1 overrides
    const double fill = (double)n_elem / (64.0 * std::max(1, m->h.ntiles));
    const bool lane_ok = (m->t.total - m->t.off_tr) * 8 <= 64 * 1024 && m->t.total * 8 <= 100 * 1024;
    const char* lt = std::getenv("DGCONV_LANE_TABLES");
    const bool lane = lane_ok && (lt ? std::string(lt) == "1" : fill < 0.75);
    if (lane) dgmesh::use_lane_tables(m->h);
    // With a given velocity field (frozen or extrapolated) the VALU kernel holds a second
    // set of coefficients and spills from 10 basis functions on (2D P4: 228 us against 84 us
    // per launch on the matrix cores), so that mode takes the matrix cores from there.
    const char* fk = std::getenv("DGCONV_FP64_KERNEL");
    m->fp64_mfma = fk ? std::string(fk) == "mfma"
                      : (m->h.np >= 20 || (dim == 2 && k == 3)) && !lane;
    m->fp64_mfma_frozen = fk ? std::string(fk) == "mfma" : m->h.np >= 10 && !lane;
    // FP64 self-convection on the VALU goes through the pipelined kernel, whose neighbour loads
    // overlap the volume work (2D P4: 47.4 -> 46.5 us per launch, same-box A/B);
    // DGCONV_SELF_PIPE=0 takes the general kernel
    const char* sp = std::getenv("DGCONV_SELF_PIPE");
    m->self_pipe = !(sp && std::string(sp) == "0");
    // Two lanes per element for the 2D FP64 self-convection kernel (P2 to P4) on meshes with
    // fewer than 1024 tiles, which leave SIMDs idle with one lane per element: 2D 16x16x2 P2
    // 7.44 -> 5.36 us per launch.  On full meshes it loses (2D 256x256x2 P4: 43.2 against 41.6
    // us; 2D 128x128x2 P3: 11.2-11.3, as the matrix-core kernel).  DGCONV_PAIR=0|1 overrides
    const char* pr = std::getenv("DGCONV_PAIR");
    m->pair = pr ? std::string(pr) == "1"
                 : dim == 2 && k >= 2 && k <= 4 && m->h.ntiles < 1024 && !lane && m->h.nbf == 0;
  }
  *out = m;
  return DG_OK;
}

dg_status dg_mesh_create_box(int dim, int n, int k, dg_mesh** out) {
  if (dim != 2 && dim != 3) return fail(DG_EINVAL, "dim must be 2 or 3");
  if (n < 1 || n > 4096) return fail(DG_EINVAL, "n out of range");
  std::vector<double> xyz;
  std::vector<int64_t> elem;
  dgmesh::box_connectivity(dim, n, xyz, elem);
  const double period[3] = {1.0, 1.0, 1.0};
  return dg_mesh_create(dim, k, (int64_t)(xyz.size() / dim), xyz.data(),
                        (int64_t)(elem.size() / (dim + 1)), elem.data(), period, out);
}

void dg_mesh_destroy(dg_mesh* mesh) {
  if (!mesh) return;
  if (mesh->on_device) (void)hipDeviceSynchronize();
  free_mesh(mesh);
}

dg_status dg_volume_rule(int dim, int k, int* n_out, double* pts_out, double* wts_out) {
  dg_status st = check_k(dim, k);
  if (st != DG_OK) return st;
  if (!n_out) return fail(DG_EINVAL, "null pointer");
  std::vector<double> p, w;
  dgref::volume_rule<double>(dim, k, p, w);
  *n_out = (int)w.size();
  if (pts_out && wts_out) {
    std::memcpy(pts_out, p.data(), p.size() * sizeof(double));
    std::memcpy(wts_out, w.data(), w.size() * sizeof(double));
  }
  return DG_OK;
}

dg_status dg_facet_rule(int dim, int k, int* n_out, double* pts_out, double* wts_out) {
  dg_status st = check_k(dim, k);
  if (st != DG_OK) return st;
  if (!n_out) return fail(DG_EINVAL, "null pointer");
  std::vector<double> p, w;
  dgref::operator_facet_rule<double>(dim, k, p, w);
  *n_out = (int)w.size();
  if (pts_out && wts_out) {
    std::memcpy(pts_out, p.data(), p.size() * sizeof(double));
    std::memcpy(wts_out, w.data(), w.size() * sizeof(double));
  }
  return DG_OK;
}

dg_status dg_eval_basis(int dim, int k, int64_t n_pts, const double* pts, double* vals,
                        double* grads) {
  dg_status st = check_k(dim, k);
  if (st != DG_OK) return st;
  if (n_pts < 0 || (n_pts > 0 && (!pts || !vals))) return fail(DG_EINVAL, "null pointer");
  const int np = dgref::n_basis(dim, k);
  for (int64_t i = 0; i < n_pts; ++i)
    dgref::eval_basis(dim, k, pts + i * dim, vals + i * np, grads ? grads + i * np * dim : nullptr);
  return DG_OK;
}

dg_status dg_mesh_get_info(const dg_mesh* m, dg_mesh_info* out) {
  if (!m || !out) return fail(DG_EINVAL, "null pointer");
  out->dim = m->h.dim;
  out->k = m->h.k;
  out->n_basis = m->h.np;
  out->n_elem = m->h.E;
  out->n_facet = (m->h.E * (m->h.dim + 1) + m->h.nbf) / 2;
  out->n_bfacet = m->h.nbf;
  out->n_dof = m->h.E * m->h.dim * m->h.np;
  out->nq_vol = m->t.nq;
  out->nq_facet = m->t.nfq;
  out->n_types = m->h.ntypes;
  out->n_tiles = m->h.ntiles;
  out->h_min = m->h.hmin;
  out->volume = m->h.volume;
  return DG_OK;
}

dg_status dg_mesh_get_vertices(const dg_mesh* m, double* xyz_out) {
  if (!m || !xyz_out) return fail(DG_EINVAL, "null pointer");
  std::memcpy(xyz_out, m->h.X.data(), m->h.X.size() * sizeof(double));
  return DG_OK;
}

dg_status dg_mesh_get_neighbors(const dg_mesh* m, int32_t* nbr_out, int32_t* nbr_facet_out) {
  if (!m || !nbr_out || !nbr_facet_out) return fail(DG_EINVAL, "null pointer");
  std::memcpy(nbr_out, m->h.nbr.data(), m->h.nbr.size() * sizeof(int32_t));
  std::memcpy(nbr_facet_out, m->h.nbr_facet.data(), m->h.nbr_facet.size() * sizeof(int32_t));
  return DG_OK;
}

dg_status dg_project_points(const dg_mesh* m, int n, double* xyz_out) {
  if (!m || !xyz_out) return fail(DG_EINVAL, "null pointer");
  if (n < 1 || n > 32) return fail(DG_EINVAL, "n must be in 1..32");
  const int d = m->h.dim, nv = d + 1;
  std::vector<double> p, w;
  dgref::collapsed_rule<double>(d, n, p, w);
  const size_t nq = w.size();
  for (int64_t t = 0; t < m->h.E; ++t) {
    const double* X = &m->h.X[(size_t)t * nv * d];
    for (size_t q = 0; q < nq; ++q)
      for (int i = 0; i < d; ++i) {
        double x = X[i];
        for (int j = 0; j < d; ++j) x += (X[(j + 1) * d + i] - X[i]) * p[q * d + j];
        xyz_out[((size_t)t * nq + q) * d + i] = x;
      }
  }
  return DG_OK;
}

dg_status dg_project(const dg_mesh* m, int n, const double* vals, double* coef_out) {
  if (!m || !vals || !coef_out) return fail(DG_EINVAL, "null pointer");
  if (n < 1 || n > 32) return fail(DG_EINVAL, "n must be in 1..32");
  const int d = m->h.dim, np = m->h.np;
  std::vector<double> p, w;
  dgref::collapsed_rule<double>(d, n, p, w);
  const size_t nq = w.size();
  std::vector<double> phi(nq * np);
  for (size_t q = 0; q < nq; ++q) dgref::eval_basis(d, m->h.k, &p[q * d], &phi[q * np], nullptr);
  // orthonormal reference basis: c_m = int_T^ f phi_m dxi (the |det J| of M_T cancels)
  for (int64_t t = 0; t < m->h.E; ++t)
    for (int i = 0; i < d; ++i)
      for (int mm = 0; mm < np; ++mm) {
        double s = 0;
        for (size_t q = 0; q < nq; ++q) s += w[q] * phi[q * np + mm] * vals[((size_t)t * nq + q) * d + i];
        coef_out[((size_t)t * d + i) * np + mm] = s;
      }
  return DG_OK;
}

namespace {
dg_status apply_common(const dg_mesh* m, dg_precision prec, const void* w, const void* u,
                       void* r, void* stream, const Bnd* bc) {
  if (!m || !w || !r) return fail(DG_EINVAL, "null pointer");
  if (!aligned16(w) || !aligned16(r) || (u && !aligned16(u)))
    return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (r == w || r == u) return fail(DG_EINVAL, "r must not alias w or u");
  if (!known_precision(prec)) return fail(DG_EINVAL, "unknown precision");
  dg_status st = ensure_device(m);
  if (st != DG_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  const int engine = engine_of(m, prec, u != nullptr);
  if (engine >= 0) return run_apply_m(m, engine, w, u, r, s, bc);
  switch (prec) {
    case DG_FP64: return run_apply<double>(m, w, u, r, s, bc);
    case DG_FP32: return run_apply<float>(m, w, u, r, s, bc);
    case DG_MIX_F32: return run_apply<double, float>(m, w, u, r, s, bc);
    default: return fail(DG_EUNSUPPORTED, "precision not available for dg_convection_apply");
  }
}

// the outer values a mesh with boundary facets needs: wb always, ub in frozen mode
dg_status check_bc(const dg_mesh* m, const void* u, const void* wb, const void* ub) {
  if (m->h.nbf == 0) return DG_OK;
  if (!wb) return fail(DG_EINVAL, "the mesh has boundary facets: wb is required");
  if (u && !ub) return fail(DG_EINVAL, "frozen mode on a mesh with boundary facets needs ub");
  return DG_OK;
}
}  // namespace

dg_status dg_convection_apply(const dg_mesh* m, dg_precision prec, const void* w, const void* u,
                              void* r, void* stream) {
  if (m && m->h.nbf > 0)
    return fail(DG_EINVAL, "the mesh has boundary facets: use dg_convection_apply_bc");
  return apply_common(m, prec, w, u, r, stream, nullptr);
}

dg_status dg_convection_apply_bc(const dg_mesh* m, dg_precision prec, const void* w,
                                 const void* u, const void* wb, const void* ub, void* r,
                                 void* stream) {
  if (!m) return fail(DG_EINVAL, "null pointer");
  dg_status st = check_bc(m, u, wb, ub);
  if (st != DG_OK) return st;
  const Bnd bc{wb, ub};
  return apply_common(m, prec, w, u, r, stream, &bc);
}

dg_status dg_boundary_points(const dg_mesh* m, double* xyz_out) {
  if (!m || (!xyz_out && m->h.nbf > 0)) return fail(DG_EINVAL, "null pointer");
  std::vector<double> pts;
  dgmesh::boundary_points(m->h, pts);
  if (!pts.empty()) std::memcpy(xyz_out, pts.data(), pts.size() * sizeof(double));
  return DG_OK;
}

namespace {
dg_status rk_common(const dg_mesh* m, dg_precision prec, void* w, double dt, int n,
                    const void* u, void* work, void* stream, const Extrap* ex,
                    const Bnd* bc = nullptr) {
  if (!m || !w) return fail(DG_EINVAL, "null pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(DG_EINVAL, "dt must be positive and finite");
  if (n < 0) return fail(DG_EINVAL, "n must be >= 0");
  if (!aligned16(w) || (u && !aligned16(u)) || (work && !aligned16(work)))
    return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (u == w) return fail(DG_EINVAL, "u must not alias w");
  if (!known_precision(prec)) return fail(DG_EINVAL, "unknown precision");
  dg_status st = ensure_device(m);
  if (st != DG_OK) return st;
  const int engine = engine_of(m, prec, u != nullptr);
  if (engine >= 0 && (st = ensure_frags(m, engine)) != DG_OK) return st;
  if (!work) {
    // the mesh-owned work buffer (2 states), grown on demand
    std::lock_guard<std::mutex> lock(const_cast<dg_mesh*>(m)->mu);
    const size_t esz = prec == DG_FP32 ? 4 : 8;
    const size_t bytes = 2 * (size_t)m->h.E * m->h.dim * m->h.np * esz + 16;
    if (m->work_bytes < bytes) {
      if (m->d_work) HIP_TRY(hipFree(m->d_work));
      m->d_work = nullptr;
      m->work_bytes = 0;
      HIP_TRY(hipMalloc(&m->d_work, bytes));
      m->work_bytes = bytes;
    }
    work = m->d_work;
  }
  const hipStream_t s = (hipStream_t)stream;
  if (engine >= 0) return run_rk_m(m, engine, w, dt, n, u, work, s, ex, bc);
  if (prec == DG_MIX_F32) return run_rk<double, float>(m, w, dt, n, u, work, s, ex, bc);
  return prec == DG_FP64 ? run_rk<double>(m, w, dt, n, u, work, s, ex, bc)
                         : run_rk<float>(m, w, dt, n, u, work, s, ex, bc);
}
}  // namespace

dg_status dg_rk_substeps(const dg_mesh* m, dg_precision prec, void* w, double dt, int n,
                         const void* u, void* work, void* stream) {
  if (m && m->h.nbf > 0)
    return fail(DG_EINVAL, "the mesh has boundary facets: use dg_rk_substeps_bc");
  return rk_common(m, prec, w, dt, n, u, work, stream, nullptr);
}

dg_status dg_rk_substeps_bc(const dg_mesh* m, dg_precision prec, void* w, double dt, int n,
                            const void* u, const void* wb, const void* ub, void* work,
                            void* stream) {
  if (!m) return fail(DG_EINVAL, "null pointer");
  dg_status st = check_bc(m, u, wb, ub);
  if (st != DG_OK) return st;
  const Bnd bc{wb, ub};
  return rk_common(m, prec, w, dt, n, u, work, stream, nullptr, &bc);
}

dg_status dg_richardson(const dg_mesh* m, dg_precision prec, double* v, const double* g,
                        const double* u, double tau, double ds, double rtol, int max_it,
                        double* work, void* stream, int* iters_out, double* res_out) {
  if (!m || !v || !g || !u) return fail(DG_EINVAL, "null pointer");
  if (m->h.nbf > 0) return fail(DG_EUNSUPPORTED, "the pseudo-time iteration needs a periodic mesh");
  if (!aligned16(v) || !aligned16(g) || !aligned16(u) || (work && !aligned16(work)))
    return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (g == v || u == v || (work && (work == v || work == g || work == u)))
    return fail(DG_EINVAL, "v must not alias g, u or work");
  if (!std::isfinite(tau) || !(ds > 0) || !std::isfinite(ds) || !(rtol >= 0) ||
      !std::isfinite(rtol) || max_it < 0)
    return fail(DG_EINVAL, "need finite tau, ds > 0, rtol >= 0, max_it >= 0");
  if (prec == DG_FP32) return fail(DG_EUNSUPPORTED, "the iteration runs on FP64 states");
  if (!known_precision(prec)) return fail(DG_EINVAL, "unknown precision");
  dg_status st = ensure_device(m);
  if (st != DG_OK) return st;
  const int engine = prec == DG_MIX_F32 ? -2 : engine_of(m, prec, u != nullptr);
  if (engine >= 0 && (st = ensure_frags(m, engine)) != DG_OK) return st;
  if (!work) {
    std::lock_guard<std::mutex> lock(const_cast<dg_mesh*>(m)->mu);
    const size_t bytes = 2 * (size_t)m->h.E * m->h.dim * m->h.np * 8 + 16;
    if (m->work_bytes < bytes) {
      if (m->d_work) HIP_TRY(hipFree(m->d_work));
      m->d_work = nullptr;
      m->work_bytes = 0;
      HIP_TRY(hipMalloc(&m->d_work, bytes));
      m->work_bytes = bytes;
    }
    work = (double*)m->d_work;
  }
  return run_richardson(m, engine, v, g, u, tau, ds, rtol, max_it, work, (hipStream_t)stream,
                        iters_out, res_out);
}

dg_status dg_rk_substeps_extrap(const dg_mesh* m, dg_precision prec, void* w, double dt, int n,
                                double t0, const void* ua, double ta, const void* ub, double tb,
                                void* work, void* stream) {
  if (m && m->h.nbf > 0)
    return fail(DG_EUNSUPPORTED, "extrapolated-velocity substeps need a periodic mesh");
  if (!ua || !ub) return fail(DG_EINVAL, "null velocity field");
  if (ua == w || ub == w) return fail(DG_EINVAL, "velocity fields must not alias w");
  if (!aligned16(ub)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (!std::isfinite(t0) || !std::isfinite(ta) || !std::isfinite(tb) || !(tb != ta))
    return fail(DG_EINVAL, "t0, ta, tb must be finite with tb != ta");
  const Extrap ex{ub, t0, ta, tb};
  return rk_common(m, prec, w, dt, n, ua, work, stream, &ex);
}

dg_status dg_reduce(const dg_mesh* m, int what, const double* a, const double* b,
                    double* out_dev, void* stream) {
  dg_status st = check_reduce(m, what, a, b, out_dev);
  if (st != DG_OK) return st;
  if ((st = ensure_device(m)) != DG_OK) return st;
  return run_reduce(m, what, a, b, out_dev, m->d_partial, (hipStream_t)stream);
}

dg_status dg_reduce_noalloc(const dg_mesh* m, int what, const double* a, const double* b,
                            double* out_dev, void* stream) {
  dg_status st = check_reduce(m, what, a, b, out_dev);
  if (st != DG_OK) return st;
  if (m->n_partial > kScratchBlocks)
    return fail(DG_EINVAL, "mesh too large for dg_reduce_noalloc (at most " +
                               std::to_string((long long)kScratchBlocks * kRedBlock) +
                               " elements)");
  // the mesh tables must be resident already: uploading them would allocate
  if (!m->on_device)
    return fail(DG_EINVAL, "the mesh's device tables are not resident yet (any other compute "
                           "call on this device uploads them)");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != m->device) return fail(DG_EINVAL, "mesh was uploaded to another device");
  double* partial = nullptr;
  if ((st = scratch_of_device(dev, &partial)) != DG_OK) return st;
  return run_reduce(m, what, a, b, out_dev, partial, (hipStream_t)stream);
}

}  // extern "C"
