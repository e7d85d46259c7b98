// CDNA4 (gfx950) matrix-core kernels of the upwind-DG convection operator.
//
// Every basis contraction of the operator is a small dense GEMM whose N dimension runs over
// elements, so one wavefront takes a tile of 16 elements of one element class and runs each
// contraction as 16x16 MFMA blocks (M = quadrature points or basis functions, N = the 16
// elements, K in chunks of 16):
//   volume  W_i = Bv c_i                      (values at the volume points, A1)
//           G_ij = w_i (J^-1 u)_j             (pointwise, A2)
//           R_i += sum_j Dv_j^T G_ij          (test-function contraction, A3)
//   facets  w^-, w^+ = Tr_own c, Tr_nbr c_nbr (traces, own and neighbour side, A4)
//           F = b {w} + |b|/2 [w]             (upwind flux, FP64, A5)
//           R_i -= Lf^T F_i                   (lift, A6)
// The accumulator layout of one 16-row output block is, lane by lane, exactly the B-operand
// layout of a K = 16 chunk in natural row order, so the pointwise results feed the next
// contraction from registers without any data movement.  Table operands (A) are stored on
// the host in per-lane fragment order and read with coalesced loads.
//
// Contraction engines:
//   EngF64        v_mfma_f64_16x16x4 (four per K = 16 chunk); the FP64 path.
//   EngSplit<..>  v_mfma_f32_16x16x16 on FP16 or BF16 pieces: x = x0 + x1 (+ x2) split by
//                 successive rounding, products x_a y_b with a + b < pieces (3 or 6 MFMAs),
//                 FP32 accumulation inside one K chunk.  Across K chunks the facet lifts are
//                 folded into FP64 accumulators (mma_into), while the volume interpolation W
//                 and the volume test contraction Rv keep accumulating in FP32 (mma_acc) and
//                 reach FP64 only when the volume term is added to R.  FP16 operands are
//                 scaled per element and chunk by a power of two so the largest magnitude
//                 sits in [1, 2).  The flux, the facet sums, the state and the Runge-Kutta
//                 update stay FP64.
#pragma once
#include <hip/hip_runtime.h>

#include "conv_kernels.hpp"

namespace dgm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

template <int D, int K>
struct MShape {
  using S = dgk::Shape<D, K>;
  static constexpr int NP = S::NP, NQ = S::NQ, NFQ = S::NFQ, NTAB = S::NTAB;
  static constexpr int KP = (NP + 15) / 16;  // 16-chunks over the basis index (= m tiles)
  static constexpr int QT = (NQ + 15) / 16;  // volume point tiles
  static constexpr int FT = (NFQ + 15) / 16; // facet point tiles
  // fragment blocks: one block = a 16 x 16 piece of a table in A-operand lane order
  static constexpr int OFF_BV = 0;                       // [qt][kc]      Bv
  static constexpr int OFF_DV = OFF_BV + QT * KP;        // [j][mt][qt]   Dv_j^T (weights in)
  static constexpr int OFF_TR = OFF_DV + D * KP * QT;    // [tab][ft][kc] traces
  static constexpr int OFF_LF = OFF_TR + NTAB * FT * KP; // [tab][mt][ft] -(lift)^T
  static constexpr int NBLK = OFF_LF + NTAB * KP * FT;
};

// ------------------------------------------------------------------ engines
struct EngF64 {
  static constexpr bool SPLIT = false;
  static constexpr bool SCALED = false;
  static constexpr int BLK = 256;  // doubles per fragment block
  struct frag { double v[4]; };
  // K index (within a 16-chunk) of B element j in lane group g; row of accumulator reg r
  __device__ static __forceinline__ int kidx(int g, int j) { return 4 * j + g; }
  __device__ static __forceinline__ int row(int g, int r) { return g + 4 * r; }
  // nk: K sub-chunks of 4 (of the chunk's 4) that hold rows inside the contraction; the
  // rest are zero padding on both operands and are neither loaded nor multiplied
  __device__ static __forceinline__ frag load_a(const void* base, int blk, int lane, int nk = 4) {
    const double* p = (const double*)base + (size_t)blk * BLK;
    frag f;
#pragma unroll
    for (int j = 0; j < 4; ++j) f.v[j] = j < nk ? p[j * 64 + lane] : 0.0;
    return f;
  }
  template <typename V>
  __device__ static __forceinline__ frag make_b(const V (&x)[4], int& e) {
    frag f;
#pragma unroll
    for (int j = 0; j < 4; ++j) f.v[j] = (double)x[j];
    e = 0;
    return f;
  }
  // acc += A B  (double accumulator); nk is wave-uniform, so every lane takes each MFMA
  __device__ static __forceinline__ void mma(d4& acc, const frag& a, const frag& b, int nk = 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nk) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[j], b.v[j], acc, 0, 0, 0);
  }
};

template <bool F16, int NS>
struct EngSplit {
  static constexpr bool SPLIT = true;
  static constexpr bool SCALED = F16;  // power-of-two operand scaling (FP16 range)
  typedef typename std::conditional<F16, h4, s4>::type h_t;
  static constexpr int BLK = NS * 64;  // h_t (8 bytes) per fragment block
  struct frag { h_t p[NS]; };
  __device__ static __forceinline__ int kidx(int g, int j) { return 4 * g + j; }
  __device__ static __forceinline__ int row(int g, int r) { return 4 * g + r; }
  __device__ static __forceinline__ frag load_a(const void* base, int blk, int lane, int = 4) {
    const h_t* p = (const h_t*)base + (size_t)blk * BLK;
    frag f;
#pragma unroll
    for (int s = 0; s < NS; ++s) f.p[s] = p[s * 64 + lane];
    return f;
  }
  // one 16-bit piece of v, rounded toward zero (hardware conversion); the residual v - back
  // is exact, so the pieces together carry 11 (FP16) or 8 (BF16) more bits each
  __device__ static __forceinline__ short to_piece(float v, float& back) {
    if constexpr (F16) {
      const auto h2 = __builtin_amdgcn_cvt_pkrtz(v, 0.0f);
      back = (float)h2[0];
      return __builtin_bit_cast(short, h2[0]);
    } else {
      const unsigned u = __float_as_uint(v) & 0xffff0000u;
      back = __uint_as_float(u);
      return (short)(u >> 16);
    }
  }
  // split 4 values into pieces; FP16 values are first scaled by 2^-e, e the exponent of the
  // largest magnitude over the element's column (the 4 lane groups), so they sit in [1, 2)
  template <typename V>
  __device__ static __forceinline__ frag make_b(const V (&x)[4], int& e) {
    e = 0;
    if constexpr (F16) {
      float m = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) m = fmaxf(m, fabsf((float)x[j]));
      m = fmaxf(m, __shfl_xor(m, 16));
      m = fmaxf(m, __shfl_xor(m, 32));
      e = m > 0.f ? __builtin_amdgcn_frexp_expf(m) - 1 : 0;
    }
    frag f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      V r = F16 ? (V)ldexp(x[j], -e) : x[j];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        float back;
        const short pc = to_piece((float)r, back);
        r = r - (V)back;
        if constexpr (F16) f.p[s][j] = __builtin_bit_cast(_Float16, pc);
        else f.p[s][j] = pc;
      }
    }
    return f;
  }
  __device__ static __forceinline__ f4 mm(const h_t& a, const h_t& b, f4 acc) {
    if constexpr (F16) return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  // acc += A B over the product terms a + b < NS (smallest first); K = 16 per instruction
  __device__ static __forceinline__ void mma(f4& acc, const frag& a, const frag& b, int = 4) {
    if constexpr (NS == 3) {
      acc = mm(a.p[1], b.p[1], acc);
      acc = mm(a.p[0], b.p[2], acc);
      acc = mm(a.p[2], b.p[0], acc);
    }
    acc = mm(a.p[0], b.p[1], acc);
    acc = mm(a.p[1], b.p[0], acc);
    acc = mm(a.p[0], b.p[0], acc);
  }
};

template <class E>
struct AccOf { typedef f4 type; };
template <>
struct AccOf<EngF64> { typedef d4 type; };

// number of 4-row K sub-chunks of a 16-row chunk that hold rows below n_valid (n_valid = the
// contraction length minus the chunk's first row)
__device__ __forceinline__ constexpr int nk_of(int n_valid) {
  return n_valid >= 16 ? 4 : n_valid <= 0 ? 0 : (n_valid + 3) / 4;
}

// one K-chunk product folded into an FP64 accumulator: out[r] += 2^e (A B)[r]
template <class E>
__device__ __forceinline__ void mma_into(double (&out)[4], const typename E::frag& a,
                                         const typename E::frag& b, int e, int nk = 4) {
  if constexpr (!E::SPLIT) {
    d4 acc = {out[0], out[1], out[2], out[3]};  // FP64: chain directly in the accumulator
    E::mma(acc, a, b, nk);
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = acc[r];
  } else {
    f4 acc = {0, 0, 0, 0};
    E::mma(acc, a, b);
    const double sc = e ? ldexp(1.0, e) : 1.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = fma((double)acc[r], sc, out[r]);
  }
}

// one K-chunk product accumulated in the engine's value type: out[r] += 2^e (A B)[r]
// (FP32 for the split engines; chained in the accumulator when the engine never scales).
// The choice is made at compile time: a branch on the per-element scale would diverge
// around a matrix instruction, which must run with every lane active.
template <class E, typename V>
__device__ __forceinline__ void mma_acc(V (&out)[4], const typename E::frag& a,
                                        const typename E::frag& b, int e, int nk = 4) {
  if constexpr (!E::SPLIT) {
    mma_into<E>(out, a, b, e, nk);
  } else {
    if constexpr (!E::SCALED) {
      f4 acc = {out[0], out[1], out[2], out[3]};
      E::mma(acc, a, b);
#pragma unroll
      for (int r = 0; r < 4; ++r) out[r] = acc[r];
    } else {
      f4 acc = {0, 0, 0, 0};
      E::mma(acc, a, b);
      const float sc = __builtin_amdgcn_ldexpf(1.0f, e);
#pragma unroll
      for (int r = 0; r < 4; ++r) out[r] = fmaf(acc[r], sc, out[r]);
    }
  }
}

template <typename T>
struct MArgs {
  const double* x;       // state the operator acts on
  const double* u;       // frozen convecting velocity or nullptr
  const double* wb;      // outer values at the boundary facet points [nbf][NFQ][D] (or nullptr)
  const double* ub;      // outer convecting velocity there (frozen mode)
  const double* u2;      // second velocity field or nullptr: u(s) = u + uth (u2 - u)
  const double* w0;      // Runge-Kutta base state (mode 1, a != 0)
  double* out;
  const void* frag;      // fragment tables (engine layout)
  const double* jinv;    // [E][D][D]
  const int* nbr;        // [E][D+1]
  const int* elem_list;  // [ntiles*16], -1 padded
  const int* tile_type;  // [ntiles], -1 = empty tile
  const int* type_tab;   // [ntypes][D+1]
  int ntiles;
  int mode;              // 0: r;  1: Runge-Kutta stage;  2: pseudo-time (Richardson) update
  double a, b, dt;
  double uth;            // time weight of u2 (extrapolated convecting velocity)
  // mode 2 as in the VALU kernel: res = g - x + tau r, out = x + ds res, tile sums of
  // |det J| res^2 into partial[tile]; skipped when *stop != 0
  double tau, ds;
  const double* absdet;
  double* partial;
  const int* stop;
};

// B fragments of a state block: element n, component i, K chunk kc
template <class E, int D, int NP>
__device__ __forceinline__ typename E::frag state_frag(const double* p, int i, int kc, int g,
                                                       int& e) {
  double v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 16 * kc + E::kidx(g, j);
    v[j] = k < NP ? p[i * NP + k] : 0.0;
  }
  return E::make_b(v, e);
}

// B fragments of a velocity block, u + th (u2 - u) when a second field is given
template <class E, int D, int NP>
__device__ __forceinline__ typename E::frag vel_frag(const double* p, const double* p2, double th,
                                                     int i, int kc, int g, int& e) {
  double v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 16 * kc + E::kidx(g, j);
    v[j] = k < NP ? p[i * NP + k] : 0.0;
    if (p2 && k < NP) v[j] = fma(th, p2[i * NP + k] - v[j], v[j]);
  }
  return E::make_b(v, e);
}

// occupancy target: two waves per SIMD (<= 256 registers per lane), which the compiler meets
// without spilling below 35 basis functions in self mode and below 20 with a separate
// velocity field; larger elements keep one
template <int D, int K, bool SELF>
constexpr int mconv_min_waves() { return dgk::Shape<D, K>::NP >= (SELF ? 35 : 20) ? 1 : (D == 2 && SELF && dgk::Shape<D, K>::NP <= 15 ? 3 : 2); }

template <int D, int K, class E, bool SELF, bool BND>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mconv_min_waves<D, K, SELF>(), 8)))
mconv_kernel(MArgs<double> A) {
  using M = MShape<D, K>;
  constexpr int NP = M::NP, KP = M::KP;
  typedef typename std::conditional<E::SPLIT, float, double>::type V;  // pointwise volume type
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15;
  const int blk = dgk::xcd_block(blockIdx.x, gridDim.x);
  const int tile = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
  if (dgk::stopped(A.stop)) return;  // uniform over the grid
  // fragment tables small enough are staged in LDS once per workgroup (every wave of the
  // block takes part before any of them may leave), larger ones are read from L2
  constexpr size_t kFragBytes = (size_t)M::NBLK * E::BLK * 8;
  constexpr bool kFragLds = kFragBytes <= 48 * 1024;
  __shared__ __attribute__((aligned(16))) char sfrag[kFragLds ? kFragBytes : 16];
  const void* fr = A.frag;
  if constexpr (kFragLds) {
    const uint4* src = (const uint4*)A.frag;
    uint4* dst = (uint4*)sfrag;
    for (int i = threadIdx.x; i < (int)(kFragBytes / 16); i += 256) dst[i] = src[i];
    __syncthreads();
    fr = sfrag;
  }
  const int type = __builtin_amdgcn_readfirstlane(A.tile_type[tile]);
  if (type < 0) {
    if (A.mode == 2 && lane == 0) A.partial[tile] = 0.0;
    return;
  }
  const int e_raw = A.elem_list[tile * 16 + n];
  const int e = e_raw >= 0 ? e_raw : A.elem_list[tile * 16];
  const double* px = A.x + (size_t)e * D * NP;
  const double* pu = SELF ? px : A.u + (size_t)e * D * NP;
  double ji[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int j = 0; j < D; ++j) ji[a][j] = A.jinv[(size_t)e * D * D + a * D + j];

  double R[D][KP][4];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int mt = 0; mt < KP; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) R[i][mt][r] = 0.0;

  // state fragments (own), kept for the volume and the own traces
  typename E::frag cB[D][KP], uB[SELF ? 1 : D][SELF ? 1 : KP];
  int ce[D][KP], ue[SELF ? 1 : D][SELF ? 1 : KP];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int kc = 0; kc < KP; ++kc) {
      cB[i][kc] = state_frag<E, D, NP>(px, i, kc, g, ce[i][kc]);
      if constexpr (!SELF)
        uB[i][kc] = vel_frag<E, D, NP>(pu, A.u2 ? A.u2 + (size_t)e * D * NP : nullptr, A.uth,
                                       i, kc, g, ue[i][kc]);
    }

  // neighbour fragments: in 2D all facets' are loaded up front so the gathers overlap the
  // volume work; in 3D (larger fragments) each facet loads its own just before use
  typedef const int __attribute__((address_space(4)))* ciptr;
  const ciptr ttab = (ciptr)A.type_tab;
  constexpr int NPF = (D == 2 && SELF) ? D + 1 : 1;
  typename E::frag nB[NPF][D][KP], nuB[SELF ? 1 : NPF][SELF ? 1 : D][SELF ? 1 : KP];
  int nce[NPF][D][KP], nue[SELF ? 1 : NPF][SELF ? 1 : D][SELF ? 1 : KP];
  auto load_nbr = [&](int f, int slot) {
    // a boundary facet has no neighbour: the own element stands in (its traces are replaced
    // by the boundary data below)
    const int ne_raw = A.nbr[(size_t)e * (D + 1) + f];
    const int ne = (BND && ne_raw < 0) ? e : ne_raw;
    const double* pnx = A.x + (size_t)ne * D * NP;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int kc = 0; kc < KP; ++kc) {
        nB[slot][i][kc] = state_frag<E, D, NP>(pnx, i, kc, g, nce[slot][i][kc]);
        if constexpr (!SELF)
          nuB[slot][i][kc] =
              vel_frag<E, D, NP>(A.u + (size_t)ne * D * NP,
                                 A.u2 ? A.u2 + (size_t)ne * D * NP : nullptr, A.uth, i, kc, g,
                                 nue[slot][i][kc]);
      }
  };
  if constexpr (NPF > 1) {
#pragma unroll
    for (int f = 0; f <= D; ++f) load_nbr(f, f);
  }

  // ---------------- volume (in V: FP64 on the f64 engine, FP32 on the split engines)
  V ji_v[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int j = 0; j < D; ++j) ji_v[a][j] = (V)ji[a][j];
  // 2D: one accumulator set per gradient direction a, so the test contraction runs 2 D
  // independent MFMA chains instead of D (summed after the loop)
  constexpr int NA = D == 2 ? D : 1;
  V Rv[NA][D][KP][4];
#pragma unroll
  for (int b = 0; b < NA; ++b)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int mt = 0; mt < KP; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) Rv[b][i][mt][r] = V(0);
#pragma unroll(M::QT <= 4 ? M::QT : 1)
  for (int qt = 0; qt < M::QT; ++qt) {
    V W[D][4], U[SELF ? 1 : D][4];
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        W[i][r] = V(0);
        if constexpr (!SELF) U[i][r] = V(0);
      }
#pragma unroll
      for (int kc = 0; kc < KP; ++kc) {
        const int nkc = nk_of(NP - 16 * kc);
        const auto a = E::load_a(fr, M::OFF_BV + qt * KP + kc, lane, nkc);
        mma_acc<E>(W[i], a, cB[i][kc], ce[i][kc], nkc);
        if constexpr (!SELF) mma_acc<E>(U[i], a, uB[i][kc], ue[i][kc], nkc);
      }
    }
    // pointwise: G_ij = w_i (J^-1 u)_j at the 4 points this lane holds
    V G[D][D][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      V uh[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        V s = V(0);
#pragma unroll
        for (int j = 0; j < D; ++j) s = fma(ji_v[a][j], SELF ? W[j][r] : U[j][r], s);
        uh[a] = s;
      }
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int a = 0; a < D; ++a) G[i][a][r] = W[i][r] * uh[a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      typename E::frag gB[D];
      int ge[D];
#pragma unroll
      for (int i = 0; i < D; ++i) gB[i] = E::make_b(G[i][a], ge[i]);
#pragma unroll
      for (int mt = 0; mt < KP; ++mt) {
        const int nkq = nk_of(M::NQ - 16 * qt);
        const auto af = E::load_a(fr, M::OFF_DV + (a * KP + mt) * M::QT + qt, lane, nkq);
#pragma unroll
        for (int i = 0; i < D; ++i) mma_acc<E>(Rv[NA > 1 ? a : 0][i][mt], af, gB[i], ge[i], nkq);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int mt = 0; mt < KP; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < NA; ++b) acc += (double)Rv[b][i][mt][r];
        R[i][mt][r] = acc;
      }

  // ---------------- facets
#pragma unroll(D == 2 ? D + 1 : 1)
  for (int f = 0; f <= D; ++f) {
    const int tt = ttab[type * (D + 1) + f];
    const int own = __builtin_amdgcn_readfirstlane(tt & 0xffff);
    const int nbt = __builtin_amdgcn_readfirstlane(tt >> 16);
    const int slot = NPF > 1 ? f : 0;
    if constexpr (NPF == 1) load_nbr(f, 0);
    const bool bnd = BND && nbt == dgk::kBoundaryTable;  // uniform: the class fixes it
    const int nbt_tab = bnd ? own : nbt;  // a valid table for the discarded neighbour product
    double Nt[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) s = fma(ji[a][j], dgk::nref<D, double>(f, a), s);
      Nt[j] = s;
    }
#pragma unroll(M::FT)
    for (int ft = 0; ft < M::FT; ++ft) {
      V wm[D][4], wp[D][4], um[SELF ? 1 : D][4], up[SELF ? 1 : D][4];
#pragma unroll
      for (int i = 0; i < D; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          wm[i][r] = V(0);
          wp[i][r] = V(0);
          if constexpr (!SELF) { um[i][r] = V(0); up[i][r] = V(0); }
        }
#pragma unroll
        for (int kc = 0; kc < KP; ++kc) {
          const int nkc = nk_of(NP - 16 * kc);
          const auto ao = E::load_a(fr, M::OFF_TR + (own * M::FT + ft) * KP + kc, lane, nkc);
          const auto an = E::load_a(fr, M::OFF_TR + (nbt_tab * M::FT + ft) * KP + kc, lane, nkc);
          mma_acc<E>(wm[i], ao, cB[i][kc], ce[i][kc], nkc);
          mma_acc<E>(wp[i], an, nB[slot][i][kc], nce[slot][i][kc], nkc);
          if constexpr (!SELF) {
            mma_acc<E>(um[i], ao, uB[i][kc], ue[i][kc], nkc);
            mma_acc<E>(up[i], an, nuB[slot][i][kc], nue[slot][i][kc], nkc);
          }
        }
      }
      if (bnd) {
        // outer values from the boundary data, rows q = 16 ft + row(g, r) of this lane
        const size_t bf = (size_t)(-1 - A.nbr[(size_t)e * (D + 1) + f]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 16 * ft + E::row(g, r);
#pragma unroll
          for (int i = 0; i < D; ++i) {
            wp[i][r] = q < M::NFQ ? (V)A.wb[(bf * M::NFQ + q) * D + i] : V(0);
            if constexpr (!SELF) up[i][r] = q < M::NFQ ? (V)A.ub[(bf * M::NFQ + q) * D + i] : V(0);
          }
        }
      }
      // upwind flux in FP64; rows beyond the facet rule carry zero traces and zero flux
      double F[D][4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double bb = 0;
#pragma unroll
        for (int j = 0; j < D; ++j)
          bb = fma(SELF ? (double)wm[j][r] + (double)wp[j][r]
                        : (double)um[j][r] + (double)up[j][r], Nt[j], bb);
        const double hb = 0.25 * bb, ha = 0.25 * fabs(bb);
#pragma unroll
        for (int i = 0; i < D; ++i) {
          const double a = wm[i][r], b = wp[i][r];
          F[i][r] = hb * (a + b) + ha * (a - b);
        }
      }
      typename E::frag fB[D];
      int fe[D];
#pragma unroll
      for (int i = 0; i < D; ++i) fB[i] = E::make_b(F[i], fe[i]);
#pragma unroll
      for (int mt = 0; mt < KP; ++mt) {
        const int nkf = nk_of(M::NFQ - 16 * ft);
        const auto al = E::load_a(fr, M::OFF_LF + (own * KP + mt) * M::FT + ft, lane, nkf);
#pragma unroll
        for (int i = 0; i < D; ++i) mma_into<E>(R[i][mt], al, fB[i], fe[i], nkf);
      }
    }
  }

  // ---------------- epilogue: rows m = 16 mt + row(g, r) of element n
  double* o = A.out + (size_t)e * D * NP;
  if (A.mode == 2) {
    // rows m of element n held by this lane; padded lanes store nothing and add zero
    const double* pg = A.w0 + (size_t)e * D * NP;
    double gv[D][KP][4], cv[D][KP][4];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int mt = 0; mt < KP; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = 16 * mt + E::row(g, r);
          gv[i][mt][r] = m < NP ? pg[i * NP + m] : 0.0;
          cv[i][mt][r] = m < NP ? px[i * NP + m] : 0.0;
        }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int mt = 0; mt < KP; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = 16 * mt + E::row(g, r);
          if (m < NP) {
            const double res = fma(A.tau, R[i][mt][r], gv[i][mt][r] - cv[i][mt][r]);
            if (e_raw >= 0) o[i * NP + m] = fma(A.ds, res, cv[i][mt][r]);
            acc = fma(res, res, acc);
          }
        }
    acc = dgk::wave_sum(e_raw >= 0 ? acc * A.absdet[e] : 0.0);
    if (lane == 0) A.partial[tile] = acc;
    return;
  }
  if (e_raw < 0) return;
  if (A.mode == 0) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int mt = 0; mt < KP; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = 16 * mt + E::row(g, r);
          if (m < NP) o[i * NP + m] = R[i][mt][r];
        }
    return;
  }
  double cv[D][KP][4], wv[D][KP][4];
  const double* pw = A.w0 + (size_t)e * D * NP;
  const bool has_w0 = A.a != 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int mt = 0; mt < KP; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * mt + E::row(g, r);
        cv[i][mt][r] = m < NP ? px[i * NP + m] : 0.0;
        wv[i][mt][r] = (m < NP && has_w0) ? pw[i * NP + m] : 0.0;
      }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int mt = 0; mt < KP; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * mt + E::row(g, r);
        if (m < NP) o[i * NP + m] = fma(A.a, wv[i][mt][r], A.b * fma(A.dt, R[i][mt][r], cv[i][mt][r]));
      }
}

}  // namespace dgm
