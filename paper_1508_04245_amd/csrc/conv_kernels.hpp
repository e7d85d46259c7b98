// CDNA4 (gfx950) kernels of the upwind-DG convection operator, plain FP64 / FP32 path.
//
// One lane per element, one wavefront per 64-element tile of a single element class
// (identical facet tables), so every table entry a lane needs is wave-uniform.  A workgroup
// (4 wavefronts) covers one block of 256 consecutive elements, so all writes to a cache line
// of the state come from one CU, and hardware blocks are remapped so that each XCD (blocks
// are dealt round-robin over the 8 XCDs) works on one contiguous range of the mesh and finds
// most neighbour states in its own L2.  Each reference table is read either from LDS (staged
// per workgroup when the tables fit in 64 KiB; wave-uniform broadcast reads) or through a
// constant-address-space pointer (scalar loads into SGPRs); the split is chosen per element
// type so that neither the LDS return path nor the scalar loads' latency dominates.  Each
// multiply-add of a basis contraction is one VALU FMA.  The per-element state, the neighbour
// states and the accumulators stay in VGPRs.
//
// Per element and application (Sec. 2.3 upwind form, Sec. 2.4 discrete operator, inverse of
// the diagonal mass matrix folded in):
//   volume:  R[i][m] += sum_q w_i(x_q) (uh(x_q) . w_q grad^ phi_m(x_q)),  uh = J^-1 u
//   facets:  R[i][m] -= sum_f sum_q w^F_q phi_m(x_q) [ b {w_i} + |b|/2 [w_i] ],
//            b = 1/2 (u^- + u^+) . (J^-T n^_f |F^_f|)   (= beta |F| / |det J|)
//   r = R   (the orthonormal reference basis makes M_T = |det J| I, which cancels)
// and, in the fused Runge-Kutta mode, out = a w0 + b (x + dt r) for the stage of SSP-RK3.
//
// Two arithmetic types: TS for the state, the facet flux, the facet sums and the update, TC for
// the basis contractions (coefficients and tables as TC, products and the volume sums in TC).
// TS = TC = double is the FP64 path and TS = TC = float the FP32 path; TS = double with
// TC = float keeps the state, the flux, the lifted facet sums and the Runge-Kutta update in
// FP64 around FP32 contractions (the volume sums reach FP64 once, when the volume term is
// added to R).
#pragma once
#include <hip/hip_runtime.h>

#include "sym_rules.hpp"

namespace dgk {

template <int D, int K>
struct Shape {
  static constexpr int NP = D == 2 ? (K + 1) * (K + 2) / 2 : (K + 1) * (K + 2) * (K + 3) / 6;
  // collapsed rule exact to 3k-1: NV1 points per direction, NS in all (the points of the
  // speed reduction); the volume rule is the symmetric one with fewer points where it exists
  static constexpr int NV1 = (3 * K + 1) / 2 < 1 ? 1 : (3 * K + 1) / 2;
  static constexpr int NS = D == 2 ? NV1 * NV1 : NV1 * NV1 * NV1;
  static constexpr int NQ = dgref::sym_vol_points(D, K) > 0 ? dgref::sym_vol_points(D, K) : NS;
  // facet rule exact to 3k: NF1 Gauss points on an edge; on a triangle the symmetric rule
  // where there is one, else NF1^2 collapsed points
  static constexpr int NF1 = (3 * K + 2) / 2 < 1 ? 1 : (3 * K + 2) / 2;
  static constexpr int NFQ = D == 2 ? NF1
                                    : (dgref::sym_facet_points(K) > 0 ? dgref::sym_facet_points(K)
                                                                      : NF1 * NF1);
  static constexpr int NPERM = D == 2 ? 2 : 6;
  static constexpr int NTAB = (D + 1) * NPERM;
  static constexpr int OFF_BV = 0;
  static constexpr int OFF_DV = NQ * NP;
  static constexpr int OFF_TR = OFF_DV + NQ * NP * D;
  static constexpr int OFF_LF = OFF_TR + NTAB * NFQ * NP;
  static constexpr int TOTAL = OFF_LF + NTAB * NFQ * NP;
};

template <typename T, typename TC = T>
struct ConvArgs {
  const T* x;          // state the operator acts on (neighbour traces are read from it)
  const T* u;          // frozen convecting velocity, or nullptr (u := x)
  const T* wb;         // outer values at the boundary facet points [nbf][NFQ][D] (or nullptr)
  const T* ub;         // outer convecting velocity there (frozen mode)
  const T* u2;         // second velocity field or nullptr: u(s) = u + uth (u2 - u)
  const T* w0;         // Runge-Kutta base state (mode 1, a != 0)
  T* out;              // mode 0: r;  mode 1: a w0 + b (x + dt r)
  const TC* tab;       // reference tables (Shape offsets), in the contraction type
  const T* jinv;       // [E][D][D]
  const int* nbr;      // [E][D+1]
  const int* elem_list;// [ntiles*64], -1 padded
  const int* tile_type;// [ntiles]
  const int* type_tab; // [ntypes][D+1]: own table | nbr table << 16
  const int* elem_tab; // [E][D+1]: the same per element (per-lane table mode)
  int ntiles;
  int mode;            // 0: r;  1: Runge-Kutta stage;  2: pseudo-time (Richardson) update
  T a, b, dt;
  T uth;               // time weight of u2 (extrapolated convecting velocity)
  // mode 2: res = g - x + tau r (g passed as w0), out = x + ds res, and per tile the sum
  // over its elements of |det J| sum res^2 into partial[tile]; skipped when *stop != 0
  T tau, ds;
  const double* absdet;
  double* partial;
  const int* stop;
};

// mode 2 (pseudo-time iteration): sum over the wave of the per-lane partial sums, in a fixed
// butterfly order (deterministic); every lane of the wave must take part
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// stop flag of an iteration driven from the host (nullptr: none); read once per launch
__device__ __forceinline__ bool stopped(const int* flag) {
  return flag && *(const int __attribute__((address_space(4)))*)flag != 0;
}


// scaled outward reference normal n^_f |F^_f| of local facet f (opposite vertex f)
template <int D, typename T>
__device__ __forceinline__ T nref(int f, int j) {
  if (f == 0) return D == 2 ? T(1) : T(0.5);
  return j == f - 1 ? (D == 2 ? T(-1) : T(-0.5)) : T(0);
}

// tables fit in LDS (bytes)
template <int D, int K, typename T>
constexpr bool tables_in_lds() { return Shape<D, K>::TOTAL * sizeof(T) <= 65536; }

// hardware block -> logical block: XCD x = b % 8 gets the contiguous logical range
// [x q + min(x, r), ...) of q + (x < r) blocks, q = n / 8, r = n % 8 (a bijection of [0, n))
__device__ __forceinline__ int xcd_block(int b, int n) {
  const int x = b & 7, j = b >> 3, q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + j;
}

// Source of each reference table: bit t of the mask set = table t is read through a
// constant-address-space pointer (wave-uniform scalar loads into SGPRs, one copy per wave),
// clear = staged in LDS and read with broadcast addresses (the LDS returns the value to every
// lane, so those reads cost LDS bandwidth per lane).  Splitting the tables between the two
// paths keeps the LDS return bandwidth below the FP64 FMA rate.
enum { TB_BV = 0, TB_DV = 1, TB_TRO = 2, TB_TRN = 3, TB_LF = 4 };
// neighbour-table index that marks a boundary facet in the per-class facet table list
constexpr int kBoundaryTable = 0x7fff;
constexpr int SM_ALL = 31;

// [lo, hi): the part of the table block staged in LDS for source mask SM (the staged tables
// in block order; both trace tables share one range)
template <int D, int K, int SM>
constexpr int staged_lo() {
  using S = Shape<D, K>;
  const bool tr = !((SM >> TB_TRO) & 1) || !((SM >> TB_TRN) & 1);
  return !((SM >> TB_BV) & 1) ? S::OFF_BV : !((SM >> TB_DV) & 1) ? S::OFF_DV
         : tr ? S::OFF_TR : !((SM >> TB_LF) & 1) ? S::OFF_LF : 0;
}
template <int D, int K, int SM>
constexpr int staged_hi() {
  using S = Shape<D, K>;
  const bool tr = !((SM >> TB_TRO) & 1) || !((SM >> TB_TRN) & 1);
  return !((SM >> TB_LF) & 1) ? S::TOTAL : tr ? S::OFF_LF : !((SM >> TB_DV) & 1) ? S::OFF_TR
         : !((SM >> TB_BV) & 1) ? S::OFF_DV : 0;
}

// the tables mask SM stages fit in 64 KiB of LDS
template <int D, int K, typename T, int SM>
constexpr bool staged_fits() {
  return (size_t)(staged_hi<D, K, SM>() - staged_lo<D, K, SM>()) * sizeof(T) <= 65536;
}

// LO: table index of the first staged value (the LDS copy holds [LO, hi) only)
template <int SM, typename T, int LO = 0>
struct Tabs {
  typedef const T __attribute__((address_space(4)))* cptr;
  const T* l;
  cptr c;
  template <int ID>
  __device__ __forceinline__ T get(int i) const {
    if constexpr ((SM >> ID) & 1) return c[i];
    else return l[i - LO];
  }
};

// stage the LDS-sourced tables (contiguous ranges of the table block) into LDS
template <int D, int K, int SM, typename T>
__device__ __forceinline__ void stage_tables(T* stab, const T* tab) {
  using S = Shape<D, K>;
  constexpr int LO = staged_lo<D, K, SM>();
  constexpr int beg[5] = {S::OFF_BV, S::OFF_DV, S::OFF_TR, S::OFF_TR, S::OFF_LF};
  constexpr int end[5] = {S::OFF_DV, S::OFF_TR, S::OFF_LF, S::OFF_LF, S::TOTAL};
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    if (t == TB_TRN && !((SM >> TB_TRO) & 1)) continue;  // same range as the own traces
    if ((SM >> t) & 1) continue;
    for (int i = beg[t] + (int)threadIdx.x; i < end[t]; i += 256) stab[i - LO] = tab[i];
  }
}

// occupancy target: two waves per SIMD (<= 256 VGPR+AGPR per lane) where the state fits
template <int D, int K, typename T>
constexpr int min_waves() { return Shape<D, K>::NP * D * sizeof(T) <= 15 * 2 * 8 ? 2 : 1; }

// LANE: tiles of consecutive elements whatever their classes, each lane reading its own facet
// tables (from LDS, per-lane addresses; an LDS read returns 8 bytes to each lane either way,
// so this costs no more LDS bandwidth than a broadcast read), for meshes whose classes would
// leave class-grouped tiles mostly empty.  Boundary facets are then selected per lane.
template <int D, int K, typename T>
constexpr bool lane_tables_ok() {
  return (size_t)(Shape<D, K>::TOTAL - Shape<D, K>::OFF_TR) * sizeof(T) <= 64 * 1024 &&
         (size_t)Shape<D, K>::TOTAL * sizeof(T) <= 100 * 1024;
}

template <int D, int K, typename TS, bool SELF, int SM, bool BND, bool LANE = false,
          typename T = TS>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(min_waves<D, K, T>(), 8))) conv_kernel(ConvArgs<TS, T> A) {
  // T: contraction type (coefficients, tables, volume sums); TS: state, flux, facet sums
  using S = Shape<D, K>;
  constexpr int NP = S::NP;
  constexpr bool MIX = sizeof(TS) != sizeof(T);
  typedef const int __attribute__((address_space(4)))* ciptr;
  const int lane = threadIdx.x & 63;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int tile = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
  if (stopped(A.stop)) return;  // uniform over the grid
  static_assert(SM == SM_ALL || staged_fits<D, K, T, SM>(), "staged tables exceed 64 KiB");
  constexpr int LO = SM == SM_ALL ? 0 : staged_lo<D, K, SM>();
  Tabs<SM, T, LO> tab;
  tab.c = (typename Tabs<SM, T, LO>::cptr)A.tab;
  if constexpr (SM != SM_ALL) {
    __shared__ T stab[staged_hi<D, K, SM>() - LO];
    stage_tables<D, K, SM>(stab, A.tab);
    __syncthreads();
    tab.l = stab;
  } else {
    tab.l = A.tab;
  }
  const int type = __builtin_amdgcn_readfirstlane(A.tile_type[tile]);
  if (type < 0) {  // empty tile padding a block
    if (A.mode == 2 && lane == 0) A.partial[tile] = 0.0;
    return;
  }
  const int e_raw = A.elem_list[tile * 64 + lane];
  const int e = e_raw >= 0 ? e_raw : A.elem_list[tile * 64];  // padded lanes redo lane 0
  const ciptr ttab = (ciptr)A.type_tab;

  T c[D][NP], uc[SELF ? 1 : D][SELF ? 1 : NP], Rv[D][NP], jic[D][D];
  TS ji[D][D];
  {
    const TS* __restrict__ p = A.x + (size_t)e * D * NP;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) c[i][m] = (T)p[i * NP + m];
    if constexpr (!SELF) {
      const TS* __restrict__ pu = A.u + (size_t)e * D * NP;
      TS uw[D][NP];
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 0; m < NP; ++m) uw[i][m] = pu[i * NP + m];
      if (A.u2) {
        const TS* __restrict__ pu2 = A.u2 + (size_t)e * D * NP;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int m = 0; m < NP; ++m) uw[i][m] = fma(A.uth, pu2[i * NP + m] - uw[i][m], uw[i][m]);
      }
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 0; m < NP; ++m) uc[i][m] = (T)uw[i][m];
    }
    const TS* __restrict__ pj = A.jinv + (size_t)e * D * D;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        ji[i][j] = pj[i * D + j];
        jic[i][j] = (T)ji[i][j];
      }
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int m = 0; m < NP; ++m) Rv[i][m] = T(0);

  // ---- volume term
#pragma unroll 1
  for (int q = 0; q < S::NQ; ++q) {
    const int bq = S::OFF_BV + q * NP;
    const int dq = S::OFF_DV + q * NP * D;
    T wq[D], uq[D], uh[D];
#pragma unroll
    for (int i = 0; i < D; ++i) wq[i] = T(0);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      const T bm = tab.template get<TB_BV>(bq + m);
#pragma unroll
      for (int i = 0; i < D; ++i) wq[i] = fma(bm, c[i][m], wq[i]);
    }
    if constexpr (SELF) {
#pragma unroll
      for (int i = 0; i < D; ++i) uq[i] = wq[i];
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) uq[i] = T(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const T bm = tab.template get<TB_BV>(bq + m);
#pragma unroll
        for (int i = 0; i < D; ++i) uq[i] = fma(bm, uc[i][m], uq[i]);
      }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T s = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) s = fma(jic[a][j], uq[j], s);
      uh[a] = s;
    }
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      T P = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) P = fma(uh[a], tab.template get<TB_DV>(dq + m * D + a), P);
#pragma unroll
      for (int i = 0; i < D; ++i) Rv[i][m] = fma(wq[i], P, Rv[i][m]);
    }
  }
  // the volume term enters the state-type accumulator once
  TS R[D][NP];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int m = 0; m < NP; ++m) R[i][m] = (TS)Rv[i][m];

  // ---- facet terms (pointwise upwind flux)
#pragma unroll
  for (int f = 0; f <= D; ++f) {
    int own, nbt;
    if constexpr (LANE) {
      const int tt = A.elem_tab[(size_t)e * (D + 1) + f];
      own = tt & 0xffff;
      nbt = tt >> 16;
    } else {
      const int tt = ttab[type * (D + 1) + f];
      own = __builtin_amdgcn_readfirstlane(tt & 0xffff);
      nbt = __builtin_amdgcn_readfirstlane(tt >> 16);
    }
    const int tro = S::OFF_TR + own * S::NFQ * NP;
    const int lfo = S::OFF_LF + own * S::NFQ * NP;
    const int ne_raw = A.nbr[(size_t)e * (D + 1) + f];
    // per-lane boundary facet (LANE): the own element and table stand in for the neighbour,
    // and the outer values replace the traces below
    const bool lbnd = LANE && BND && nbt == kBoundaryTable;
    const int ne = lbnd ? e : ne_raw;
    TS Nt[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      TS s = TS(0);
#pragma unroll
      for (int a = 0; a < D; ++a) s = fma(ji[a][j], nref<D, TS>(f, a), s);
      Nt[j] = s;
    }
    // upwind flux at facet point q from the inner and outer traces (state type), lifted into R
    auto flux_lift = [&](int q, const TS (&wm)[D], const TS (&wp)[D], const TS (&um)[D],
                         const TS (&up)[D]) {
      TS bb = TS(0);
#pragma unroll
      for (int j = 0; j < D; ++j) bb = fma(um[j] + up[j], Nt[j], bb);
      // b = bb / 2;  F = b (wm + wp) / 2 + |b| (wm - wp) / 2
      const TS hb = TS(0.25) * bb;
      const TS ha = TS(0.25) * fabs(bb);
      TS F[D];
#pragma unroll
      for (int i = 0; i < D; ++i) F[i] = hb * (wm[i] + wp[i]) + ha * (wm[i] - wp[i]);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const TS l = (TS)tab.template get<TB_LF>(lfo + q * NP + m);
#pragma unroll
        for (int i = 0; i < D; ++i) R[i][m] = fma(-l, F[i], R[i][m]);
      }
    };
    if (!LANE && BND && nbt == kBoundaryTable) {
      // boundary facet (the class fixes it for the whole tile; compiled only for meshes that
      // have boundary facets): the outer values are the given boundary data at the facet
      // points, [boundary facet][point][component]
      const size_t bf = (size_t)(-1 - ne_raw);
      const TS* __restrict__ pb = A.wb + bf * S::NFQ * D;
      const TS* __restrict__ pub = SELF ? pb : A.ub + bf * S::NFQ * D;
#pragma unroll 1
      for (int q = 0; q < S::NFQ; ++q) {
        T am[D], aum[D];
#pragma unroll
        for (int i = 0; i < D; ++i) { am[i] = T(0); aum[i] = T(0); }
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const T to = tab.template get<TB_TRO>(tro + q * NP + m);
#pragma unroll
          for (int i = 0; i < D; ++i) {
            am[i] = fma(to, c[i][m], am[i]);
            if constexpr (!SELF) aum[i] = fma(to, uc[i][m], aum[i]);
          }
        }
        TS wm[D], wp[D], um[D], up[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          wm[i] = (TS)am[i];
          um[i] = SELF ? wm[i] : (TS)aum[i];
          wp[i] = pb[q * D + i];
          up[i] = pub[q * D + i];
        }
        flux_lift(q, wm, wp, um, up);
      }
      continue;
    }
    const int trn = S::OFF_TR + (lbnd ? own : nbt) * S::NFQ * NP;
    const size_t lbf = lbnd ? (size_t)(-1 - ne_raw) : 0;
    T cn[D][NP], un[SELF ? 1 : D][SELF ? 1 : NP];
    {
      const TS* __restrict__ p = A.x + (size_t)ne * D * NP;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 0; m < NP; ++m) cn[i][m] = (T)p[i * NP + m];
      if constexpr (!SELF) {
        const TS* __restrict__ pu = A.u + (size_t)ne * D * NP;
        TS uw[D][NP];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int m = 0; m < NP; ++m) uw[i][m] = pu[i * NP + m];
        if (A.u2) {
          const TS* __restrict__ pu2 = A.u2 + (size_t)ne * D * NP;
#pragma unroll
          for (int i = 0; i < D; ++i)
#pragma unroll
            for (int m = 0; m < NP; ++m) uw[i][m] = fma(A.uth, pu2[i * NP + m] - uw[i][m], uw[i][m]);
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int m = 0; m < NP; ++m) un[i][m] = (T)uw[i][m];
      }
    }
#pragma unroll 1
    for (int q = 0; q < S::NFQ; ++q) {
      T am[D], ap[D];
#pragma unroll
      for (int i = 0; i < D; ++i) { am[i] = T(0); ap[i] = T(0); }
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const T to = tab.template get<TB_TRO>(tro + q * NP + m);
        const T tn = tab.template get<TB_TRN>(trn + q * NP + m);
#pragma unroll
        for (int i = 0; i < D; ++i) {
          am[i] = fma(to, c[i][m], am[i]);
          ap[i] = fma(tn, cn[i][m], ap[i]);
        }
      }
      TS wm[D], wp[D], um[D], up[D];
#pragma unroll
      for (int i = 0; i < D; ++i) { wm[i] = (TS)am[i]; wp[i] = (TS)ap[i]; }
      if constexpr (SELF) {
#pragma unroll
        for (int i = 0; i < D; ++i) { um[i] = wm[i]; up[i] = wp[i]; }
      } else {
        T aum[D], aup[D];
#pragma unroll
        for (int i = 0; i < D; ++i) { aum[i] = T(0); aup[i] = T(0); }
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const T to = tab.template get<TB_TRO>(tro + q * NP + m);
          const T tn = tab.template get<TB_TRN>(trn + q * NP + m);
#pragma unroll
          for (int i = 0; i < D; ++i) {
            aum[i] = fma(to, uc[i][m], aum[i]);
            aup[i] = fma(tn, un[i][m], aup[i]);
          }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) { um[i] = (TS)aum[i]; up[i] = (TS)aup[i]; }
      }
      if constexpr (LANE && BND) {
        if (lbnd) {
#pragma unroll
          for (int i = 0; i < D; ++i) {
            wp[i] = A.wb[(lbf * S::NFQ + q) * D + i];
            up[i] = SELF ? wp[i] : A.ub[(lbf * S::NFQ + q) * D + i];
          }
        }
      }
      flux_lift(q, wm, wp, um, up);
    }
  }

  // the state the update starts from, in the state type (the contraction copy is rounded when
  // the types differ, so the state is read again)
  TS xs[D][NP];
  if constexpr (MIX) {
    const TS* __restrict__ p = A.x + (size_t)e * D * NP;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) xs[i][m] = p[i * NP + m];
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) xs[i][m] = (TS)c[i][m];
  }
  TS* o = A.out + (size_t)e * D * NP;
  if (A.mode == 2) {
    // every lane takes part in the wave sum; padded lanes store nothing and add zero
    const TS* pg = A.w0 + (size_t)e * D * NP;
    TS gv[D][NP];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) gv[i][m] = pg[i * NP + m];
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const TS res = fma(A.tau, R[i][m], gv[i][m] - xs[i][m]);
        if (e_raw >= 0) o[i * NP + m] = fma(A.ds, res, xs[i][m]);
        acc = fma((double)res, (double)res, acc);
      }
    acc = wave_sum(e_raw >= 0 ? acc * A.absdet[e] : 0.0);
    if (lane == 0) A.partial[tile] = acc;
    return;
  }
  if (e_raw < 0) return;
  if (A.mode == 0) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) o[i * NP + m] = R[i][m];
  } else {
    const TS a = A.a, b = A.b, dt = A.dt;
    if (a != TS(0)) {
      // all loads of w0 before any store: out may be w0 itself (in-place last stage), and
      // back-to-back stores let whole cache lines complete in L2 before eviction
      const TS* pw = A.w0 + (size_t)e * D * NP;
      TS w0v[D][NP];
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 0; m < NP; ++m) w0v[i][m] = pw[i * NP + m];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 0; m < NP; ++m)
          o[i * NP + m] = fma(a, w0v[i][m], b * fma(dt, R[i][m], xs[i][m]));
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 0; m < NP; ++m) o[i * NP + m] = b * fma(dt, R[i][m], xs[i][m]);
    }
  }
}

// FP64 self-convection on a periodic mesh with tiles of one element class (the workloads'
// default path): the same arithmetic as conv_kernel<D, K, double, true, SM, false, false>, with
// the volume loop cut into D + 2 pieces and the facets between them.  The neighbour state of
// each facet is requested before the volume piece that precedes it, so its memory latency
// overlaps that piece (the registers of one neighbour state are free during the volume loop),
// and the volume and facet terms accumulate into one set of sums.  The Runge-Kutta base
// state takes the neighbour registers after the last facet, before the last volume piece.
template <int D, int K, int SM>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(min_waves<D, K, double>(), 8))) conv_self_kernel(ConvArgs<double> A) {
  using S = Shape<D, K>;
  using T = double;
  constexpr int NP = S::NP;
  typedef const int __attribute__((address_space(4)))* ciptr;
  const int lane = threadIdx.x & 63;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int tile = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
  if (stopped(A.stop)) return;  // uniform over the grid
  static_assert(SM == SM_ALL || staged_fits<D, K, T, SM>(), "staged tables exceed 64 KiB");
  constexpr int LO = SM == SM_ALL ? 0 : staged_lo<D, K, SM>();
  Tabs<SM, T, LO> tab;
  tab.c = (typename Tabs<SM, T, LO>::cptr)A.tab;
  if constexpr (SM != SM_ALL) {
    __shared__ T stab[staged_hi<D, K, SM>() - LO];
    stage_tables<D, K, SM>(stab, A.tab);
    __syncthreads();
    tab.l = stab;
  } else {
    tab.l = A.tab;
  }
  const int type = __builtin_amdgcn_readfirstlane(A.tile_type[tile]);
  if (type < 0) {  // empty tile padding a block
    if (A.mode == 2 && lane == 0) A.partial[tile] = 0.0;
    return;
  }
  const int e_raw = A.elem_list[tile * 64 + lane];
  const int e = e_raw >= 0 ? e_raw : A.elem_list[tile * 64];  // padded lanes redo lane 0
  const ciptr ttab = (ciptr)A.type_tab;

  T c[D][NP], ji[D][D], R[D][NP];
  int nbv[D + 1];
  {
    const T* __restrict__ p = A.x + (size_t)e * D * NP;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) c[i][m] = p[i * NP + m];
    const T* __restrict__ pj = A.jinv + (size_t)e * D * D;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) ji[i][j] = pj[i * D + j];
#pragma unroll
    for (int f = 0; f <= D; ++f) nbv[f] = A.nbr[(size_t)e * (D + 1) + f];
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int m = 0; m < NP; ++m) R[i][m] = T(0);

  // neighbour state of the facet about to come
  T cn[D][NP];
  auto load_nbr_state_from = [&](const T* __restrict__ src, int ne) {
    const T* __restrict__ p = src + (size_t)ne * D * NP;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) cn[i][m] = p[i * NP + m];
  };
  auto load_nbr_state = [&](int ne) { load_nbr_state_from(A.x, ne); };

  // volume term over the points [q0, q1): R[i][m] += w_i(x_q) (J^-1 w(x_q)) . w_q grad^ phi_m
  auto volume = [&](int q0, int q1) {
#pragma unroll 1
    for (int q = q0; q < q1; ++q) {
      const int bq = S::OFF_BV + q * NP;
      const int dq = S::OFF_DV + q * NP * D;
      T wq[D], uh[D];
#pragma unroll
      for (int i = 0; i < D; ++i) wq[i] = T(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const T bm = tab.template get<TB_BV>(bq + m);
#pragma unroll
        for (int i = 0; i < D; ++i) wq[i] = fma(bm, c[i][m], wq[i]);
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < D; ++j) s = fma(ji[a][j], wq[j], s);
        uh[a] = s;
      }
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        T P = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) P = fma(uh[a], tab.template get<TB_DV>(dq + m * D + a), P);
#pragma unroll
        for (int i = 0; i < D; ++i) R[i][m] = fma(wq[i], P, R[i][m]);
      }
    }
  };

  // facet term of local facet f with the neighbour state in cn (pointwise upwind flux)
  auto facet = [&](int f) {
    const int tt = ttab[type * (D + 1) + f];
    const int own = __builtin_amdgcn_readfirstlane(tt & 0xffff);
    const int nbt = __builtin_amdgcn_readfirstlane(tt >> 16);
    const int tro = S::OFF_TR + own * S::NFQ * NP;
    const int trn = S::OFF_TR + nbt * S::NFQ * NP;
    const int lfo = S::OFF_LF + own * S::NFQ * NP;
    T Nt[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T s = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) s = fma(ji[a][j], nref<D, T>(f, a), s);
      Nt[j] = s;
    }
#pragma unroll 1
    for (int q = 0; q < S::NFQ; ++q) {
      T wm[D], wp[D];
#pragma unroll
      for (int i = 0; i < D; ++i) { wm[i] = T(0); wp[i] = T(0); }
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const T to = tab.template get<TB_TRO>(tro + q * NP + m);
        const T tn = tab.template get<TB_TRN>(trn + q * NP + m);
#pragma unroll
        for (int i = 0; i < D; ++i) {
          wm[i] = fma(to, c[i][m], wm[i]);
          wp[i] = fma(tn, cn[i][m], wp[i]);
        }
      }
      // b = bb / 2;  F = b (wm + wp) / 2 + |b| (wm - wp) / 2
      T bb = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) bb = fma(wm[j] + wp[j], Nt[j], bb);
      const T hb = T(0.25) * bb;
      const T ha = T(0.25) * fabs(bb);
      T F[D];
#pragma unroll
      for (int i = 0; i < D; ++i) F[i] = hb * (wm[i] + wp[i]) + ha * (wm[i] - wp[i]);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const T l = tab.template get<TB_LF>(lfo + q * NP + m);
#pragma unroll
        for (int i = 0; i < D; ++i) R[i][m] = fma(-l, F[i], R[i][m]);
      }
    }
  };

  // D + 3 shares of the volume points: one before each facet, two after the last facet, where
  // the base state's latency must be covered as well
  constexpr int NCH = D + 3;
  load_nbr_state(nbv[0]);
#pragma unroll
  for (int f = 0; f <= D; ++f) {
    volume(f * S::NQ / NCH, (f + 1) * S::NQ / NCH);
    facet(f);
    if (f < D) load_nbr_state(nbv[f + 1]);
  }
  // the base state w0 of the stage goes into the registers of the last neighbour state,
  // requested before the last volume piece so that its latency overlaps that piece
  const bool base = A.mode == 2 || (A.mode == 1 && A.a != T(0));
  if (base) load_nbr_state_from(A.w0, e);
  volume((D + 1) * S::NQ / NCH, S::NQ);

  T* o = A.out + (size_t)e * D * NP;
  if (A.mode == 2) {
    // every lane takes part in the wave sum; padded lanes store nothing and add zero
    const T(&gv)[D][NP] = cn;  // w0
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const T res = fma(A.tau, R[i][m], gv[i][m] - c[i][m]);
        if (e_raw >= 0) o[i * NP + m] = fma(A.ds, res, c[i][m]);
        acc = fma(res, res, acc);
      }
    // the element index is read again here (volatile; e_raw once more), so that no 64-bit
    // offset stays live in registers through the loops for this one use
    const int e_sum = *(volatile const int*)(A.elem_list + tile * 64 + lane);
    acc = wave_sum(e_sum >= 0 ? acc * A.absdet[e_sum >= 0 ? e_sum : 0] : 0.0);
    if (lane == 0) A.partial[tile] = acc;
    return;
  }
  if (e_raw < 0) return;
  if (A.mode == 0) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < NP; ++m) o[i * NP + m] = R[i][m];
  } else {
    const T a = A.a, b = A.b, dt = A.dt;
    if (a != T(0)) {
      // w0 (in cn) was loaded before the last volume piece, so before any store: out may be
      // w0 itself (in-place last stage), and back-to-back stores let whole cache lines
      // complete in L2 before eviction
      const T(&w0v)[D][NP] = cn;
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 0; m < NP; ++m)
          o[i * NP + m] = fma(a, w0v[i][m], b * fma(dt, R[i][m], c[i][m]));
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int m = 0; m < NP; ++m) o[i * NP + m] = b * fma(dt, R[i][m], c[i][m]);
    }
  }
}

// The partner lane's value within a lane pair (2j, 2j + 1): DPP quad permutation [1, 0, 3, 2],
// two 32-bit moves for a double.
__device__ __forceinline__ double pair_swap(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(v & 0xffffffffll), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), 0xB1, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// 2D FP64 self-convection on a periodic mesh with tiles of one element class, two lanes per
// element: lane pair (2j, 2j + 1) of a wave holds element j of one half (32 elements) of a
// 64-element tile, lane 2j + h its velocity component h (coefficients, the sums R, the neighbour
// coefficients), so a tile takes two waves and a workgroup of four waves two tiles.  At a point,
// each lane interpolates its component, takes the partner's by a DPP exchange, and contracts
// the flux row w_h (J^-1 w) with the test gradients into its own sums; on a facet each lane
// forms the traces of its component, exchanges them, and both lanes form the normal speed
// as the sum of the two component products (a + b, rounded alike in both lanes).  Twice the
// waves of conv_self_kernel at 30 coefficients of state per lane instead of 60.  Modes 0 and 1.
template <int K, int SM>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(4, 8))) conv_pair_kernel(ConvArgs<double> A) {
  constexpr int D = 2;
  using S = Shape<D, K>;
  using T = double;
  constexpr int NP = S::NP;
  typedef const int __attribute__((address_space(4)))* ciptr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane & 1;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int tile = __builtin_amdgcn_readfirstlane(blk * 2 + (wv >> 1));
  static_assert(SM == SM_ALL || staged_fits<D, K, T, SM>(), "staged tables exceed 64 KiB");
  constexpr int LO = SM == SM_ALL ? 0 : staged_lo<D, K, SM>();
  Tabs<SM, T, LO> tab;
  tab.c = (typename Tabs<SM, T, LO>::cptr)A.tab;
  if constexpr (SM != SM_ALL) {
    __shared__ T stab[staged_hi<D, K, SM>() - LO];
    stage_tables<D, K, SM>(stab, A.tab);
    __syncthreads();
    tab.l = stab;
  } else {
    tab.l = A.tab;
  }
  if (tile >= A.ntiles) return;
  const int type = __builtin_amdgcn_readfirstlane(A.tile_type[tile]);
  if (type < 0) return;  // empty tile padding a block
  const int slot = tile * 64 + (wv & 1) * 32 + (lane >> 1);
  const int e_raw = A.elem_list[slot];
  const int e = e_raw >= 0 ? e_raw : A.elem_list[tile * 64];  // padded pairs redo element 0
  const ciptr ttab = (ciptr)A.type_tab;

  T c[NP], R[NP], jo[D], jt[D];  // own component; J^-1 columns h and 1 - h
  int nbv[D + 1];
  {
    const T* __restrict__ p = A.x + (size_t)e * D * NP + h * NP;
#pragma unroll
    for (int m = 0; m < NP; ++m) c[m] = p[m];
    const T* __restrict__ pj = A.jinv + (size_t)e * D * D;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const T j0 = pj[a * D], j1 = pj[a * D + 1];
      jo[a] = h ? j1 : j0;
      jt[a] = h ? j0 : j1;
    }
#pragma unroll
    for (int f = 0; f <= D; ++f) nbv[f] = A.nbr[(size_t)e * (D + 1) + f];
  }
#pragma unroll
  for (int m = 0; m < NP; ++m) R[m] = T(0);

  // volume term: R_hm += w_h(x_q) (J^-1 w(x_q)) . w_q grad^ phi_m
#pragma unroll 1
  for (int q = 0; q < S::NQ; ++q) {
    const int bq = S::OFF_BV + q * NP;
    const int dq = S::OFF_DV + q * NP * D;
    T wh = T(0);
#pragma unroll
    for (int m = 0; m < NP; ++m) wh = fma(tab.template get<TB_BV>(bq + m), c[m], wh);
    const T wo = pair_swap(wh);
    const T g0 = wh * fma(jo[0], wh, jt[0] * wo);
    const T g1 = wh * fma(jo[1], wh, jt[1] * wo);
#pragma unroll
    for (int m = 0; m < NP; ++m)
      R[m] = fma(g0, tab.template get<TB_DV>(dq + m * D), fma(g1, tab.template get<TB_DV>(dq + m * D + 1), R[m]));
  }

  // facets: pointwise upwind flux with the neighbour across local facet f
#pragma unroll
  for (int f = 0; f <= D; ++f) {
    T cn[NP];
    {
      const T* __restrict__ p = A.x + (size_t)nbv[f] * D * NP + h * NP;
#pragma unroll
      for (int m = 0; m < NP; ++m) cn[m] = p[m];
    }
    const int tt = ttab[type * (D + 1) + f];
    const int own = __builtin_amdgcn_readfirstlane(tt & 0xffff);
    const int nbt = __builtin_amdgcn_readfirstlane(tt >> 16);
    const int tro = S::OFF_TR + own * S::NFQ * NP;
    const int trn = S::OFF_TR + nbt * S::NFQ * NP;
    const int lfo = S::OFF_LF + own * S::NFQ * NP;
    T Nh = T(0);  // component h of the scaled normal J^-T n^
#pragma unroll
    for (int a = 0; a < D; ++a) Nh = fma(jo[a], nref<D, T>(f, a), Nh);
#pragma unroll 1
    for (int q = 0; q < S::NFQ; ++q) {
      T wm = T(0), wp = T(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        wm = fma(tab.template get<TB_TRO>(tro + q * NP + m), c[m], wm);
        wp = fma(tab.template get<TB_TRN>(trn + q * NP + m), cn[m], wp);
      }
      // b = bb / 2 with bb = sum_j (wm_j + wp_j) Nt_j;  F = b (wm + wp) / 2 + |b| (wm - wp) / 2
      const T th = (wm + wp) * Nh;
      const T bb = th + pair_swap(th);
      const T hb = T(0.25) * bb;
      const T ha = T(0.25) * fabs(bb);
      const T F = hb * (wm + wp) + ha * (wm - wp);
#pragma unroll
      for (int m = 0; m < NP; ++m) R[m] = fma(-tab.template get<TB_LF>(lfo + q * NP + m), F, R[m]);
    }
  }

  if (e_raw < 0) return;
  T* o = A.out + (size_t)e * D * NP + h * NP;
  if (A.mode == 0) {
#pragma unroll
    for (int m = 0; m < NP; ++m) o[m] = R[m];
  } else {
    const T a = A.a, b = A.b, dt = A.dt;
    if (a != T(0)) {
      // all loads of w0 before any store: out may be w0 itself (in-place last stage)
      const T* pw = A.w0 + (size_t)e * D * NP + h * NP;
      T w0v[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) w0v[m] = pw[m];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) o[m] = fma(a, w0v[m], b * fma(dt, R[m], c[m]));
    } else {
#pragma unroll
      for (int m = 0; m < NP; ++m) o[m] = b * fma(dt, R[m], c[m]);
    }
  }
}

}  // namespace dgk
