// Internal declarations shared by the translation units of libdgconv.so (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/dgconv.h"
#include "hdiv.hpp"
#include "mesh.hpp"

namespace dgi {

// record an error message for dg_last_error() and return the status
dg_status fail(dg_status s, const std::string& msg);

}  // namespace dgi

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return dgi::fail(e_ == hipErrorOutOfMemory ? DG_ENOMEM : DG_EDEVICE,              \
                       std::string(#expr ": ") + hipGetErrorString(e_));                \
  } while (0)

struct dg_mesh {
  dgmesh::Host h;
  dgmesh::Tables t;
  int device = 0;
  double* d_tab = nullptr;
  double* d_spd = nullptr;   // basis values at the speed-reduction points
  float* d_tab_f = nullptr;
  double* d_jinv = nullptr;
  float* d_jinv_f = nullptr;
  double* d_absdet = nullptr;
  int* d_nbr = nullptr;
  int* d_elem_list = nullptr;
  int* d_tile_type = nullptr;
  int* d_type_tab = nullptr;
  int* d_elem_tab = nullptr;  // per-element facet tables (per-lane table mode)
  mutable void* d_work = nullptr;
  mutable size_t work_bytes = 0;
  double* d_partial = nullptr;  // reduction partials
  double* d_rich_partial = nullptr;  // pseudo-time iteration: per-tile residual sums
  void* d_rich_state = nullptr;      // pseudo-time iteration: device-side control block
  int n_partial = 0;
  bool on_device = false;
  int tab_src = -1;  // VALU kernel table sources (bit t: table t via scalar loads); -1: default
  bool fp64_mfma = false;   // FP64 self-convection on the matrix cores instead of the VALU kernel
  bool fp64_mfma_frozen = false;  // the same for a given (frozen or extrapolated) velocity
  bool self_pipe = true;
  bool pair = false;          // 2D FP64 self-convection with two lanes per element  // FP64 self-convection on the VALU: the pipelined kernel (conv_self_kernel)
  // matrix-core path: 16-wide tiles and fragment tables per contraction engine
  int* d_elem_list16 = nullptr;
  int* d_tile_type16 = nullptr;
  void* d_frag[3] = {nullptr, nullptr, nullptr};  // 0: f64, 1: fp16 x2, 2: bf16 x3
  // H(div) transfer (2D): numbering and tables built on first use
  bool hd_ready = false;
  dghdiv::Host hd;
  int* d_hfacet = nullptr;          // [E][3] facet id and signs
  int64_t* d_hfelem = nullptr;      // [nfacet][2] sides of each facet
  double* d_htab = nullptr;         // [ndof][2][np] reference dual basis
  double* d_hlocal = nullptr;       // [E][ndof] element contributions of the transpose
  std::mutex mu;
};

namespace dgi {
// upload the mesh's device tables on first use (synchronous)
dg_status ensure_device(const dg_mesh* m);
}  // namespace dgi
