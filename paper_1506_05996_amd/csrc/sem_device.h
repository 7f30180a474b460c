// Device-side state of a sem_mesh handle and the internal operations shared by
// the single-mesh entry points (sem_device.hip) and the batched solver
// (sem_batch.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>

#include <functional>
#include <string>

#include "sem_internal.h"

namespace sem {

#define SEM_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t err_ = (call);                                                             \
    if (err_ != hipSuccess)                                                               \
      throw ::sem::Error{SEM_EHIP, std::string(#call) + ": " + hipGetErrorString(err_)}; \
  } while (0)

// device buffer owned by a handle
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    hipError_t err = hipMalloc((void**)&p, count * sizeof(T));
    if (err != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error{SEM_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    n = count;
  }
  void upload(const T* h, size_t count) {
    alloc(count);
    if (count) SEM_HIP(hipMemcpy(p, h, count * sizeof(T), hipMemcpyHostToDevice));
  }
  // same contents as upload, in place when the size is unchanged (the device
  // address stays valid for launches recorded earlier)
  void copy_in(const T* h, size_t count) {
    if (p == nullptr || count != n) return upload(h, count);
    if (count) SEM_HIP(hipMemcpy(p, h, count * sizeof(T), hipMemcpyHostToDevice));
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DBuf() { release(); }
};

template <typename TD, typename TS>
static std::vector<TD> convert(const std::vector<TS>& v) {
  return std::vector<TD>(v.begin(), v.end());
}

}  // namespace sem

using namespace sem;

struct sem_mesh_s {
  HostTables T;
  bool host_only = false;
  bool fp32 = true;
  int device = 0;
  // numbering / gather
  DBuf<int32_t> rec, vinc_off, vinc_ec, einc_off, cidx, order;
  DBuf<uint8_t> dir, fcount;
  // operator
  DBuf<double> G64, D64, w64, X864, tq64;  // X8: vertex coordinates, tq: GLL points and weights
  DBuf<float> G32, D32, w32, X832, tq32;
  // fine preconditioner
  // patch corrections: zo = [zc: E x (N+1)^3 own nodes | zx: E x nx consumer layout]
  DBuf<int32_t> ip, xdest;
  DBuf<double> S64, lam64, h64, zo64;
  DBuf<float> S32, lam32, h32, zo32;
  // coarse: vectors in coarse order (R, y, Z, X), vertex-order solution Zv,
  // the nested-dissection fronts and their work lists
  DBuf<double> phi, Re, Rlev, Ylev, Wlev, Xlev, Zv;
  DBuf<double> fwd_pool, bwd_pool, cvec;
  DBuf<FrontNode> fnodes;
  DBuf<int32_t> fb_idx, ct_off, ct_pos, fy_items;
  DBuf<RowItem> fr_items, br_items, fs_items;
  hipGraphExec_t coarse_graph = nullptr;  // the solve sweeps, captured once per factorisation
  bool direct_coarse = false;             // launch the sweeps directly (inside an enclosing capture)
  int epb[2] = {0, 0};                    // operator tile (elements per workgroup) for FP64, FP32
  hipStream_t side_stream = nullptr;      // coarse chain of the preconditioner, beside the patch solves
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // PCG's convergence check read back without draining the stream: r . r and
  // the breakdown flag land in pinned host memory, signalled by ev_check
  double* check_host = nullptr;
  hipEvent_t ev_check = nullptr;
  hipStream_t capture_stream = nullptr;
  // lumped mass m_N for the mass term of the operator (uploaded when c != 0),
  // and the right-hand side of a heat-equation step
  DBuf<double> mN64, hb;
  DBuf<float> mN32;
  // per-element coefficients kappa_e, c_e [E] and the local mass [E][(N+1)^3]
  bool per_elem = false, any_ce = false;
  DBuf<double> ke64, ce64, mL64;
  DBuf<float> ke32, ce32, mL32;
  // per-node coefficients: kappa_{ijk;e} is folded into the device factors G
  // (the host keeps the plain G) and kept per local node (kn) for the kernel
  // that rebuilds G; the element kernels take kappa_e = 1 (nk), c_e = 1 where
  // the element has some c != 0 (nc) and c_{ijk;e} m_{ijk;e} in place of the
  // local mass (nm); ke/ce then hold the element means that the patch solves
  // and the coarse matrix use (per_elem is set too)
  bool per_node = false;
  DBuf<double> nk64, nc64, nm64, kn64;
  DBuf<float> nk32, nc32, nm32, kn32;
  // coarse solver: 0 exact (nested dissection), 1 aggregation AMG with a K-cycle
  int coarse_solver = 0;
  struct AmgDev {
    int64_t n = 0;
    DBuf<int32_t> off, col, agg, moff, mem;
    DBuf<double> val, wd;
    DBuf<double> B, X, R, T, V, W, B2, V2, W2;  // cycle input/output/temporaries, flexible-CG vectors
  };
  std::vector<std::unique_ptr<AmgDev>> amg;
  DBuf<double> amg_inv, amg_sc;
  DBuf<int32_t> amg_nd, amg_pos;
  hipGraphExec_t amg_graph = nullptr;
  // PCG work: the handle's own buffers (allocated by the first solve that
  // needs them) ...
  DBuf<double> v64[5];
  DBuf<float> v32[5];
  DBuf<double> part, sc, dpart;
  // ... and the pointers one solve works in: the buffers above, or views into
  // the library's static scratch array (sem_pcg_solve_noalloc)
  struct SolveWork {
    double* v64[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float* v32[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double* part = nullptr;   // kRedBlocks partial sums
    double* sc = nullptr;     // 16 device scalars of Algorithm 1
    double* dpart = nullptr;  // per-workgroup partial dot products of the operator and preconditioner
  } wk;
  bool no_alloc = false;      // inside sem_pcg_solve_noalloc: no lazy set-up may run
};

namespace sem {

constexpr int kThreads = 256;
inline int64_t blocks_of(int64_t n, int t = kThreads) { return n < 1 ? 1 : (n + t - 1) / t; }

// internal operations on a handle (all stream-ordered, no synchronisation)
template <typename T>
void apply_A(sem_mesh m, const T* u, T* y, hipStream_t s);
template <typename T>
void precond(sem_mesh m, const T* r, T* z, int pc, hipStream_t s);
sem_mesh_s* create_mesh(const double* vtx, int64_t n_vtx, const int64_t* hex, int64_t n_hex, int order,
                        const sem_setup_opts* opts);
int guarded_call(const std::function<int()>& f);

}  // namespace sem
