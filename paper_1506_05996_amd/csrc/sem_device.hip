// Device state, kernel launches and the C ABI of the spectral-element solver.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <mutex>
#include <vector>

#include "sem_device.h"
#include "sem_internal.h"
#include "sem_kernels.h"

namespace sem {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace sem

using namespace sem;

namespace sem {

constexpr int kGS = 256;

inline int64_t blocks_for(int64_t n, int t = kGS) { return std::max<int64_t>(1, (n + t - 1) / t); }
// grid of the grid-stride streaming kernels: up to 65,536 workgroups (more
// loads in flight than the 8,192 a stream of n_global doubles would need to
// cover the chip once: the p/x update streams at 5.2 TB/s instead of 4.5)
inline int grid_stride_blocks(int64_t n) { return (int)std::min<int64_t>(blocks_for(n), 65536); }

// every pointer 16-byte aligned (the streaming kernels then move two entries per access)
template <typename... P>
bool aligned16(const P*... ptrs) {
  return ((reinterpret_cast<uintptr_t>(ptrs) % 16 == 0) && ...);
}

template <typename T>
const T* Gp(sem_mesh m);
template <>
const double* Gp<double>(sem_mesh m) { return m->G64.p; }
template <>
const float* Gp<float>(sem_mesh m) { return m->G32.p; }
template <typename T>
const T* Dp(sem_mesh m);
template <>
const double* Dp<double>(sem_mesh m) { return m->D64.p; }
template <typename T>
const T* X8p(sem_mesh m);
template <>
const double* X8p<double>(sem_mesh m) { return m->X864.p; }
template <>
const float* X8p<float>(sem_mesh m) { return m->X832.p; }
template <typename T>
const T* TQp(sem_mesh m);
template <>
const double* TQp<double>(sem_mesh m) { return m->tq64.p; }
template <>
const float* TQp<float>(sem_mesh m) { return m->tq32.p; }
template <>
const float* Dp<float>(sem_mesh m) { return m->D32.p; }
template <typename T>
T* Wp(sem_mesh m);
template <>
double* Wp<double>(sem_mesh m) { return m->w64.p; }
template <>
float* Wp<float>(sem_mesh m) { return m->w32.p; }
template <typename T>
T* ZOp(sem_mesh m);
template <>
double* ZOp<double>(sem_mesh m) { return m->zo64.p; }
template <>
float* ZOp<float>(sem_mesh m) { return m->zo32.p; }
template <typename T>
const T* Sp(sem_mesh m);
template <>
const double* Sp<double>(sem_mesh m) { return m->S64.p; }
template <>
const float* Sp<float>(sem_mesh m) { return m->S32.p; }
template <typename T>
const T* Lp(sem_mesh m);
template <>
const double* Lp<double>(sem_mesh m) { return m->lam64.p; }
template <>
const float* Lp<float>(sem_mesh m) { return m->lam32.p; }
template <typename T>
const T* Hp(sem_mesh m);
template <>
const double* Hp<double>(sem_mesh m) { return m->h64.p; }
template <>
const float* Hp<float>(sem_mesh m) { return m->h32.p; }
template <typename T>
const T* KEp(sem_mesh m);
template <>
const double* KEp<double>(sem_mesh m) { return m->ke64.p; }
template <>
const float* KEp<float>(sem_mesh m) { return m->ke32.p; }
template <typename T>
const T* CEp(sem_mesh m);
template <>
const double* CEp<double>(sem_mesh m) { return m->ce64.p; }
template <>
const float* CEp<float>(sem_mesh m) { return m->ce32.p; }

// --- operator ---------------------------------------------------------------
// tile candidates: elements per workgroup, workgroups of at most 1024 lanes;
// kTileMfma selects the matrix-core kernel (N = 15), kTileGeo the kernel
// that rebuilds the geometric factors from the vertices
constexpr int kTileCandidates[4] = {1, 2, 4, 8};
constexpr int kTileMfma = 16;
constexpr int kTileGeo = 32;  // factors rebuilt from the vertices, default elements per workgroup
// the line-phase kernel: factors rebuilt from the vertices, or stored
constexpr int kTileLineGeo = 64;
constexpr int kTileLineStored = 48;

bool tile_code_ok(int epb, int N) {
  if (epb == 1 || epb == 2 || epb == 4 || epb == 8) return epb * (N + 1) * (N + 1) <= 1024;
  return epb == kTileGeo || epb == kTileLineGeo || epb == kTileLineStored || (epb == kTileMfma && N == 15);
}

template <int N>
constexpr bool tile_ok(int epb) {
  return epb * (N + 1) * (N + 1) <= 1024;
}

// coefficients of the operator for dtype T (kappa = 1, c = 0 unless set)
template <typename T>
OpCoef<T> op_coef(sem_mesh m) {
  OpCoef<T> oc{T(1), T(0), nullptr, 0, nullptr, nullptr, nullptr, nullptr};
  if (m->per_node) {  // kappa per node is inside the stored G (kn: for the rebuilt G); c m per local node
    if constexpr (std::is_same<T, double>::value) {
      oc.ke = m->nk64.p;
      oc.ce = m->nc64.p;
      oc.mL = m->nm64.p;
      oc.kn = m->kn64.p;
    } else {
      oc.ke = m->nk32.p;
      oc.ce = m->nc32.p;
      oc.mL = m->nm32.p;
      oc.kn = m->kn32.p;
    }
    if (oc.ke == nullptr || oc.ce == nullptr || oc.kn == nullptr || (m->any_ce && oc.mL == nullptr))
      throw Error{SEM_EINVAL, "per-node coefficients not on the device"};
    return oc;
  }
  if (m->per_elem) {  // per-element coefficients: applied by the element kernels
    if constexpr (std::is_same<T, double>::value) {
      oc.ke = m->ke64.p;
      oc.ce = m->ce64.p;
      oc.mL = m->mL64.p;
    } else {
      oc.ke = m->ke32.p;
      oc.ce = m->ce32.p;
      oc.mL = m->mL32.p;
    }
    if (oc.ke == nullptr || oc.ce == nullptr || (m->any_ce && oc.mL == nullptr))
      throw Error{SEM_EINVAL, "per-element coefficients not on the device"};
    return oc;
  }
  oc.kap = (T)m->T.kappa;
  oc.cm = (T)m->T.cmass;
  oc.scaled = (m->T.kappa != 1.0 || m->T.cmass != 0.0) ? 1 : 0;
  if constexpr (std::is_same<T, double>::value)
    oc.mN = m->mN64.p;
  else
    oc.mN = m->mN32.p;
  if (m->T.cmass != 0.0 && oc.mN == nullptr) throw Error{SEM_EINVAL, "lumped mass not on the device"};
  return oc;
}

// element kernel launches; with dpart, each workgroup also leaves its share
// of u . y over the element interiors in dpart[block] (the grid size is
// returned so the caller knows how many)
template <int N, typename T, int EPB, bool GEO = false, bool KN = false>
int64_t launch_ax_tile(sem_mesh m, const T* u, T* y, double* dpart, hipStream_t s) {
  if constexpr (tile_ok<N>(EPB)) {
    const HostTables& T_ = m->T;
    const int64_t grid = xcd_grid((T_.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((ax_kernel<N, T, EPB, GEO, KN>), dim3((unsigned)grid), dim3(EPB * (N + 1) * (N + 1)), 0, s, u,
                       y, Wp<T>(m), GEO ? X8p<T>(m) : Gp<T>(m), m->rec.p, Dp<T>(m), m->dir.p, m->order.p, T_.E, dpart,
                       TQp<T>(m), op_coef<T>(m));
    SEM_HIP(hipGetLastError());
    return grid;
  } else {
    throw Error{SEM_EINVAL, "operator tile too large for the order"};
  }
}

template <int N, typename T, bool GEO, bool KN = false>
int64_t launch_ax_line(sem_mesh m, const T* u, T* y, double* dpart, hipStream_t s) {
  constexpr int EPB = ax_epb<N>();
  const HostTables& T_ = m->T;
  const int64_t grid = xcd_grid((T_.E + EPB - 1) / EPB);
  hipLaunchKernelGGL((ax_line_kernel<N, T, EPB, GEO, KN>), dim3((unsigned)grid), dim3(EPB * (N + 1) * (N + 1)), 0, s,
                     u, y, Wp<T>(m), GEO ? X8p<T>(m) : Gp<T>(m), m->rec.p, Dp<T>(m), m->dir.p, m->order.p, T_.E, dpart,
                     TQp<T>(m), op_coef<T>(m));
  SEM_HIP(hipGetLastError());
  return grid;
}

template <int N, typename T>
int64_t launch_ax(sem_mesh m, const T* u, T* y, double* dpart, hipStream_t s) {
  const int epb = m->epb[std::is_same<T, double>::value ? 0 : 1];
  if (epb == kTileMfma) {
    if constexpr (N == 15) {
      const HostTables& T_ = m->T;
      const int64_t grid = xcd_grid(T_.E);
      hipLaunchKernelGGL((ax_mfma15_kernel<T>), dim3((unsigned)grid), dim3(256), 0, s, u, y, Wp<T>(m), Gp<T>(m),
                         m->rec.p, Dp<T>(m), m->dir.p, m->order.p, T_.E, dpart, op_coef<T>(m));
      SEM_HIP(hipGetLastError());
      return grid;
    } else {
      throw Error{SEM_EINVAL, "the matrix-core operator exists at N = 15"};
    }
  }
  if (epb == kTileGeo) {
    // per-node kappa: read per node by its own instance of the kernel
    if (m->per_node) return launch_ax_tile<N, T, ax_epb<N>(), true, true>(m, u, y, dpart, s);
    return launch_ax_tile<N, T, ax_epb<N>(), true>(m, u, y, dpart, s);
  }
  if (epb == kTileLineGeo) {
    if (m->per_node) return launch_ax_line<N, T, true, true>(m, u, y, dpart, s);
    return launch_ax_line<N, T, true>(m, u, y, dpart, s);
  }
  if (epb == kTileLineStored) return launch_ax_line<N, T, false>(m, u, y, dpart, s);
  switch (epb > 0 ? epb : ax_epb<N>()) {
    case 1: return launch_ax_tile<N, T, 1>(m, u, y, dpart, s);
    case 2: return launch_ax_tile<N, T, 2>(m, u, y, dpart, s);
    case 4: return launch_ax_tile<N, T, 4>(m, u, y, dpart, s);
    case 8: return launch_ax_tile<N, T, 8>(m, u, y, dpart, s);
    default: throw Error{SEM_EINVAL, "operator tile"};
  }
}

int default_tile(int N) {
  switch (N) {
#define CASE(NN) \
  case NN:       \
    return ax_epb<NN>();
    CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14)
    CASE(15)
#undef CASE
  }
  return 1;
}

// the shared-node gather; as the operator's last step (u_op = the operator's
// input) it also applies the coefficients, as the preconditioner's it only sums
template <typename T>
int64_t launch_gs(sem_mesh m, T* y, hipStream_t s, const T* pd = nullptr, double* dpart = nullptr,
                  const T* u_op = nullptr) {
  const HostTables& T_ = m->T;
  const int64_t grid = blocks_for(T_.base_i);
  OpCoef<T> oc{T(1), T(0), nullptr, 0, nullptr, nullptr, nullptr, nullptr};
  if (u_op != nullptr && !m->per_elem) oc = op_coef<T>(m);
  hipLaunchKernelGGL((gs_kernel<T>), dim3((unsigned)grid), dim3(kGS), 0, s, y, Wp<T>(m), m->vinc_off.p,
                     m->einc_off.p, m->fcount.p, m->dir.p, T_.V, T_.base_f, T_.base_i, T_.N - 1, T_.wedge_off,
                     T_.wvert_off, pd, dpart, oc, u_op);
  SEM_HIP(hipGetLastError());
  return grid;
}

// element kernel only (the gather follows separately); returns the grid size
template <typename T>
int64_t apply_A_elements(sem_mesh m, const T* u, T* y, hipStream_t s, double* dpart = nullptr) {
  switch (m->T.N) {
#define CASE(NN) \
  case NN:       \
    return launch_ax<NN, T>(m, u, y, dpart, s);
    CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14)
    CASE(15)
#undef CASE
    default:
      throw Error{SEM_EUNSUPPORTED, "order not compiled"};
  }
}

template <typename T>
void apply_A(sem_mesh m, const T* u, T* y, hipStream_t s) {
  apply_A_elements<T>(m, u, y, s);
  launch_gs<T>(m, y, s, nullptr, nullptr, u);
}

// the n partial sums in the work's dpart into scalar slot dst (dot_final mode
// `mode`): through kRedBlocks chunk sums when there are many; a single launch
// when there are at most kRedBlocks (the chunk sums would then copy them one
// by one, so the result is the same bit for bit)
void reduce_partials(sem_mesh m, int64_t n, int dst, int mode, hipStream_t s) {
  if (n <= kRedBlocks) {
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kRedThreads), 0, s, (const double*)m->wk.dpart, m->wk.sc, (int)n,
                       dst, mode);
  } else {
    const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    const int nb = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(nb), dim3(kRedThreads), 0, s, (const double*)m->wk.dpart, m->wk.part,
                       n, chunk);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kRedThreads), 0, s, m->wk.part, m->wk.sc, nb, dst, mode);
  }
  SEM_HIP(hipGetLastError());
}

// y = A u and u . y into the scalar slot dst (dot_final mode `mode`), the dot
// product taken from the operator's own kernels (no extra pass over u and y)
template <typename T>
void apply_A_dot(sem_mesh m, const T* u, T* y, int dst, int mode, hipStream_t s) {
  const int64_t na = apply_A_elements<T>(m, u, y, s, m->wk.dpart);
  const int64_t ng = launch_gs<T>(m, y, s, u, m->wk.dpart + na, u);
  const int64_t n = na + ng;
  reduce_partials(m, n, dst, mode, s);
}

// --- fine and coarse preconditioner -----------------------------------------
template <int N, typename T>
void launch_fdm(sem_mesh m, const T* r, hipStream_t s) {
  T* zc = ZOp<T>(m);
  T* zx = zc + m->T.E * (int64_t)m->T.n1 * m->T.n1 * m->T.n1;
  hipLaunchKernelGGL((fdm_kernel<N, T>), dim3((unsigned)xcd_grid((m->T.E + fdm_ppb<N>() - 1) / fdm_ppb<N>())), dim3(fdm_threads<N>()), 0, s, r, zc, zx,
                     m->ip.p, m->xdest.p, Sp<T>(m), Lp<T>(m), Hp<T>(m), m->order.p, m->T.E,
                     (T)m->T.kappa, (T)m->T.cmass, m->per_elem ? KEp<T>(m) : nullptr,
                     m->per_elem ? CEp<T>(m) : nullptr);
  SEM_HIP(hipGetLastError());
}

// element-wise sum of the corrections (+ coarse interpolation) into z and w
template <int N, typename T>
int64_t launch_schwarz_sum(sem_mesh m, T* z, bool fine, const double* Zv, hipStream_t s, const T* rd,
                           double* dpart) {
  constexpr int EPB = ax_epb<N>();
  const T* zc = ZOp<T>(m);
  const T* zx = zc + m->T.E * (int64_t)m->T.n1 * m->T.n1 * m->T.n1;
  const int64_t grid = xcd_grid((m->T.E + EPB - 1) / EPB);
  hipLaunchKernelGGL((schwarz_sum_kernel<N, T, EPB>), dim3((unsigned)grid), dim3(EPB * (N + 1) * (N + 1)), 0, s, z,
                     Wp<T>(m), zc, zx, m->rec.p, m->dir.p, m->order.p, m->T.E, (int)fine, Zv, m->phi.p, rd, dpart);
  SEM_HIP(hipGetLastError());
  return grid;
}

// the preconditioner's result from the patch corrections and the coarse
// interpolation; with dpart, also the partial sums of rd . z (returns their count)
template <typename T>
int64_t schwarz_sum(sem_mesh m, T* z, bool fine, const double* Zv, hipStream_t s, const T* rd = nullptr,
                    double* dpart = nullptr) {
  int64_t na = 0;
  switch (m->T.N) {
#define CASE(NN)                                                     \
  case NN:                                                           \
    na = launch_schwarz_sum<NN, T>(m, z, fine, Zv, s, rd, dpart);    \
    break;
    CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14)
    CASE(15)
#undef CASE
    default:
      throw Error{SEM_EUNSUPPORTED, "order not compiled"};
  }
  const int64_t ng = launch_gs<T>(m, z, s, rd, dpart != nullptr ? dpart + na : nullptr);
  return na + ng;
}

template <int N, typename T>
void launch_restrict(sem_mesh m, const T* r, hipStream_t s) {
  hipLaunchKernelGGL((restrict_kernel<N, T>), dim3((unsigned)xcd_grid(m->T.E)), dim3((N + 1) * (N + 1)), 0, s, r,
                     m->Re.p, m->rec.p, m->phi.p, m->order.p, m->T.E);
  SEM_HIP(hipGetLastError());
}

template <typename T>
void fdm_and_restrict(sem_mesh m, const T* r, bool fine, bool coarse, hipStream_t s) {
  switch (m->T.N) {
#define CASE(NN)                                        \
  case NN:                                              \
    if (fine) launch_fdm<NN, T>(m, r, s);               \
    if (coarse) launch_restrict<NN, T>(m, r, s);        \
    break;
    CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14)
    CASE(15)
#undef CASE
    default:
      throw Error{SEM_EUNSUPPORTED, "order not compiled"};
  }
}

// one tiled launch of the forward (large nodes) or backward sweep at a height
template <int RW, bool SPLIT>
void launch_coarse_fwd_t(sem_mesh m, hipStream_t s, const RowItem* tiles, int64_t n) {
  hipLaunchKernelGGL((coarse_fwd_kernel<RW, SPLIT>), dim3((unsigned)n), dim3(256), 0, s, m->Wlev.p, m->cvec.p,
                     (const double*)m->Ylev.p, (const double*)m->fwd_pool.p, m->fnodes.p, tiles);
}

template <int RW, bool SPLIT>
void launch_coarse_bwd_t(sem_mesh m, hipStream_t s, const RowItem* tiles, int64_t n) {
  hipLaunchKernelGGL((coarse_bwd_kernel<RW, SPLIT>), dim3((unsigned)n), dim3(256), 0, s, m->Xlev.p,
                     (const double*)m->Wlev.p, (const double*)m->bwd_pool.p, m->fb_idx.p, m->fnodes.p, tiles);
}

void launch_coarse_fwd(sem_mesh m, hipStream_t s, const CoarseTileShape& t, const RowItem* tiles, int64_t n) {
  if (t.rw == 4)
    launch_coarse_fwd_t<4, false>(m, s, tiles, n);
  else if (!t.split)
    launch_coarse_fwd_t<2, false>(m, s, tiles, n);
  else
    launch_coarse_fwd_t<2, true>(m, s, tiles, n);
}

void launch_coarse_bwd(sem_mesh m, hipStream_t s, const CoarseTileShape& t, const RowItem* tiles, int64_t n) {
  if (t.rw == 4)
    launch_coarse_bwd_t<4, false>(m, s, tiles, n);
  else if (!t.split)
    launch_coarse_bwd_t<2, false>(m, s, tiles, n);
  else
    launch_coarse_bwd_t<2, true>(m, s, tiles, n);
}

// Rlev (coarse order) -> Zv (vertex order): nested-dissection sweeps
void coarse_sweeps(sem_mesh m, hipStream_t s) {
  const HostTables& T = m->T;
  const int H = T.n_heights;
  for (int h = 0; h < H; ++h) {
    const int64_t ny = T.fy_off[h + 1] - T.fy_off[h], nr = T.fr_off[h + 1] - T.fr_off[h];
    const int64_t ns = T.fs_off[h + 1] - T.fs_off[h];
    if (ny > 0)  // rows of the large nodes (small nodes assemble their own)
      hipLaunchKernelGGL(coarse_assemble_kernel, dim3((unsigned)blocks_for(8 * ny)), dim3(kGS), 0, s, m->Ylev.p,
                         (const double*)m->Rlev.p, (const double*)m->cvec.p, m->ct_off.p, m->ct_pos.p,
                         m->fy_items.p + T.fy_off[h], ny);
    if (ns > 0)
      hipLaunchKernelGGL(coarse_fwd_small_kernel, dim3((unsigned)((ns + 3) / 4)), dim3(256), 0, s, m->Wlev.p,
                         m->cvec.p, (const double*)m->Rlev.p, (const int32_t*)m->ct_off.p,
                         (const int32_t*)m->ct_pos.p, (const double*)m->fwd_pool.p, m->fnodes.p,
                         m->fs_items.p + T.fs_off[h], ns);
    if (nr > 0)
      launch_coarse_fwd(m, s, T.fr_shape[h], m->fr_items.p + T.fr_off[h], nr);
    SEM_HIP(hipGetLastError());
  }
  for (int h = H - 1; h >= 0; --h) {
    const int64_t nb = T.br_off[h + 1] - T.br_off[h];
    if (nb == 0) continue;
    launch_coarse_bwd(m, s, T.br_shape[h], m->br_items.p + T.br_off[h], nb);
    SEM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(coarse_scatter_kernel, dim3((unsigned)blocks_for(T.V)), dim3(kGS), 0, s, m->Zv.p, m->Xlev.p,
                     m->cidx.p, T.V);
  SEM_HIP(hipGetLastError());
}

void release_coarse_graph(sem_mesh m) {
  if (m->coarse_graph) (void)hipGraphExecDestroy(m->coarse_graph);
  m->coarse_graph = nullptr;
  if (m->amg_graph) (void)hipGraphExecDestroy(m->amg_graph);
  m->amg_graph = nullptr;
}

// --- aggregation AMG (Section 4.1, "Algebraic multigrid") ------------------
constexpr double kAmgOmega = 2.0 / 3.0;  // damped Jacobi

// host hierarchy -> device (work vectors per level, Jacobi weights omega / a_ii)
void amg_setup(sem_mesh m) {
  const HostTables& T = m->T;
  m->amg.clear();
  if (T.nc == 0) return;
  AmgHierarchy H;
  build_amg(T, H);
  for (const AmgLevel& L : H.levels) {
    auto d = std::make_unique<sem_mesh_s::AmgDev>();
    d->n = L.n;
    d->off.upload(L.off.data(), L.off.size());
    d->col.upload(L.col.data(), L.col.size());
    d->val.upload(L.val.data(), L.val.size());
    std::vector<double> wd(L.n);
    for (int64_t i = 0; i < L.n; ++i) wd[i] = kAmgOmega / L.diag[i];
    d->wd.upload(wd.data(), wd.size());
    if (!L.agg.empty()) {
      d->agg.upload(L.agg.data(), L.agg.size());
      d->moff.upload(L.moff.data(), L.moff.size());
      d->mem.upload(L.mem.data(), L.mem.size());
    }
    for (DBuf<double>* b : {&d->B, &d->X, &d->R, &d->T, &d->V, &d->W, &d->B2, &d->V2, &d->W2}) b->alloc(L.n);
    m->amg.push_back(std::move(d));
  }
  m->amg_inv.upload(H.coarse_inv.data(), H.coarse_inv.size());
  m->amg_sc.alloc(5 * H.levels.size());
  m->amg_nd.upload(H.nd_of.data(), H.nd_of.size());
  std::vector<int32_t> pos(T.nc);
  for (size_t q = 0; q < H.nd_of.size(); ++q) pos[H.nd_of[q]] = (int32_t)q;
  m->amg_pos.upload(pos.data(), pos.size());
}

void amg_fcg2(sem_mesh m, int l, const double* b, double* x, hipStream_t s);

// one K-cycle on level l: x ~= A_l^{-1} b
void amg_kcycle(sem_mesh m, int l, const double* b, double* x, hipStream_t s) {
  const int L = (int)m->amg.size() - 1;
  auto& d = *m->amg[l];
  const int64_t n = d.n;
  const unsigned g = (unsigned)blocks_for(n);
  if (l == L) {
    hipLaunchKernelGGL(amg_gemv_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, x, m->amg_inv.p, b, n);
    SEM_HIP(hipGetLastError());
    return;
  }
  auto& c = *m->amg[l + 1];
  hipLaunchKernelGGL(amg_presmooth_kernel, dim3(g), dim3(kGS), 0, s, x, d.R.p, b, d.wd.p, d.off.p, d.col.p, d.val.p,
                     n);
  hipLaunchKernelGGL(amg_restrict_kernel, dim3((unsigned)blocks_for(c.n)), dim3(kGS), 0, s, c.B.p, d.R.p, d.moff.p,
                     d.mem.p, c.n);
  SEM_HIP(hipGetLastError());
  if (l + 1 == L)
    amg_kcycle(m, l + 1, c.B.p, c.X.p, s);
  else
    amg_fcg2(m, l + 1, c.B.p, c.X.p, s);
  hipLaunchKernelGGL(amg_prolong_kernel, dim3(g), dim3(kGS), 0, s, d.T.p, x, c.X.p, d.agg.p, n);
  hipLaunchKernelGGL(amg_post_kernel, dim3(g), dim3(kGS), 0, s, x, d.T.p, b, d.off.p, d.col.p, d.val.p, d.wd.p, n);
  SEM_HIP(hipGetLastError());
}

// two flexible-CG steps on level l preconditioned by the K-cycle of level l
void amg_fcg2(sem_mesh m, int l, const double* b, double* x, hipStream_t s) {
  auto& d = *m->amg[l];
  const int64_t n = d.n;
  const unsigned g = (unsigned)blocks_for(n);
  double* sc = m->amg_sc.p + 5 * l;
  amg_kcycle(m, l, b, d.V.p, s);
  hipLaunchKernelGGL(amg_spmv_kernel, dim3(g), dim3(kGS), 0, s, d.W.p, d.V.p, d.off.p, d.col.p, d.val.p, n);
  hipLaunchKernelGGL((amg_dots_kernel<2>), dim3(1), dim3(1024), 0, s, sc, 0, d.V.p, b, (const double*)d.W.p,
                     (const double*)nullptr, n);
  hipLaunchKernelGGL(amg_r2_kernel, dim3(g), dim3(kGS), 0, s, d.B2.p, b, d.W.p, sc, n);
  SEM_HIP(hipGetLastError());
  amg_kcycle(m, l, d.B2.p, d.V2.p, s);
  hipLaunchKernelGGL(amg_spmv_kernel, dim3(g), dim3(kGS), 0, s, d.W2.p, d.V2.p, d.off.p, d.col.p, d.val.p, n);
  hipLaunchKernelGGL((amg_dots_kernel<3>), dim3(1), dim3(1024), 0, s, sc, 2, d.V2.p, (const double*)d.W.p,
                     (const double*)d.W2.p, (const double*)d.B2.p, n);
  hipLaunchKernelGGL(amg_combine_kernel, dim3(g), dim3(kGS), 0, s, x, d.V.p, d.V2.p, sc, n);
  SEM_HIP(hipGetLastError());
}

// Rlev (coarse order) -> Zv (vertex order) by one K-cycle
void amg_sweeps(sem_mesh m, hipStream_t s) {
  const HostTables& T = m->T;
  auto& d0 = *m->amg[0];
  hipLaunchKernelGGL(amg_in_kernel, dim3((unsigned)blocks_for(d0.n)), dim3(kGS), 0, s, d0.B.p, m->Rlev.p,
                     m->amg_nd.p, d0.n);
  amg_kcycle(m, 0, d0.B.p, d0.X.p, s);
  hipLaunchKernelGGL(amg_out_kernel, dim3((unsigned)blocks_for(T.V)), dim3(kGS), 0, s, m->Zv.p, d0.X.p, m->cidx.p,
                     m->amg_pos.p, T.V);
  SEM_HIP(hipGetLastError());
}

// Capture the coarse solve of the current coarse solver (nested-dissection
// sweeps or one K-cycle) once, on a private stream; the preconditioner replays
// it on the caller's stream.  Built at set-up and whenever the coarse matrix or
// solver changes.
void build_coarse_graph(sem_mesh m) {
  if (m->T.nc == 0) return;
  const bool amg = m->coarse_solver == SEM_COARSE_AMG;
  if (amg && m->amg.empty()) throw Error{SEM_EINVAL, "AMG hierarchy not built"};
  hipGraphExec_t& exec = amg ? m->amg_graph : m->coarse_graph;
  if (exec) return;
  if (m->no_alloc) throw Error{SEM_EINVAL, "coarse-solve graph missing (it is built at set-up)"};
  if (!m->capture_stream) SEM_HIP(hipStreamCreateWithFlags(&m->capture_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  SEM_HIP(hipStreamBeginCapture(m->capture_stream, hipStreamCaptureModeThreadLocal));
  try {
    if (amg)
      amg_sweeps(m, m->capture_stream);
    else
      coarse_sweeps(m, m->capture_stream);
  } catch (...) {
    (void)hipStreamEndCapture(m->capture_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  SEM_HIP(hipStreamEndCapture(m->capture_stream, &g));
  hipError_t err = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (err != hipSuccess) {
    exec = nullptr;
    throw Error{SEM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(err)};
  }
}

// Rlev (coarse order) -> Zv (vertex order): the coarse solve P_0
void coarse_solve_tree(sem_mesh m, hipStream_t s) {
  const bool amg = m->coarse_solver == SEM_COARSE_AMG;
  if (m->direct_coarse) {  // inside an enclosing capture: launch the kernels themselves
    if (amg)
      amg_sweeps(m, s);
    else
      coarse_sweeps(m, s);
    return;
  }
  build_coarse_graph(m);
  SEM_HIP(hipGraphLaunch(amg ? m->amg_graph : m->coarse_graph, s));
}

// the second stream (and its fork/join events) that runs the coarse chain
// beside the patch solves; created at set-up
void ensure_side_stream(sem_mesh m) {
  if (m->side_stream) return;
  if (m->no_alloc) throw Error{SEM_EINVAL, "side stream missing (it is created at set-up)"};
  SEM_HIP(hipStreamCreateWithFlags(&m->side_stream, hipStreamNonBlocking));
  SEM_HIP(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
  SEM_HIP(hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming));
}

template <typename T>
void precond_dot(sem_mesh m, const T* r, T* z, int pc, int dot_dst, int dot_mode, hipStream_t s,
                 bool coarse_started = false);

template <typename T>
void precond(sem_mesh m, const T* r, T* z, int pc, hipStream_t s) {
  precond_dot<T>(m, r, z, pc, -1, 0, s);
}

template <typename TA, typename TB>
void dot(sem_mesh m, const TA* a, const TB* b, int dst, int mode, hipStream_t s);

// z = P r; with dot_dst >= 0 also r . z into scalar slot dot_dst (dot_final
// mode dot_mode), taken from the preconditioner's own output kernels
// coarse_started: the coarse chain of this application (restriction, coarse
// solve) is already running on the side stream (pcg_core forks it right after
// the update of r); only its join remains.
template <typename T>
void precond_dot(sem_mesh m, const T* r, T* z, int pc, int dot_dst, int dot_mode, hipStream_t s,
                 bool coarse_started) {
  const HostTables& H = m->T;
  const bool fine = pc & SEM_PC_FINE, coarse = (pc & SEM_PC_COARSE) && H.nc > 0;
  if (pc == SEM_PC_NONE) {
    hipLaunchKernelGGL((copy_kernel<T, T>), dim3(grid_stride_blocks(H.n_global)), dim3(kGS), 0, s, z, r, H.n_global);
    SEM_HIP(hipGetLastError());
    if (dot_dst >= 0) dot<T, T>(m, r, z, dot_dst, dot_mode, s);
    return;
  }
  // The coarse and fine parts are independent until the final sum: the
  // coarse chain (restriction, coarse sweeps) runs on a second stream while
  // the patch solves run on the caller's stream; both join before the sum.
  // The patch solves are issued first, so that the host's launches of the
  // coarse chain do not hold them back.
  hipStream_t sc = s;
  if (coarse_started) {
    fdm_and_restrict<T>(m, r, true, false, s);
    SEM_HIP(hipStreamWaitEvent(s, m->ev_join, 0));
  } else if (coarse && fine) {
    ensure_side_stream(m);
    SEM_HIP(hipEventRecord(m->ev_fork, s));
    SEM_HIP(hipStreamWaitEvent(m->side_stream, m->ev_fork, 0));
    sc = m->side_stream;
  }
  if (coarse_started) {
    // fine part and join done above
  } else {
  if (fine) fdm_and_restrict<T>(m, r, true, false, s);
  if (coarse) {
    fdm_and_restrict<T>(m, r, false, true, sc);
    hipLaunchKernelGGL(restrict_gather_kernel, dim3((unsigned)blocks_for(H.V)), dim3(kGS), 0, sc, m->Rlev.p, m->Re.p,
                       m->vinc_off.p, m->vinc_ec.p, m->cidx.p, H.V);
    SEM_HIP(hipGetLastError());
    coarse_solve_tree(m, sc);
  }
  if (sc != s) {
    SEM_HIP(hipEventRecord(m->ev_join, sc));
    SEM_HIP(hipStreamWaitEvent(s, m->ev_join, 0));
  }
  }
  if (dot_dst < 0) {
    schwarz_sum<T>(m, z, fine, coarse ? (const double*)m->Zv.p : nullptr, s);
    return;
  }
  const int64_t n = schwarz_sum<T>(m, z, fine, coarse ? (const double*)m->Zv.p : nullptr, s, r, m->wk.dpart);
  reduce_partials(m, n, dot_dst, dot_mode, s);
}

// PCG's update of r fused with the coarse restriction (update_r_restrict_kernel),
// r . r into scalar slot 4, then the rest of the coarse chain (vertex sums,
// coarse solve) forked onto the side stream; precond_dot(..., true) joins it.
template <int N, typename T>
int64_t launch_update_r_restrict(sem_mesh m, T* r, const T* w, hipStream_t s) {
  const int64_t grid = xcd_grid(m->T.E);
  hipLaunchKernelGGL((update_r_restrict_kernel<N, T>), dim3((unsigned)grid), dim3((N + 1) * (N + 1)), 0, s, r, w,
                     (const double*)m->wk.sc, m->Re.p, m->wk.dpart, m->rec.p, (const double*)m->phi.p, m->order.p,
                     m->T.E);
  SEM_HIP(hipGetLastError());
  return grid;
}

template <typename T>
void update_r_and_fork_coarse(sem_mesh m, T* r, const T* w, hipStream_t s) {
  int64_t n = 0;
  switch (m->T.N) {
#define CASE(NN)                                             \
  case NN:                                                   \
    n = launch_update_r_restrict<NN, T>(m, r, w, s);         \
    break;
    CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14)
    CASE(15)
#undef CASE
    default:
      throw Error{SEM_EUNSUPPORTED, "order not compiled"};
  }
  reduce_partials(m, n, 4, 0, s);
  const HostTables& H = m->T;
  ensure_side_stream(m);
  hipStream_t sc = m->side_stream;
  SEM_HIP(hipEventRecord(m->ev_fork, s));
  SEM_HIP(hipStreamWaitEvent(sc, m->ev_fork, 0));
  hipLaunchKernelGGL(restrict_gather_kernel, dim3((unsigned)blocks_for(H.V)), dim3(kGS), 0, sc, m->Rlev.p, m->Re.p,
                     m->vinc_off.p, m->vinc_ec.p, m->cidx.p, H.V);
  SEM_HIP(hipGetLastError());
  coarse_solve_tree(m, sc);
  SEM_HIP(hipEventRecord(m->ev_join, sc));
}

// --- coarse factorisation (set-up), multifrontal in post-order.  Node t's
// front F (f = s + b, column-major) holds the entries of A_c with the smaller
// index in t's own range, plus the update matrices of its children
// (extend-add).  Then S = F_II, S^-1 by Cholesky, W^T = S^-1 F_IB,
// W = F_BI S^-1 and the update U = F_BB - W F_IB for the parent.
void factor_coarse(sem_mesh m) {
  HostTables& T = m->T;
  release_coarse_graph(m);
  if (m->coarse_solver == SEM_COARSE_AMG) amg_setup(m);
  m->cidx.upload(T.cidx.data(), T.cidx.size());
  const size_t nc = std::max<int64_t>(T.nc, 1);
  m->Rlev.alloc(nc);
  m->Ylev.alloc(nc);
  m->Wlev.alloc(nc);
  m->Xlev.alloc(nc);
  if (T.nc == 0) {
    m->fwd_pool.release();
    m->bwd_pool.release();
    return;
  }
  // fronts are factored densely: bound their size
  if (T.max_front > 16384)
    throw Error{SEM_EUNSUPPORTED, "coarse front of " + std::to_string(T.max_front) + " vertices exceeds 16384"};
  m->fnodes.upload(T.fnodes.data(), T.fnodes.size());
  m->fb_idx.upload(T.fb_idx.data(), T.fb_idx.size());
  m->ct_off.upload(T.ct_off.data(), T.ct_off.size());
  m->ct_pos.upload(T.ct_pos.data(), T.ct_pos.size());
  m->fy_items.upload(T.fy_items.data(), T.fy_items.size());
  m->fr_items.upload(T.fr_items.data(), T.fr_items.size());
  m->br_items.upload(T.br_items.data(), T.br_items.size());
  m->fs_items.upload(T.fs_items.data(), T.fs_items.size());
  m->cvec.alloc(std::max<int64_t>(T.c_size, 1));
  m->fwd_pool.alloc(T.fwd_size);
  m->bwd_pool.alloc(std::max<int64_t>(T.bwd_size, 1));
  rocblas_handle hb;
  if (rocblas_create_handle(&hb) != rocblas_status_success) throw Error{SEM_EHIP, "rocblas_create_handle failed"};
  std::unique_ptr<std::remove_pointer<rocblas_handle>::type, decltype(&rocblas_destroy_handle)> guard(
      hb, rocblas_destroy_handle);
  const int64_t mf = T.max_front;
  DBuf<double> Fd, Ust;
  DBuf<int32_t> mapd;
  DBuf<rocblas_int> info;
  info.alloc(1);
  Fd.alloc((size_t)mf * mf);
  Ust.alloc(std::max<int64_t>(T.ustack_size, 1));
  mapd.alloc((size_t)mf);
  std::vector<double> cols;
  std::vector<int32_t> map;
  std::vector<int64_t> u_at(T.fnodes.size(), -1);  // update matrix position in the stack
  int64_t top = 0;
  const double one = 1.0, zero = 0.0, mone = -1.0;
  for (size_t q = 0; q < T.fnodes.size(); ++q) {
    const FrontNode& F = T.fnodes[q];
    const int64_t s = F.s, b = F.b, f = s + b, end = F.off + s;
    const int32_t* B = T.fb_idx.data() + F.bidx;
    auto local = [&](int64_t g) -> int64_t {
      if (g >= F.off && g < end) return g - F.off;
      const int32_t* p = std::lower_bound(B, B + b, (int32_t)g);
      if (p == B + b || *p != g) throw Error{SEM_EMESH, "coarse front: entry outside the node's front"};
      return s + (p - B);
    };
    // columns of the own vertices: A_c(idx, own) (entries towards eliminated
    // vertices were taken by the descendants' fronts)
    cols.assign((size_t)f * s, 0.0);
    for (int64_t r = 0; r < s; ++r)
      for (int32_t k = T.ac_off[F.off + r]; k < T.ac_off[F.off + r + 1]; ++k) {
        if (T.ac_col[k] < F.off) continue;
        cols[(size_t)r * f + local(T.ac_col[k])] = T.ac_val[k];
      }
    SEM_HIP(hipMemcpy(Fd.p, cols.data(), cols.size() * sizeof(double), hipMemcpyHostToDevice));
    if (b > 0) {
      SEM_HIP(hipMemset(Fd.p + s * f, 0, (size_t)b * f * sizeof(double)));
      hipLaunchKernelGGL(front_transpose_kernel, dim3((unsigned)blocks_for(s * b)), dim3(kGS), 0, 0, Fd.p, f, s, b);
      SEM_HIP(hipGetLastError());
    }
    // extend-add the children's update matrices, then pop them
    int64_t first = -1;
    for (int32_t c : T.fchildren[q]) {
      const FrontNode& C = T.fnodes[c];
      if (C.b == 0) continue;
      map.resize(C.b);
      for (int32_t k = 0; k < C.b; ++k) map[k] = (int32_t)local(T.fb_idx[C.bidx + k]);
      SEM_HIP(hipMemcpy(mapd.p, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      hipLaunchKernelGGL(front_extend_add_kernel, dim3((unsigned)blocks_for((int64_t)C.b * C.b)), dim3(kGS), 0, 0,
                         Fd.p, f, (const double*)Ust.p + u_at[c], (int64_t)C.b, (const int32_t*)mapd.p);
      SEM_HIP(hipGetLastError());
      if (first < 0 || u_at[c] < first) first = u_at[c];
    }
    if (first >= 0) top = first;
    // S^-1 in place (lower triangle), mirrored
    if (rocsolver_dpotrf(hb, rocblas_fill_lower, (rocblas_int)s, Fd.p, (rocblas_int)f, info.p) !=
        rocblas_status_success)
      throw Error{SEM_EHIP, "rocsolver_dpotrf failed"};
    rocblas_int ih = 0;
    SEM_HIP(hipMemcpy(&ih, info.p, sizeof(ih), hipMemcpyDeviceToHost));
    if (ih != 0) throw Error{SEM_EMESH, "coarse matrix is not positive definite"};
    if (rocsolver_dpotri(hb, rocblas_fill_lower, (rocblas_int)s, Fd.p, (rocblas_int)f, info.p) !=
        rocblas_status_success)
      throw Error{SEM_EHIP, "rocsolver_dpotri failed"};
    hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)blocks_for(s * s)), dim3(kGS), 0, 0, Fd.p, s, f);
    SEM_HIP(hipGetLastError());
    // Large node: forward [S^-1 ; W] row-major = column-major s x (s + b):
    // [S^-1 | W^T].  Small node: forward [S^-1 ; W] column-major (ld s + b).
    // Backward, every node: W^T row-major = W column-major (ld b).
    double* X = m->fwd_pool.p + F.fwd;
    double* Wb = m->bwd_pool.p + F.bwd;
    const int64_t ldx = F.small ? f : s;
    SEM_HIP(hipMemcpy2D(X, ldx * sizeof(double), Fd.p, f * sizeof(double), s * sizeof(double), s,
                        hipMemcpyDeviceToDevice));
    if (b > 0) {
      const rocblas_int si = (rocblas_int)s, bi = (rocblas_int)b, fi = (rocblas_int)f;
      // W = F_BI S^-1  (b x s), column-major (ld b) for the backward sweep
      double* W = Wb;
      const rocblas_int ldw = bi;
      if (rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, bi, si, si, &one, Fd.p + s, fi, Fd.p,
                        fi, &zero, W, ldw) != rocblas_status_success)
        throw Error{SEM_EHIP, "rocblas_dgemm failed"};
      if (F.small) {
        // forward rows s.. of the column-major [S^-1; W]
        SEM_HIP(hipMemcpy2D(X + s, f * sizeof(double), W, b * sizeof(double), b * sizeof(double), s,
                            hipMemcpyDeviceToDevice));
      } else {
        // W^T = S^-1 F_IB  (s x b), the forward columns s..
        if (rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, si, bi, si, &one, Fd.p, fi,
                          Fd.p + s * f, fi, &zero, X + s * s, si) != rocblas_status_success)
          throw Error{SEM_EHIP, "rocblas_dgemm failed"};
      }
      // U = F_BB - W F_IB, pushed for the parent
      if (top + b * b > std::max<int64_t>(T.ustack_size, 1)) throw Error{SEM_EHIP, "coarse update stack overflow"};
      double* U = Ust.p + top;
      SEM_HIP(hipMemcpy2D(U, b * sizeof(double), Fd.p + s + s * f, f * sizeof(double), b * sizeof(double), b,
                          hipMemcpyDeviceToDevice));
      if (rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, bi, bi, si, &mone, W, ldw, Fd.p + s * f,
                        fi, &one, U, bi) != rocblas_status_success)
        throw Error{SEM_EHIP, "rocblas_dgemm failed"};
      u_at[q] = top;
      top += b * b;
    }
  }
  SEM_HIP(hipDeviceSynchronize());
  build_coarse_graph(m);
}

// D (n1 x n1, row-major) followed by the even/odd split that the line-phase
// operator kernel uses for D and for D^T (see line_pairs in the kernels):
// rows q < H = n1/2 of (D[q][m] + D[q][n1-1-m]) / 2 for m < H, D[q][H] when
// n1 is odd, (D[q][m] - D[q][n1-1-m]) / 2 for m < H; for odd n1 a last row of
// the middle output's (D[H][m] - D[H][n1-1-m]) / 2.  The other kernels read
// only the first n1 x n1 entries.
std::vector<double> d_with_split(const std::vector<double>& D, int n1) {
  const int H = n1 / 2, od = n1 % 2;
  std::vector<double> out(D);
  for (int t = 0; t < 2; ++t) {
    auto d = [&](int q, int m) { return t == 0 ? D[(size_t)q * n1 + m] : D[(size_t)m * n1 + q]; };
    for (int q = 0; q < H; ++q) {
      for (int m = 0; m < H; ++m) out.push_back(0.5 * (d(q, m) + d(q, n1 - 1 - m)));
      if (od) out.push_back(d(q, H));
      for (int m = 0; m < H; ++m) out.push_back(0.5 * (d(q, m) - d(q, n1 - 1 - m)));
    }
    if (od)
      for (int m = 0; m < H; ++m) out.push_back(0.5 * (d(H, m) - d(H, n1 - 1 - m)));
  }
  return out;
}

void upload_all(sem_mesh m) {
  HostTables& T = m->T;
  SEM_HIP(hipSetDevice(m->device));
  m->rec.upload(T.rec.data(), T.rec.size());
  m->order.upload(T.order.data(), T.order.size());
  m->vinc_off.upload(T.vinc_off.data(), T.vinc_off.size());
  m->einc_off.upload(T.einc_off.data(), T.einc_off.size());
  m->dir.upload(T.dir.data(), T.dir.size());
  m->fcount.upload(T.fcount.data(), T.fcount.size());
  {
    // vertex incidence -> element * 8 + corner
    std::vector<int32_t> ec(T.vinc_off.back());
    std::vector<int32_t> fill(T.vinc_off.begin(), T.vinc_off.end() - 1);
    const int N = T.N;
    for (int64_t e = 0; e < T.E; ++e)
      for (int p = 0; p < 8; ++p) {
        const int64_t v = gid_of(T, e, (p & 1) * N, ((p >> 1) & 1) * N, (p >> 2) * N);
        ec[fill[v]++] = (int32_t)(e * 8 + p);
      }
    m->vinc_ec.upload(ec.data(), ec.size());
  }
  m->G64.upload(T.G.data(), T.G.size());
  const std::vector<double> Dx = d_with_split(T.D, T.n1);
  m->D64.upload(Dx.data(), Dx.size());
  m->X864.upload(T.X8.data(), T.X8.size());
  std::vector<double> tq(T.t);
  tq.insert(tq.end(), T.rho.begin(), T.rho.end());
  m->tq64.upload(tq.data(), tq.size());
  m->w64.alloc(T.w_size);
  m->ip.upload(T.ip.data(), T.ip.size());
  m->xdest.upload(T.xdest.data(), T.xdest.size());
  m->S64.upload(T.S.data(), T.S.size());
  m->lam64.upload(T.lam.data(), T.lam.size());
  m->h64.upload(T.h.data(), T.h.size());
  // consumer slots no patch writes (NULL) stay zero for good
  m->zo64.alloc((size_t)T.E * T.np * T.np * T.np);
  SEM_HIP(hipMemset(m->zo64.p, 0, m->zo64.n * sizeof(double)));
  if (m->fp32) {
    auto G32 = convert<float>(T.G);
    m->G32.upload(G32.data(), G32.size());
    auto D32 = convert<float>(Dx);
    m->D32.upload(D32.data(), D32.size());
    auto X832 = convert<float>(T.X8);
    m->X832.upload(X832.data(), X832.size());
    auto tq32 = convert<float>(tq);
    m->tq32.upload(tq32.data(), tq32.size());
    m->w32.alloc(T.w_size);
    auto S32 = convert<float>(T.S);
    m->S32.upload(S32.data(), S32.size());
    auto l32 = convert<float>(T.lam);
    m->lam32.upload(l32.data(), l32.size());
    auto h32 = convert<float>(T.h);
    m->h32.upload(h32.data(), h32.size());
    m->zo32.alloc((size_t)T.E * T.np * T.np * T.np);
    SEM_HIP(hipMemset(m->zo32.p, 0, m->zo32.n * sizeof(float)));
  }
  // Phi_I(t_i): row I = 0, 1
  std::vector<double> phi(2 * T.n1);
  for (int i = 0; i < T.n1; ++i) {
    phi[i] = 0.5 * (1.0 - T.t[i]);
    phi[T.n1 + i] = 0.5 * (1.0 + T.t[i]);
  }
  m->phi.upload(phi.data(), phi.size());
  m->Re.alloc((size_t)T.E * 8);
  m->Zv.alloc(std::max<int64_t>(T.V, 1));
  m->part.alloc(kRedBlocks);
  m->sc.alloc(16);
  ensure_side_stream(m);
  factor_coarse(m);
}

// partial dot products of the operator and the preconditioner's sum (one per
// element workgroup at most, one per gather workgroup)
size_t dpart_count(sem_mesh m) { return (size_t)(xcd_grid(m->T.E) + blocks_for(m->T.base_i)); }

// the handle's own solve buffers (allocated on first need) as the work of the next solve
void ensure_work(sem_mesh m, bool need32) {
  const int64_t n = m->T.n_global;
  for (auto& b : m->v64)
    if (b.n != (size_t)n) b.alloc(n);
  const size_t nd = dpart_count(m);
  if (m->dpart.n < nd) m->dpart.alloc(nd);
  if (need32)
    for (auto& b : m->v32)
      if (b.n != (size_t)n) b.alloc(n);
  for (int q = 0; q < 5; ++q) {
    m->wk.v64[q] = m->v64[q].p;
    m->wk.v32[q] = need32 ? m->v32[q].p : nullptr;
  }
  m->wk.part = m->part.p;
  m->wk.sc = m->sc.p;
  m->wk.dpart = m->dpart.p;
  if (!m->check_host) SEM_HIP(hipHostMalloc((void**)&m->check_host, 4 * sizeof(double), hipHostMallocDefault));
  if (!m->ev_check) SEM_HIP(hipEventCreateWithFlags(&m->ev_check, hipEventDisableTiming));
}

// --- static scratch of sem_pcg_solve_noalloc ------------------------------
// The work of one solve (Algorithm 1's scalars, partial sums and the five FP64
// vectors, plus five FP32 vectors for the refined form) as views into one
// file-scope device array, for callers that cannot allocate device memory.
// Every device holds its own copy of the array, at its own address, resolved
// once per device at set-up (create_mesh) with that device current; host code
// uses only that address, never the array's name.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;  // by device id: the device address of scratch (NULL until resolved)

void resolve_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize((size_t)device + 1, nullptr);
  if (g_scratch_dev[device] != nullptr) return;
  void* p = nullptr;
  SEM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (p == nullptr) throw Error{SEM_EHIP, "hipGetSymbolAddress(scratch) returned NULL"};
  g_scratch_dev[device] = static_cast<double*>(p);
}

double* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < (int)g_scratch_dev.size() ? g_scratch_dev[device] : nullptr;
}

// byte offsets of one solve's work inside the scratch array (256-aligned parts)
struct ScratchLayout {
  size_t sc, part, dpart, v64, v32, total;
};

ScratchLayout scratch_layout(sem_mesh m, bool need32) {
  auto up = [](size_t bytes) { return (bytes + 255) / 256 * 256; };
  const size_t n = (size_t)m->T.n_global;
  ScratchLayout L{};
  size_t o = 0;
  L.sc = o;
  o += up(16 * sizeof(double));
  L.part = o;
  o += up(kRedBlocks * sizeof(double));
  L.dpart = o;
  o += up(dpart_count(m) * sizeof(double));
  L.v64 = o;
  o += 5 * up(n * sizeof(double));
  L.v32 = o;
  if (need32) o += 5 * up(n * sizeof(float));
  L.total = o;
  return L;
}

// the next solve's work as views into the scratch array at `base`
void scratch_work(sem_mesh m, bool need32, double* base) {
  const ScratchLayout L = scratch_layout(m, need32);
  const size_t n = (size_t)m->T.n_global;
  char* c = reinterpret_cast<char*>(base);
  const size_t s64 = (n * sizeof(double) + 255) / 256 * 256, s32 = (n * sizeof(float) + 255) / 256 * 256;
  for (int q = 0; q < 5; ++q) {
    m->wk.v64[q] = reinterpret_cast<double*>(c + L.v64 + q * s64);
    m->wk.v32[q] = need32 ? reinterpret_cast<float*>(c + L.v32 + q * s32) : nullptr;
  }
  m->wk.part = reinterpret_cast<double*>(c + L.part);
  m->wk.sc = reinterpret_cast<double*>(c + L.sc);
  m->wk.dpart = reinterpret_cast<double*>(c + L.dpart);
}

template <typename TA, typename TB>
void dot(sem_mesh m, const TA* a, const TB* b, int dst, int mode, hipStream_t s) {
  const int64_t n = m->T.n_global;
  const int nb = (int)std::min<int64_t>(kRedBlocks, blocks_for(n, kRedThreads));
  hipLaunchKernelGGL((dot_partial_kernel<TA, TB>), dim3(nb), dim3(kRedThreads), 0, s, a, b, m->wk.part, n,
                     (int)aligned16(a, b));
  SEM_HIP(hipGetLastError());
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kRedThreads), 0, s, m->wk.part, m->wk.sc, nb, dst, mode);
  SEM_HIP(hipGetLastError());
}

double read_scalar(sem_mesh m, int idx, hipStream_t s) {
  double v = 0.0;
  SEM_HIP(hipMemcpyAsync(&v, m->wk.sc + idx, sizeof(double), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  return v;
}

// One PCG solve (Algorithm 1) on vectors of type T; x, r in/out (r holds the
// residual of x, rr0 = ||r||^2).  Returns the status; *iters gets the
// iterations, *rel the last ||r|| / ||b||.  A start that already meets the
// tolerance returns at once; after a breakdown x keeps the last finite iterate
// (the vector updates skip themselves once the flag is set).
template <typename T>
int pcg_core(sem_mesh m, T* x, T* r, double bnorm2, double rr0, double rtol, int max_iter, int pc, int check_every,
             hipStream_t s, int* iters, double* rel, sem_solve_stats* st) {
  T* z;
  T* p;
  T* w;
  if constexpr (std::is_same<T, double>::value) {
    z = m->wk.v64[2];
    p = m->wk.v64[3];
    w = m->wk.v64[4];
  } else {
    z = m->wk.v32[2];
    p = m->wk.v32[3];
    w = m->wk.v32[4];
  }
  double* sc = m->wk.sc;
  const int64_t n = m->T.n_global;
  const int nb = (int)std::min<int64_t>(kRedBlocks, blocks_for(n, kRedThreads));
  const int gb = grid_stride_blocks(n);
  const double tol2 = rtol * rtol * bnorm2;
  int k = 0;
  double rr = rr0;
  *iters = 0;
  *rel = std::sqrt(rr / bnorm2);
  if (rr <= tol2) return SEM_OK;
  hipLaunchKernelGGL((fill_kernel<double>), dim3(1), dim3(kGS), 0, s, sc, 0.0, (int64_t)7);
  precond_dot<T>(m, r, z, pc, 0, 0, s);
  hipLaunchKernelGGL((copy_kernel<T, T>), dim3(gb), dim3(kGS), 0, s, p, z, n);
  int status = SEM_ENOCONV;
  bool pending_x = false;  // x += alpha p of the last iteration not yet applied
  // two-scale P with a coarse space: the update of r also restricts it, and
  // the coarse solve starts beside the convergence check and the patch solves
  const bool fused = pc == SEM_PC_TWOSCALE && m->T.nc > 0 && !m->direct_coarse;
  bool coarse_pending = false;
  // speculative ordering of the convergence check: needs the pinned read-back
  // buffer (made by an ordinary solve's set-up; not in the allocation-free one)
  const bool spec_ok = m->check_host != nullptr && m->ev_check != nullptr;
  while (k < max_iter) {
    apply_A_dot<T>(m, p, w, 1, 1, s);
    if (fused) {
      update_r_and_fork_coarse<T>(m, r, (const T*)w, s);
      coarse_pending = true;
    } else {
      hipLaunchKernelGGL((update_r_kernel<T>), dim3(nb), dim3(kRedThreads), 0, s, r, (const T*)w, (const double*)sc,
                         m->wk.part, n, (int)aligned16(r, w));
      SEM_HIP(hipGetLastError());
      hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kRedThreads), 0, s, m->wk.part, sc, nb, 4, 0);
    }
    ++k;
    pending_x = true;
    bool z_ready = false;  // the preconditioner of this step already enqueued
    if (k % check_every == 0 || k == max_iter) {
      // r^T r (slot 4) and the breakdown flag (slot 6) in one read-back.  Far
      // from the tolerance (the last r^T r above 100 tol^2) the step's
      // preconditioner is enqueued before the host waits for them, so the GPU
      // works through the round trip; if the check then ends the solve, that
      // preconditioner was spent for nothing, which this margin makes rare
      double sc46[3];
      if (spec_ok && k < max_iter && rr > 100.0 * tol2) {
        SEM_HIP(hipMemcpyAsync(m->check_host, sc + 4, sizeof(sc46), hipMemcpyDeviceToHost, s));
        SEM_HIP(hipEventRecord(m->ev_check, s));
        precond_dot<T>(m, r, z, pc, 5, 2, s, coarse_pending);
        coarse_pending = false;
        z_ready = true;
        SEM_HIP(hipEventSynchronize(m->ev_check));
        std::memcpy(sc46, m->check_host, sizeof(sc46));
      } else {
        SEM_HIP(hipMemcpyAsync(sc46, sc + 4, sizeof(sc46), hipMemcpyDeviceToHost, s));
        SEM_HIP(hipStreamSynchronize(s));
      }
      rr = sc46[0];
      const double flag = sc46[2];
      if (st && st->history && st->history_len < st->history_cap)
        st->history[st->history_len++] = std::sqrt(rr / bnorm2);
      if (flag != 0.0 || !std::isfinite(rr)) {
        status = SEM_EBREAKDOWN;
        break;
      }
      if (rr <= tol2) {
        status = SEM_OK;
        break;
      }
    }
    if (!z_ready) {
      precond_dot<T>(m, r, z, pc, 5, 2, s, coarse_pending);
      coarse_pending = false;
    }
    hipLaunchKernelGGL((update_px_kernel<T>), dim3(gb), dim3(kGS), 0, s, x, p, (const T*)z, (const double*)sc, n,
                       (int)aligned16(x, p, z));
    SEM_HIP(hipGetLastError());
    pending_x = false;
  }
  // a coarse solve forked for an iteration that did not follow: the caller's
  // stream waits for it, so no later work on the handle overlaps it
  if (coarse_pending) SEM_HIP(hipStreamWaitEvent(s, m->ev_join, 0));
  if (pending_x && status != SEM_EBREAKDOWN) {
    hipLaunchKernelGGL((update_x_kernel<T>), dim3(gb), dim3(kGS), 0, s, x, (const T*)p, (const double*)sc, n);
    SEM_HIP(hipGetLastError());
  }
  *iters = k;
  *rel = std::sqrt(rr / bnorm2);
  return status;
}

// back from per-node coefficients: the plain factors G return to the device
// (in place, so the buffers keep their addresses)
void leave_node_coefficients(sem_mesh m) {
  if (!m->per_node) return;
  m->per_node = false;
  if (m->host_only) return;
  SEM_HIP(hipSetDevice(m->device));
  SEM_HIP(hipDeviceSynchronize());
  m->G64.copy_in(m->T.G.data(), m->T.G.size());
  if (m->fp32) {
    const std::vector<float> f = convert<float>(m->T.G);
    m->G32.copy_in(f.data(), f.size());
  }
}

// kappa and c of the operator, the patch solves and the coarse matrix (whose
// values are reassembled and refactorised when they change)
void set_coefficients(sem_mesh m, double kappa, double c) {
  HostTables& T = m->T;
  if (!m->per_elem && T.kappa == kappa && T.cmass == c) return;
  leave_node_coefficients(m);
  T.kappa = kappa;
  T.cmass = c;
  T.kap_e.clear();
  T.c_e.clear();
  m->per_elem = false;
  assemble_coarse_matrix(T);
  if (m->host_only) return;
  SEM_HIP(hipSetDevice(m->device));
  SEM_HIP(hipDeviceSynchronize());
  if (c != 0.0 && m->mN64.p == nullptr) {
    m->mN64.upload(T.mN.data(), T.mN.size());
    if (m->fp32) {
      const std::vector<float> f = convert<float>(T.mN);
      m->mN32.upload(f.data(), f.size());
    }
  }
  factor_coarse(m);
}

// one kappa_e > 0 and c_e >= 0 per element (Algorithm 2): uploaded with the
// local mass m_{ijk;e} when some c_e != 0; coarse matrix reassembled
void set_element_coefficients(sem_mesh m, const double* kap, const double* c) {
  HostTables& T = m->T;
  const int64_t E = T.E;
  leave_node_coefficients(m);
  if (kap)
    T.kap_e.assign(kap, kap + E);
  else
    T.kap_e.assign(E, 1.0);
  if (c)
    T.c_e.assign(c, c + E);
  else
    T.c_e.assign(E, 0.0);
  T.kappa = T.cmass = std::nan("");
  bool any_c = false;
  for (double v : T.c_e) any_c = any_c || v != 0.0;
  assemble_coarse_matrix(T);
  m->per_elem = true;
  m->any_ce = any_c;
  if (m->host_only) return;
  SEM_HIP(hipSetDevice(m->device));
  SEM_HIP(hipDeviceSynchronize());
  m->ke64.upload(T.kap_e.data(), E);
  m->ce64.upload(T.c_e.data(), E);
  if (m->fp32) {
    const std::vector<float> kf = convert<float>(T.kap_e), cf = convert<float>(T.c_e);
    m->ke32.upload(kf.data(), E);
    m->ce32.upload(cf.data(), E);
  }
  if (any_c && m->mL64.p == nullptr) {
    m->mL64.upload(T.mass.data(), T.mass.size());
    if (m->fp32) {
      const std::vector<float> f = convert<float>(T.mass);
      m->mL32.upload(f.data(), f.size());
    }
  }
  factor_coarse(m);
}

// kappa_{ijk;e} > 0 and c_{ijk;e} >= 0 at every local node (eq. (R)): kappa
// multiplies the six factors G at its node, c the local mass.  The patch solves
// and the coarse matrix take one value per element: the mean over the
// reference cube by the GLL rule, (1/8) sum rho_i rho_j rho_k v_{ijk;e}.
void set_node_coefficients(sem_mesh m, const double* kap, const double* c) {
  HostTables& T = m->T;
  const int64_t E = T.E;
  const int n1 = T.n1;
  const int64_t NN = (int64_t)n1 * n1 * n1;
  T.kap_e.assign(E, 1.0);
  T.c_e.assign(E, 0.0);
  std::vector<double> nc(E, 0.0);
  bool any_c = false;
  for (int64_t e = 0; e < E; ++e) {
    double ks = 0.0, cs = 0.0;
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const int64_t l = e * NN + i + (int64_t)n1 * (j + (int64_t)n1 * k);
          const double w = T.rho[i] * T.rho[j] * T.rho[k] * 0.125;
          if (kap) ks += w * kap[l];
          if (c) {
            cs += w * c[l];
            if (c[l] != 0.0) nc[e] = 1.0;
          }
        }
    if (kap) T.kap_e[e] = ks;
    T.c_e[e] = cs;
    any_c = any_c || nc[e] != 0.0;
  }
  T.kappa = T.cmass = std::nan("");
  assemble_coarse_matrix(T);
  m->per_elem = true;
  m->per_node = true;
  m->any_ce = any_c;
  if (m->host_only) return;
  SEM_HIP(hipSetDevice(m->device));
  SEM_HIP(hipDeviceSynchronize());
  // factors scaled by kappa at their node; c m per local node
  std::vector<double> Gs(T.G.size());
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f)
      for (int64_t l = 0; l < NN; ++l) {
        const int64_t o = (e * 6 + f) * NN + l;
        Gs[o] = kap ? kap[e * NN + l] * T.G[o] : T.G[o];
      }
  std::vector<double> cm;
  if (any_c) {
    cm.resize((size_t)E * NN);
    for (int64_t l = 0; l < E * NN; ++l) cm[l] = c[l] * T.mass[l];
  }
  const std::vector<double> ones(E, 1.0);
  m->G64.copy_in(Gs.data(), Gs.size());
  // kappa per node for the operator kernel that rebuilds G from the vertices
  std::vector<double> kl;
  if (kap)
    kl.assign(kap, kap + E * NN);
  else
    kl.assign((size_t)E * NN, 1.0);
  m->kn64.upload(kl.data(), kl.size());
  m->ke64.upload(T.kap_e.data(), E);
  m->ce64.upload(T.c_e.data(), E);
  m->nk64.upload(ones.data(), E);
  m->nc64.upload(nc.data(), E);
  if (any_c) m->nm64.upload(cm.data(), cm.size());
  if (m->fp32) {
    const std::vector<float> Gf = convert<float>(Gs);
    m->G32.copy_in(Gf.data(), Gf.size());
    const std::vector<float> klf = convert<float>(kl);
    m->kn32.upload(klf.data(), klf.size());
    const std::vector<float> kf = convert<float>(T.kap_e), cf = convert<float>(T.c_e);
    m->ke32.upload(kf.data(), E);
    m->ce32.upload(cf.data(), E);
    const std::vector<float> of = convert<float>(ones), ncf = convert<float>(nc);
    m->nk32.upload(of.data(), E);
    m->nc32.upload(ncf.data(), E);
    if (any_c) {
      const std::vector<float> cmf = convert<float>(cm);
      m->nm32.upload(cmf.data(), cmf.size());
    }
  }
  factor_coarse(m);
}

// The solve behind sem_pcg_solve, in the work buffers m->wk (set by the caller).
// b counts on the free nodes only: r = mask(b - A x), ||b|| = ||mask(b)||.
int solve_impl(sem_mesh m, const double* b, double* x, const sem_solve_opts* o, sem_solve_stats* st,
               hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = m->T.n_global;
  const bool refined = o->mode == SEM_SOLVE_FP32_REFINED;
  if (refined && (!m->fp32 || m->wk.v32[0] == nullptr)) throw Error{SEM_EUNSUPPORTED, "no FP32 work buffers"};
  const int gb = grid_stride_blocks(n);
  const int nb = (int)std::min<int64_t>(kRedBlocks, blocks_for(n, kRedThreads));
  const int check = std::max(1, o->check_every);
  if (st) st->history_len = 0;
  double* r64 = m->wk.v64[1];
  double* Ax = m->wk.v64[4];
  // r = mask(b - A x) with ||r||^2 into scalar slot `slot` (Ax = NULL: r = mask(b))
  auto residual = [&](const double* ax, int slot) {
    hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(kRedThreads), 0, s, r64, b, ax, (const uint8_t*)m->dir.p,
                       m->wk.part, n);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kRedThreads), 0, s, m->wk.part, m->wk.sc, nb, slot, 0);
    SEM_HIP(hipGetLastError());
    return read_scalar(m, slot, s);
  };
  const double bnorm2 = residual(nullptr, 7);
  int status = SEM_OK, iters = 0, outer = 0;
  double rel = 0.0;
  if (!std::isfinite(bnorm2)) {
    status = SEM_EBREAKDOWN;
  } else if (bnorm2 == 0.0) {
    hipLaunchKernelGGL((fill_kernel<double>), dim3(gb), dim3(kGS), 0, s, x, 0.0, n);
    SEM_HIP(hipGetLastError());
    SEM_HIP(hipStreamSynchronize(s));
  } else if (!refined) {
    double rr0 = bnorm2;  // x = 0: r = mask(b) already
    if (o->use_x0) {
      apply_A<double>(m, x, Ax, s);
      rr0 = residual(Ax, 8);
    } else {
      hipLaunchKernelGGL((fill_kernel<double>), dim3(gb), dim3(kGS), 0, s, x, 0.0, n);
      SEM_HIP(hipGetLastError());
    }
    status = !std::isfinite(rr0) ? SEM_EBREAKDOWN
                                 : pcg_core<double>(m, x, r64, bnorm2, rr0, o->rtol, o->max_iter, o->pc, check, s,
                                                    &iters, &rel, st);
    // the recursive residual can drift below the true one: confirm with
    // b - A x and restart from the true residual while it is above the tolerance
    const double tol2 = o->rtol * o->rtol * bnorm2;
    while (status == SEM_OK) {
      apply_A<double>(m, x, Ax, s);
      const double rr = residual(Ax, 8);
      rel = std::sqrt(rr / bnorm2);
      if (!std::isfinite(rr)) {
        status = SEM_EBREAKDOWN;
        break;
      }
      if (rr <= tol2) break;
      if (iters >= o->max_iter) {
        status = SEM_ENOCONV;
        break;
      }
      ++outer;
      int it = 0;
      status = pcg_core<double>(m, x, r64, bnorm2, rr, o->rtol, o->max_iter - iters, o->pc, check, s, &it, &rel, st);
      iters += it;
    }
  } else {
    // outer FP64 refinement around FP32 inner PCG solves
    float* d32 = m->wk.v32[0];
    float* r32 = m->wk.v32[1];
    if (!o->use_x0) hipLaunchKernelGGL((fill_kernel<double>), dim3(gb), dim3(kGS), 0, s, x, 0.0, n);
    status = SEM_ENOCONV;
    const double tol2 = o->rtol * o->rtol * bnorm2;
    for (outer = 0; outer <= o->max_outer; ++outer) {
      apply_A<double>(m, x, Ax, s);
      const double rr = residual(Ax, 8);
      rel = std::sqrt(rr / bnorm2);
      if (st && st->history && st->history_len < st->history_cap) st->history[st->history_len++] = rel;
      if (!std::isfinite(rr)) {
        status = SEM_EBREAKDOWN;
        break;
      }
      if (rr <= tol2) {
        status = SEM_OK;
        break;
      }
      if (outer == o->max_outer) break;
      const double rn = std::sqrt(rr);
      hipLaunchKernelGGL(scale_to_f32_kernel, dim3(gb), dim3(kGS), 0, s, r32, r64, 1.0 / rn, n);
      hipLaunchKernelGGL((fill_kernel<float>), dim3(gb), dim3(kGS), 0, s, d32, 0.0f, n);
      SEM_HIP(hipGetLastError());
      // ||r32||^2 of the scaled residual (about 1)
      dot<float, float>(m, r32, r32, 9, 0, s);
      const double r32n2 = read_scalar(m, 9, s);
      int it = 0;
      double irel = 0.0;
      const int st_in = pcg_core<float>(m, d32, r32, r32n2, r32n2, o->inner_rtol, o->max_iter, o->pc, check, s, &it,
                                        &irel, nullptr);
      iters += it;
      if (st_in == SEM_EBREAKDOWN) {
        status = SEM_EBREAKDOWN;
        break;
      }
      hipLaunchKernelGGL(axpy_f32_kernel, dim3(gb), dim3(kGS), 0, s, x, d32, rn, n);
      SEM_HIP(hipGetLastError());
    }
  }
  SEM_HIP(hipStreamSynchronize(s));
  if (st) {
    st->iterations = iters;
    st->outer_iterations = outer;
    st->rel_residual = rel;
    st->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return status;
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return SEM_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return SEM_EINVAL;
  }
}

int need_device(sem_mesh m) {
  if (!m) {
    set_error("NULL handle");
    return SEM_EINVAL;
  }
  if (m->host_only) {
    set_error("host-only handle: no device state");
    return SEM_EUNSUPPORTED;
  }
  return SEM_OK;
}

template void apply_A<double>(sem_mesh, const double*, double*, hipStream_t);
template void apply_A<float>(sem_mesh, const float*, float*, hipStream_t);
template void precond<double>(sem_mesh, const double*, double*, int, hipStream_t);
template void precond<float>(sem_mesh, const float*, float*, int, hipStream_t);

// Autotuner of the operator tile: time each candidate (elements per
// workgroup) on this mesh and keep the fastest; results keyed by
// (architecture, order, dtype, element-count bucket) in an optional text cache.
template <typename T>
int tune_tile(sem_mesh m) {
  const int N = m->T.N;
  std::vector<int> cands;
  for (int c : kTileCandidates)
    if (c * (N + 1) * (N + 1) <= 1024 && c * (N + 1) * (N + 1) >= 16) cands.push_back(c);
  if (N == 15) cands.push_back(kTileMfma);
  cands.push_back(kTileGeo);
  cands.push_back(kTileLineGeo);
  cands.push_back(kTileLineStored);
  if (cands.size() <= 1) return cands.empty() ? 1 : cands[0];
  DBuf<T> u, y;
  u.alloc(m->T.n_global);
  y.alloc(m->T.n_global);
  hipLaunchKernelGGL((fill_kernel<T>), dim3(grid_stride_blocks(m->T.n_global)), dim3(kGS), 0, 0, u.p, T(1),
                     m->T.n_global);
  hipEvent_t a, b;
  SEM_HIP(hipEventCreate(&a));
  SEM_HIP(hipEventCreate(&b));
  const int idx = std::is_same<T, double>::value ? 0 : 1;
  // candidates interleaved over several rounds, best time per candidate kept,
  // so that clock drift does not favour whichever ran first
  constexpr int kRounds = 3;
  std::vector<float> best_ms(cands.size(), 1e30f);
  for (int round = 0; round < kRounds; ++round)
    for (size_t q = 0; q < cands.size(); ++q) {
      m->epb[idx] = cands[q];
      apply_A_elements<T>(m, u.p, y.p, 0);
      SEM_HIP(hipEventRecord(a, 0));
      for (int r = 0; r < 3; ++r) apply_A_elements<T>(m, u.p, y.p, 0);
      SEM_HIP(hipEventRecord(b, 0));
      SEM_HIP(hipEventSynchronize(b));
      float ms = 0.f;
      SEM_HIP(hipEventElapsedTime(&ms, a, b));
      best_ms[q] = std::min(best_ms[q], ms);
    }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  // the default tile unless another is faster by more than the timing noise
  const int def = default_tile(N);
  size_t pick = 0;
  for (size_t q = 0; q < cands.size(); ++q)
    if (cands[q] == def) pick = q;
  for (size_t q = 0; q < cands.size(); ++q)
    if (best_ms[q] < 0.98f * best_ms[pick] && best_ms[q] < best_ms[pick]) pick = q;
  return cands[pick];
}

std::string tune_key(sem_mesh m, int dtype) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, m->device) != hipSuccess) return "";
  int bucket = 0;
  for (int64_t e = m->T.E; e > 1; e >>= 2) ++bucket;  // element count, base-4 buckets
  return std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':')) + " N=" +
         std::to_string(m->T.N) + " dtype=" + std::to_string(dtype) + " ebucket=" + std::to_string(bucket);
}

void autotune(sem_mesh m, const char* cache) {
  for (int d = 0; d < (m->fp32 ? 2 : 1); ++d) {
    const std::string key = tune_key(m, d);
    int found = 0;
    if (cache && !key.empty()) {
      if (FILE* f = std::fopen(cache, "r")) {
        char line[512];
        while (std::fgets(line, sizeof line, f)) {
          std::string l(line);
          const size_t p = l.rfind(" epb=");
          if (p != std::string::npos && l.compare(0, p, key) == 0) found = std::atoi(l.c_str() + p + 5);
        }
        std::fclose(f);
      }
    }
    if (found > 0 && tile_code_ok(found, m->T.N)) {
      m->epb[d] = found;
      continue;
    }
    m->epb[d] = d == 0 ? tune_tile<double>(m) : tune_tile<float>(m);
    if (cache && !key.empty())
      if (FILE* f = std::fopen(cache, "a")) {
        std::fprintf(f, "%s epb=%d\n", key.c_str(), m->epb[d]);
        std::fclose(f);
      }
  }
  SEM_HIP(hipDeviceSynchronize());
}

sem_mesh_s* create_mesh(const double* vtx, int64_t n_vtx, const int64_t* hex, int64_t n_hex, int order,
                        const sem_setup_opts* opts) {
  if (!vtx || !hex || n_vtx <= 0 || n_hex <= 0) throw Error{SEM_EINVAL, "NULL or empty mesh input"};
  if (order < 2 || order > 15) throw Error{SEM_EUNSUPPORTED, "order must be in 2..15"};
  sem_setup_opts d;
  sem_default_setup_opts(&d);
  if (!opts) opts = &d;
  auto m = std::make_unique<sem_mesh_s>();
  m->host_only = opts->host_only != 0;
  m->fp32 = opts->build_fp32 != 0;
  m->device = opts->device;
  HostTables& T = m->T;
  build_reference(T, order);
  build_numbering(T, hex, n_hex, n_vtx);
  build_geometry(T, vtx, hex);
  build_patches(T, hex);
  build_coarse_matrices(T, vtx, hex);
  build_coarse_tree(T);
  m->epb[0] = m->epb[1] = default_tile(order);
  if (!m->host_only) {
    upload_all(m.get());
    resolve_scratch(m->device);  // upload_all left the handle's device current
    if (opts->autotune) autotune(m.get(), opts->tune_cache);
  }
  return m.release();
}

int guarded_call(const std::function<int()>& f) { return guarded(f); }

}  // namespace sem

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

void sem_default_setup_opts(sem_setup_opts* o) {
  if (!o) return;
  o->device = 0;
  o->host_only = 0;
  o->build_fp32 = 1;
  o->autotune = 1;
  o->tune_cache = nullptr;
}

int sem_mesh_set_tile(sem_mesh m, int dtype, int epb) {
  if (!m || (dtype != SEM_F64 && dtype != SEM_F32)) return SEM_EINVAL;
  if (!tile_code_ok(epb, m->T.N)) {
    set_error("tile not available for this order and dtype");
    return SEM_EINVAL;
  }
  m->epb[dtype == SEM_F64 ? 0 : 1] = epb;
  return SEM_OK;
}

int sem_mesh_tile(sem_mesh m, int dtype, int* epb) {
  if (!m || !epb || (dtype != SEM_F64 && dtype != SEM_F32)) return SEM_EINVAL;
  *epb = m->epb[dtype == SEM_F64 ? 0 : 1];
  return SEM_OK;
}

int sem_mesh_coarse_factor_size(sem_mesh m, int64_t* fwd_entries, int64_t* bwd_entries) {
  if (!m || !fwd_entries || !bwd_entries) return SEM_EINVAL;
  *fwd_entries = m->T.fwd_size;
  *bwd_entries = m->T.bwd_size;
  return SEM_OK;
}

void sem_default_solve_opts(sem_solve_opts* o) {
  if (!o) return;
  o->mode = SEM_SOLVE_FP64;
  o->pc = SEM_PC_TWOSCALE;
  o->rtol = 1e-8;
  o->max_iter = 1000;
  o->use_x0 = 0;
  o->inner_rtol = 1e-3;
  o->max_outer = 20;
  o->check_every = 1;
}

const char* sem_last_error(void) { return g_last_error.c_str(); }

int sem_mesh_setup(const double* vtx, int64_t n_vtx, const int64_t* hex, int64_t n_hex, int order,
                   const sem_setup_opts* opts, sem_mesh* out) {
  return guarded([&]() -> int {
    if (!out) throw Error{SEM_EINVAL, "NULL output handle"};
    *out = nullptr;
    *out = create_mesh(vtx, n_vtx, hex, n_hex, order, opts);
    return SEM_OK;
  });
}

int sem_mesh_destroy(sem_mesh m) {
  if (!m) return SEM_OK;
  if (!m->host_only) {
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    release_coarse_graph(m);
    if (m->capture_stream) (void)hipStreamDestroy(m->capture_stream);
    if (m->side_stream) (void)hipStreamDestroy(m->side_stream);
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->ev_join) (void)hipEventDestroy(m->ev_join);
    if (m->ev_check) (void)hipEventDestroy(m->ev_check);
    if (m->check_host) (void)hipHostFree(m->check_host);
  }
  delete m;
  return SEM_OK;
}

int sem_mesh_sizes(sem_mesh m, int64_t* n_global, int64_t* n_local, int64_t* n_vertices) {
  if (!m) return SEM_EINVAL;
  if (n_global) *n_global = m->T.n_global;
  if (n_local) *n_local = m->T.n_local;
  if (n_vertices) *n_vertices = m->T.V;
  return SEM_OK;
}

int sem_mesh_numbering(sem_mesh m, int32_t* l2g) {
  if (!m || !l2g) return SEM_EINVAL;
  return guarded([&]() -> int {
    export_l2g(m->T, l2g);
    return SEM_OK;
  });
}

int sem_mesh_gs_csr(sem_mesh m, int64_t* offsets, int32_t* idx) {
  if (!m || !offsets || !idx) return SEM_EINVAL;
  return guarded([&]() -> int {
    const HostTables& T = m->T;
    std::vector<int32_t> l2g(T.n_local);
    export_l2g(T, l2g.data());
    std::fill(offsets, offsets + T.n_global + 1, 0);
    for (int64_t x = 0; x < T.n_local; ++x) offsets[l2g[x] + 1]++;
    for (int64_t g = 0; g < T.n_global; ++g) offsets[g + 1] += offsets[g];
    std::vector<int64_t> fill(offsets, offsets + T.n_global);
    for (int64_t x = 0; x < T.n_local; ++x) idx[fill[l2g[x]]++] = (int32_t)x;
    return SEM_OK;
  });
}

int sem_mesh_patch_table(sem_mesh m, int32_t* ip) {
  if (!m || !ip) return SEM_EINVAL;
  std::copy(m->T.ip.begin(), m->T.ip.end(), ip);
  return SEM_OK;
}

int sem_mesh_node_coords(sem_mesh m, double* xyz) {
  if (!m || !xyz) return SEM_EINVAL;
  std::copy(m->T.xN.begin(), m->T.xN.end(), xyz);
  return SEM_OK;
}

int sem_mesh_lumped_mass(sem_mesh m, double* mass) {
  if (!m || !mass) return SEM_EINVAL;
  std::copy(m->T.mN.begin(), m->T.mN.end(), mass);
  return SEM_OK;
}

int sem_mesh_boundary_mask(sem_mesh m, uint8_t* mask) {
  if (!m || !mask) return SEM_EINVAL;
  std::copy(m->T.dir.begin(), m->T.dir.end(), mask);
  return SEM_OK;
}

int sem_mesh_geometry(sem_mesh m, double* G, double* mass) {
  if (!m) return SEM_EINVAL;
  if (G) std::copy(m->T.G.begin(), m->T.G.end(), G);
  if (mass) std::copy(m->T.mass.begin(), m->T.mass.end(), mass);
  return SEM_OK;
}

int sem_mesh_set_dirichlet(sem_mesh m, const uint8_t* mask) {
  if (!m || !mask) return SEM_EINVAL;
  return guarded([&]() -> int {
    HostTables& T = m->T;
    for (int64_t g = 0; g < T.n_global; ++g) T.dir[g] = mask[g] ? 1 : 0;
    // the coarse free set follows the vertex nodes: new dissection, new factor
    build_coarse_tree(T);
    update_interior_mask_flags(T);
    if (!m->host_only) {
      SEM_HIP(hipSetDevice(m->device));
      SEM_HIP(hipDeviceSynchronize());
      m->dir.upload(T.dir.data(), T.dir.size());
      m->rec.upload(T.rec.data(), T.rec.size());
      factor_coarse(m);
    }
    return SEM_OK;
  });
}

int sem_apply_A(sem_mesh m, const void* u, void* y, int dtype, void* stream) {
  int st = need_device(m);
  if (st) return st;
  if (!u || !y || u == y) return SEM_EINVAL;
  return guarded([&]() -> int {
    SEM_HIP(hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SEM_F64)
      apply_A<double>(m, (const double*)u, (double*)y, s);
    else if (dtype == SEM_F32) {
      if (!m->fp32) throw Error{SEM_EUNSUPPORTED, "handle built without FP32 copies"};
      apply_A<float>(m, (const float*)u, (float*)y, s);
    } else
      throw Error{SEM_EINVAL, "dtype"};
    return SEM_OK;
  });
}

int sem_time_apply_A(sem_mesh m, const void* u, void* y, int dtype, int reps, void* stream, double* ms_element,
                     double* ms_gather) {
  int st = need_device(m);
  if (st) return st;
  if (!u || !y || u == y || reps < 1) return SEM_EINVAL;
  if (dtype == SEM_F32 && !m->fp32) return SEM_EUNSUPPORTED;
  if (dtype != SEM_F64 && dtype != SEM_F32) return SEM_EINVAL;
  return guarded([&]() -> int {
    SEM_HIP(hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<hipEvent_t> ev(3 * (size_t)reps);
    for (auto& e : ev) SEM_HIP(hipEventCreate(&e));
    struct Cleanup {
      std::vector<hipEvent_t>& v;
      ~Cleanup() {
        for (auto e : v) (void)hipEventDestroy(e);
      }
    } cleanup{ev};
    for (int r = 0; r < reps; ++r) {
      SEM_HIP(hipEventRecord(ev[3 * r], s));
      if (dtype == SEM_F64)
        apply_A_elements<double>(m, (const double*)u, (double*)y, s);
      else
        apply_A_elements<float>(m, (const float*)u, (float*)y, s);
      SEM_HIP(hipEventRecord(ev[3 * r + 1], s));
      if (dtype == SEM_F64)
        launch_gs<double>(m, (double*)y, s, nullptr, nullptr, (const double*)u);
      else
        launch_gs<float>(m, (float*)y, s, nullptr, nullptr, (const float*)u);
      SEM_HIP(hipEventRecord(ev[3 * r + 2], s));
    }
    SEM_HIP(hipStreamSynchronize(s));
    double te = 0.0, tg = 0.0;
    for (int r = 0; r < reps; ++r) {
      float a = 0.f, b = 0.f;
      SEM_HIP(hipEventElapsedTime(&a, ev[3 * r], ev[3 * r + 1]));
      SEM_HIP(hipEventElapsedTime(&b, ev[3 * r + 1], ev[3 * r + 2]));
      te += a;
      tg += b;
    }
    if (ms_element) *ms_element = te / reps;
    if (ms_gather) *ms_gather = tg / reps;
    return SEM_OK;
  });
}

int sem_stream_bench(const double* a, double* b, double* c, int64_t n, int reps, void* stream, double* gbs) {
  if (!a || !b || !c || !gbs || n < 2 || (n & 1) || reps < 1 || a == b || a == c || b == c ||
      !aligned16(a, b, c))
    return SEM_EINVAL;
  return guarded([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    const int64_t n2 = n / 2;
    hipEvent_t e0, e1;
    SEM_HIP(hipEventCreate(&e0));
    SEM_HIP(hipEventCreate(&e1));
    struct Cleanup {
      hipEvent_t a, b;
      ~Cleanup() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } cleanup{e0, e1};
    const double bytes[3] = {16.0 * n, 24.0 * n, 8.0 * n};
    for (int q = 0; q < 3; ++q) gbs[q] = 0.0;
    // best over grid sizes (workgroups of 256 lanes), each timed over reps launches
    for (int grid : {1024, 2048, 4096, 8192, 16384, 32768, 65536}) {
      const int g = (int)std::min<int64_t>(grid, (n2 + 255) / 256);
      for (int q = 0; q < 3; ++q) {
        auto launch = [&]() {
          if (q == 0)
            hipLaunchKernelGGL(stream_copy_kernel, dim3(g), dim3(256), 0, s, (double2*)b, (const double2*)a, n2);
          else if (q == 1)
            hipLaunchKernelGGL(stream_triad_kernel, dim3(g), dim3(256), 0, s, (double2*)c, (const double2*)a,
                               (const double2*)b, 0.5, n2);
          else  // the partial sums land in c (g <= n2 entries)
            hipLaunchKernelGGL(stream_read_kernel, dim3(g), dim3(256), 0, s, (const double2*)a, n2, c);
        };
        launch();
        SEM_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch();
        SEM_HIP(hipEventRecord(e1, s));
        SEM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SEM_HIP(hipEventElapsedTime(&ms, e0, e1));
        gbs[q] = std::max(gbs[q], bytes[q] * reps / (ms * 1e-3) / 1e9);
      }
    }
    return SEM_OK;
  });
}

int sem_precond(sem_mesh m, const void* r, void* z, int dtype, int pc, void* stream) {
  int st = need_device(m);
  if (st) return st;
  if (!r || !z || r == z || pc < 0 || pc > 3) return SEM_EINVAL;
  return guarded([&]() -> int {
    SEM_HIP(hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    if (dtype == SEM_F64)
      precond<double>(m, (const double*)r, (double*)z, pc, s);
    else if (dtype == SEM_F32) {
      if (!m->fp32) throw Error{SEM_EUNSUPPORTED, "handle built without FP32 copies"};
      precond<float>(m, (const float*)r, (float*)z, pc, s);
    } else
      throw Error{SEM_EINVAL, "dtype"};
    return SEM_OK;
  });
}

int sem_coarse_solve(sem_mesh m, const double* R, double* Z, void* stream) {
  int st = need_device(m);
  if (st) return st;
  if (!R || !Z) return SEM_EINVAL;
  return guarded([&]() -> int {
    SEM_HIP(hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    const HostTables& T = m->T;
    if (T.nc > 0) {
      hipLaunchKernelGGL(coarse_gather_vertex_kernel, dim3((unsigned)blocks_for(T.V)), dim3(kGS), 0, s, m->Rlev.p, R,
                         m->cidx.p, T.V);
      SEM_HIP(hipGetLastError());
      coarse_solve_tree(m, s);
    } else {
      hipLaunchKernelGGL((fill_kernel<double>), dim3(grid_stride_blocks(T.V)), dim3(kGS), 0, s, m->Zv.p, 0.0, T.V);
    }
    SEM_HIP(hipMemcpyAsync(Z, m->Zv.p, T.V * sizeof(double), hipMemcpyDeviceToDevice, s));
    return SEM_OK;
  });
}

int sem_pcg_solve(sem_mesh m, const double* b, double* x, const sem_solve_opts* o, sem_solve_stats* st,
                  void* stream) {
  int s0 = need_device(m);
  if (s0) return s0;
  if (!b || !x || b == x) return SEM_EINVAL;
  sem_solve_opts d;
  sem_default_solve_opts(&d);
  if (!o) o = &d;
  if (o->pc < 0 || o->pc > 3 || o->max_iter < 0 || !(o->rtol >= 0.0)) return SEM_EINVAL;
  return guarded([&]() -> int {
    SEM_HIP(hipSetDevice(m->device));
    if (o->mode == SEM_SOLVE_FP32_REFINED && !m->fp32) throw Error{SEM_EUNSUPPORTED, "handle built without FP32 copies"};
    ensure_work(m, o->mode == SEM_SOLVE_FP32_REFINED);
    return solve_impl(m, b, x, o, st, (hipStream_t)stream);
  });
}

int sem_pcg_solve_noalloc(sem_mesh m, const double* b, double* x, const sem_solve_opts* o, sem_solve_stats* st,
                          void* stream) {
  if (!m) {
    set_error("NULL handle");
    return SEM_EINVAL;
  }
  if (!b || !x || b == x) return SEM_EINVAL;
  sem_solve_opts d;
  sem_default_solve_opts(&d);
  if (!o) o = &d;
  if (o->pc < 0 || o->pc > 3 || o->max_iter < 0 || !(o->rtol >= 0.0)) return SEM_EINVAL;
  const bool need32 = o->mode == SEM_SOLVE_FP32_REFINED;
  const size_t need = scratch_layout(m, need32).total;
  if (need > kScratchBytes) {
    set_error("sem_pcg_solve_noalloc: this mesh needs " + std::to_string(need) + " bytes of static scratch, more than " +
              "its maximum of " + std::to_string(kScratchBytes) + " bytes; use sem_pcg_solve");
    return SEM_EINVAL;
  }
  int s0 = need_device(m);
  if (s0) return s0;
  return guarded([&]() -> int {
    SEM_HIP(hipSetDevice(m->device));
    if (need32 && !m->fp32) throw Error{SEM_EUNSUPPORTED, "handle built without FP32 copies"};
    double* base = scratch_of(m->device);
    if (base == nullptr) throw Error{SEM_EHIP, "static scratch not resolved on this device"};
    // views into the scratch for this solve only; any lazy set-up that would
    // allocate raises instead (no_alloc); the handle's own buffers return with
    // the next sem_pcg_solve
    struct Restore {
      sem_mesh m;
      ~Restore() {
        m->no_alloc = false;
        m->wk = sem_mesh_s::SolveWork{};
      }
    } restore{m};
    m->no_alloc = true;
    scratch_work(m, need32, base);
    return solve_impl(m, b, x, o, st, (hipStream_t)stream);
  });
}

int sem_mesh_set_coefficients(sem_mesh m, double kappa, double c) {
  if (!m || !(kappa > 0.0) || !(c >= 0.0) || !std::isfinite(kappa) || !std::isfinite(c)) return SEM_EINVAL;
  return guarded([&]() -> int {
    set_coefficients(m, kappa, c);
    return SEM_OK;
  });
}

int sem_mesh_set_element_coefficients(sem_mesh m, const double* kappa, const double* c) {
  if (!m) return SEM_EINVAL;
  const int64_t E = m->T.E;
  for (int64_t e = 0; e < E; ++e) {
    if (kappa && !(kappa[e] > 0.0 && std::isfinite(kappa[e]))) return SEM_EINVAL;
    if (c && !(c[e] >= 0.0 && std::isfinite(c[e]))) return SEM_EINVAL;
  }
  return guarded([&]() -> int {
    set_element_coefficients(m, kappa, c);
    return SEM_OK;
  });
}

int sem_mesh_set_node_coefficients(sem_mesh m, const double* kappa, const double* c) {
  if (!m) return SEM_EINVAL;
  const int64_t nl = m->T.n_local;
  for (int64_t l = 0; l < nl; ++l) {
    if (kappa && !(kappa[l] > 0.0 && std::isfinite(kappa[l]))) return SEM_EINVAL;
    if (c && !(c[l] >= 0.0 && std::isfinite(c[l]))) return SEM_EINVAL;
  }
  return guarded([&]() -> int {
    set_node_coefficients(m, kappa, c);
    return SEM_OK;
  });
}

int sem_mesh_boundary_face_mass(sem_mesh m, const int64_t* faces, int64_t n_faces, double* ws) {
  if (!m || !ws || n_faces < 0 || (n_faces > 0 && !faces)) return SEM_EINVAL;
  return guarded([&]() -> int {
    boundary_face_mass(m->T, faces, n_faces, ws);
    return SEM_OK;
  });
}

int sem_mesh_set_coarse_solver(sem_mesh m, int solver) {
  if (!m || (solver != SEM_COARSE_EXACT && solver != SEM_COARSE_AMG)) return SEM_EINVAL;
  return guarded([&]() -> int {
    if (m->coarse_solver == solver) return SEM_OK;
    m->coarse_solver = solver;
    if (m->host_only) return SEM_OK;
    SEM_HIP(hipSetDevice(m->device));
    SEM_HIP(hipDeviceSynchronize());
    release_coarse_graph(m);
    if (solver == SEM_COARSE_AMG) {
      try {
        amg_setup(m);
      } catch (...) {
        m->coarse_solver = SEM_COARSE_EXACT;
        m->amg.clear();
        build_coarse_graph(m);
        throw;
      }
    } else {
      m->amg.clear();
    }
    build_coarse_graph(m);
    return SEM_OK;
  });
}

int sem_mesh_amg_hierarchy(sem_mesh m, int64_t* level_sizes, int cap, int* n_levels, int32_t* agg0) {
  if (!m || !n_levels || cap < 0 || (cap > 0 && !level_sizes)) return SEM_EINVAL;
  return guarded([&]() -> int {
    AmgHierarchy H;
    build_amg(m->T, H);
    *n_levels = (int)H.levels.size();
    for (int l = 0; l < cap && l < (int)H.levels.size(); ++l) level_sizes[l] = H.levels[l].n;
    if (agg0 && !H.levels.empty() && !H.levels[0].agg.empty())
      std::copy(H.levels[0].agg.begin(), H.levels[0].agg.end(), agg0);
    return SEM_OK;
  });
}

int sem_mesh_coefficients(sem_mesh m, double* kappa, double* c) {
  if (!m || !kappa || !c) return SEM_EINVAL;
  *kappa = m->T.kappa;
  *c = m->T.cmass;
  return SEM_OK;
}

int sem_heat_step(sem_mesh m, double kappa, double dt, const double* u_prev, const double* q, double* u_next,
                  const sem_solve_opts* o, sem_solve_stats* st, void* stream) {
  int s0 = need_device(m);
  if (s0) return s0;
  if (!u_prev || !u_next || !(dt > 0.0) || !(kappa > 0.0) || !std::isfinite(dt) || !std::isfinite(kappa))
    return SEM_EINVAL;
  if (q == u_next) return SEM_EINVAL;
  sem_solve_opts d;
  sem_default_solve_opts(&d);
  if (!o) o = &d;
  if (o->pc < 0 || o->pc > 3 || o->max_iter < 0 || !(o->rtol >= 0.0)) return SEM_EINVAL;
  return guarded([&]() -> int {
    SEM_HIP(hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    set_coefficients(m, kappa, 1.0 / dt);
    const int64_t n = m->T.n_global;
    if (m->hb.n < (size_t)n) m->hb.alloc(n);
    hipLaunchKernelGGL(heat_rhs_kernel, dim3((unsigned)blocks_for(n)), dim3(kGS), 0, s, m->hb.p, u_prev, q,
                       m->mN64.p, m->dir.p, dt, n);
    SEM_HIP(hipGetLastError());
    if (u_next != u_prev) SEM_HIP(hipMemcpyAsync(u_next, u_prev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    sem_solve_opts oo = *o;
    oo.use_x0 = 1;
    if (oo.mode == SEM_SOLVE_FP32_REFINED && !m->fp32) throw Error{SEM_EUNSUPPORTED, "handle built without FP32 copies"};
    ensure_work(m, oo.mode == SEM_SOLVE_FP32_REFINED);
    return solve_impl(m, m->hb.p, u_next, &oo, st, s);
  });
}

}  // extern "C"
