// Batched independent solves (many meshes, orders 2..15, one stream).
//
// Instances of the same order N are concatenated into one disjoint-union mesh:
// every operator, gather, patch and coarse kernel then covers all of them in
// one launch (work items = elements of all instances, in the union's Morton
// order; each component is its own tree of the coarse nested dissection, and
// nodes of all trees at one height share the coarse sweep launches).  The
// union's canonical numbering restricted to one instance is that instance's
// own numbering shifted by four offsets (vertices, edges, faces, interiors), so
// instance vectors map to union vectors by four contiguous copies.
//
// PCG (Algorithm 1) runs per instance: dot products are reduced per instance
// over fixed chunks in a fixed order (deterministic), alpha and beta are
// per-instance device scalars, and an instance stops updating the moment its
// own residual test passes, exactly where a single solve would stop.  One whole
// batched iteration (all orders) is captured once in a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

#include "sem_device.h"

namespace sem {

// per-instance scalar slots
enum : int {
  kRz = 0, kPw, kAlpha, kBeta, kRr, kBb, kActive, kIters, kTol2, kFlag, kNorm, kRestarts, kScal  // kScal = stride
};
constexpr int64_t kChunk = 16384;  // nodes per reduction chunk

struct Chunk {
  int64_t begin, end;  // union index range
  int32_t inst;        // global instance index
  int32_t pad;
};

// --- kernels ------------------------------------------------------------------
__device__ __forceinline__ double block_reduce(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += sh[q];
  return s;
}

// part[cid] = sum over chunk cid of a*b
template <typename TA, typename TB>
__global__ void __launch_bounds__(256)
seg_dot_kernel(const TA* __restrict__ a, const TB* __restrict__ b, const int32_t* __restrict__ ids,
               const Chunk* __restrict__ chunks, double* __restrict__ part) {
  __shared__ double sh[4];
  const int32_t cid = ids[blockIdx.x];
  const Chunk c = chunks[cid];
  double s = 0.0;
  for (int64_t q = c.begin + threadIdx.x; q < c.end; q += blockDim.x) s += (double)a[q] * (double)b[q];
  s = block_reduce(s, sh);
  if (threadIdx.x == 0) part[cid] = s;
}

// per instance: s = sum of its chunks in order; then
//   mode 0: sc[dst] = s
//   mode 1: p^T w -> alpha (0 for stopped instances), breakdown flag
//   mode 2: z^T r -> beta, rz
//   mode 3: r^T r -> rr; an active instance that meets its tolerance stops;
//           active ones count the iteration; sc_all[0] = number still active
__global__ void __launch_bounds__(64)
seg_final_kernel(const double* __restrict__ part, const int32_t* __restrict__ inst_chunk_off,
                 double* __restrict__ sc, int n, int dst, int mode, double* __restrict__ nactive) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double s = 0.0;
    for (int32_t c = inst_chunk_off[i]; c < inst_chunk_off[i + 1]; ++c) s += part[c];
    double* S = sc + (int64_t)i * kScal;
    const bool act = S[kActive] != 0.0;
    if (mode == 0) {
      S[dst] = s;
    } else if (mode == 1) {
      S[kPw] = s;
      double a = 0.0;
      if (act) {
        a = S[kRz] / s;
        if (!(s > 0.0) || !isfinite(a)) {
          S[kFlag] = 1.0;
          S[kActive] = 0.0;
          a = 0.0;
        }
      }
      S[kAlpha] = a;
    } else if (mode == 2) {
      if (act) {
        const double b = s / S[kRz];
        if (!isfinite(b)) {
          S[kFlag] = 1.0;
          S[kActive] = 0.0;
        }
        S[kBeta] = b;
        S[kRz] = s;
      }
    } else if (mode == 3) {
      if (act) {
        S[kRr] = s;
        S[kIters] += 1.0;
        if (!isfinite(s)) {
          S[kFlag] = 1.0;
          S[kActive] = 0.0;
        } else if (s <= S[kTol2]) {
          S[kActive] = 0.0;
        }
      }
      if (S[kActive] != 0.0) atomicAdd(&cnt, 1);
    }
  }
  __syncthreads();
  if (mode == 3 && threadIdx.x == 0) nactive[0] = (double)cnt;
}

// x += alpha p; r -= alpha w (active instances); partial sums of r^T r
template <typename T, typename TX>
__global__ void __launch_bounds__(256)
seg_update_xr_kernel(TX* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ w,
                     const int32_t* __restrict__ ids, const Chunk* __restrict__ chunks,
                     const double* __restrict__ sc, double* __restrict__ part) {
  __shared__ double sh[4];
  const int32_t cid = ids[blockIdx.x];
  const Chunk c = chunks[cid];
  const double* S = sc + (int64_t)c.inst * kScal;
  const bool act = S[kActive] != 0.0;
  const T al = (T)S[kAlpha];
  double s = 0.0;
  for (int64_t q = c.begin + threadIdx.x; q < c.end; q += blockDim.x) {
    T rn = r[q];
    if (act) {
      x[q] += (TX)(al * p[q]);
      rn = rn - al * w[q];
      r[q] = rn;
    }
    s += (double)rn * (double)rn;
  }
  s = block_reduce(s, sh);
  if (threadIdx.x == 0) part[cid] = s;
}

// p = z + beta p (active instances)
template <typename T>
__global__ void __launch_bounds__(256)
seg_update_p_kernel(T* __restrict__ p, const T* __restrict__ z, const int32_t* __restrict__ ids,
                    const Chunk* __restrict__ chunks, const double* __restrict__ sc) {
  const int32_t cid = ids[blockIdx.x];
  const Chunk c = chunks[cid];
  const double* S = sc + (int64_t)c.inst * kScal;
  if (S[kActive] == 0.0) return;
  const T b = (T)S[kBeta];
  for (int64_t q = c.begin + threadIdx.x; q < c.end; q += blockDim.x) p[q] = z[q] + b * p[q];
}

// dst = (TD)(src * scale_inst) on each chunk, scale = 1 / sc[kNorm] (or 1)
template <typename TD, typename TS>
__global__ void __launch_bounds__(256)
seg_scale_kernel(TD* __restrict__ dst, const TS* __restrict__ src, const int32_t* __restrict__ ids,
                 const Chunk* __restrict__ chunks, const double* __restrict__ sc, int by_norm) {
  const int32_t cid = ids[blockIdx.x];
  const Chunk c = chunks[cid];
  const double* S = sc + (int64_t)c.inst * kScal;
  const double nrm = S[kNorm];
  // instances that have stopped get a zero right-hand side (their inner solve is idle)
  const double f = by_norm ? ((nrm > 0.0 && S[kActive] != 0.0) ? 1.0 / nrm : 0.0) : 1.0;
  for (int64_t q = c.begin + threadIdx.x; q < c.end; q += blockDim.x) dst[q] = (TD)((double)src[q] * f);
}

// x64 += ||r||_inst * d32 for instances still refining
__global__ void __launch_bounds__(256)
seg_correct_kernel(double* __restrict__ x, const float* __restrict__ d, const int32_t* __restrict__ ids,
                   const Chunk* __restrict__ chunks, const double* __restrict__ sc_outer) {
  const int32_t cid = ids[blockIdx.x];
  const Chunk c = chunks[cid];
  const double* S = sc_outer + (int64_t)c.inst * kScal;
  if (S[kActive] == 0.0) return;
  const double f = S[kNorm];
  for (int64_t q = c.begin + threadIdx.x; q < c.end; q += blockDim.x) x[q] += f * (double)d[q];
}

// r = b - Ax with partial sums of r^T r
__global__ void __launch_bounds__(256)
seg_residual_kernel(double* __restrict__ r, const double* __restrict__ b, const double* __restrict__ Ax,
                    const int32_t* __restrict__ ids, const Chunk* __restrict__ chunks, double* __restrict__ part) {
  __shared__ double sh[4];
  const int32_t cid = ids[blockIdx.x];
  const Chunk c = chunks[cid];
  double s = 0.0;
  for (int64_t q = c.begin + threadIdx.x; q < c.end; q += blockDim.x) {
    const double v = b[q] - Ax[q];
    r[q] = v;
    s += v * v;
  }
  s = block_reduce(s, sh);
  if (threadIdx.x == 0) part[cid] = s;
}

// After a batched FP64 solve, part holds each instance's true ||b - A x||^2 (by
// chunks): instances whose true residual is still above the tolerance become
// active again (PCG restarts from it), the others stay stopped; counts restarts.
__global__ void __launch_bounds__(64)
seg_restart_kernel(const double* __restrict__ part, const int32_t* __restrict__ inst_chunk_off,
                   double* __restrict__ sc, int n, double* __restrict__ nactive) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double s = 0.0;
    for (int32_t c = inst_chunk_off[i]; c < inst_chunk_off[i + 1]; ++c) s += part[c];
    double* S = sc + (int64_t)i * kScal;
    S[kRr] = s;
    if (!isfinite(s)) S[kFlag] = 1.0;
    const bool act = S[kFlag] == 0.0 && S[kBb] > 0.0 && s > S[kTol2];
    S[kActive] = act ? 1.0 : 0.0;
    if (act) {
      S[kRestarts] += 1.0;
      atomicAdd(&cnt, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) nactive[0] = (double)cnt;
}

// b = 0 on the Dirichlet set (its values there do not take part in the solve)
__global__ void __launch_bounds__(256)
mask_vec_kernel(double* __restrict__ v, const uint8_t* __restrict__ dir, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    if (dir[q]) v[q] = 0.0;
}

// per-instance scalar initialisation of a PCG run: rz, active, tol2, counters
__global__ void seg_init_kernel(double* __restrict__ sc, const double* __restrict__ bb_src, int bb_slot, int n,
                                double rtol2) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double* S = sc + (int64_t)i * kScal;
    const double bb = bb_src[(int64_t)i * kScal + bb_slot];
    S[kBb] = bb;
    S[kTol2] = rtol2 * bb;
    S[kRr] = bb;
    S[kIters] = 0.0;
    S[kRestarts] = 0.0;
    S[kFlag] = 0.0;
    S[kActive] = (bb > 0.0 && isfinite(bb) && bb > S[kTol2]) ? 1.0 : 0.0;
  }
}

__global__ void seg_norm_kernel(double* __restrict__ sc, int n, int src_slot) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double* S = sc + (int64_t)i * kScal;
    S[kNorm] = sqrt(S[src_slot]);
  }
}

template <typename T>
__global__ void fill_vec_kernel(T* __restrict__ d, T v, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    d[q] = v;
}

template <typename T>
__global__ void copy_vec_kernel(T* __restrict__ d, const T* __restrict__ s, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    d[q] = s[q];
}

// --- host side ------------------------------------------------------------------
template <typename T>
struct Vecs {
  DBuf<T> v[6];
};

struct MeshDeleter {
  void operator()(sem_mesh_s* m) const { sem_mesh_destroy(m); }
};

struct Group {
  int N = 0;
  std::unique_ptr<sem_mesh_s, MeshDeleter> mesh;
  std::vector<int> inst;            // global instance indices, in concatenation order
  std::vector<int32_t> chunk_ids;   // global chunk ids of this group
  DBuf<int32_t> d_chunk_ids;
  Vecs<double> f64;                 // x, r, z, p, w, b   (union-sized)
  Vecs<float> f32;                  // d, r, z, p, w
};

struct Run {  // one instance's run of union entries
  int inst, group;
  int64_t src, dst, len;
};

}  // namespace sem

using namespace sem;

struct sem_batch_s {
  int n = 0;
  std::vector<int64_t> ng;        // per instance
  std::vector<Group> groups;
  std::vector<Run> runs;
  std::vector<Chunk> chunks;      // ordered by instance
  std::vector<int32_t> inst_chunk_off;
  DBuf<Chunk> d_chunks;
  DBuf<int32_t> d_inst_chunk_off;
  DBuf<double> part, sc, sc_outer, nactive;
  hipStream_t cap = nullptr;
  hipGraphExec_t it64 = nullptr, it32 = nullptr;
  int graph_pc = -1;
  ~sem_batch_s() {
    if (it64) (void)hipGraphExecDestroy(it64);
    if (it32) (void)hipGraphExecDestroy(it32);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(65536, blocks_of(n)); }

template <typename TA, typename TB>
void seg_dot(sem_batch b, Group& g, const TA* x, const TB* y, hipStream_t s) {
  if (g.chunk_ids.empty()) return;
  hipLaunchKernelGGL((seg_dot_kernel<TA, TB>), dim3((unsigned)g.chunk_ids.size()), dim3(256), 0, s, x, y,
                     g.d_chunk_ids.p, b->d_chunks.p, b->part.p);
}

void seg_final(sem_batch b, double* sc, int dst, int mode, hipStream_t s) {
  hipLaunchKernelGGL(seg_final_kernel, dim3(1), dim3(64), 0, s, b->part.p, b->d_inst_chunk_off.p, sc, b->n, dst,
                     mode, b->nactive.p);
}

// one batched PCG iteration on vectors of type T (x, r, z, p, w = v[0..4])
template <typename T>
void batched_iteration(sem_batch b, int pc, hipStream_t s) {
  for (auto& g : b->groups) {
    auto& V = [&]() -> Vecs<T>& {
      if constexpr (std::is_same<T, double>::value) return g.f64; else return g.f32;
    }();
    apply_A<T>(g.mesh.get(), V.v[3].p, V.v[4].p, s);
    seg_dot<T, T>(b, g, V.v[3].p, V.v[4].p, s);
  }
  seg_final(b, b->sc.p, 0, 1, s);
  for (auto& g : b->groups) {
    auto& V = [&]() -> Vecs<T>& {
      if constexpr (std::is_same<T, double>::value) return g.f64; else return g.f32;
    }();
    if (g.chunk_ids.empty()) continue;
    hipLaunchKernelGGL((seg_update_xr_kernel<T, T>), dim3((unsigned)g.chunk_ids.size()), dim3(256), 0, s, V.v[0].p,
                       V.v[1].p, V.v[3].p, V.v[4].p, g.d_chunk_ids.p, b->d_chunks.p, b->sc.p, b->part.p);
  }
  seg_final(b, b->sc.p, 0, 3, s);
  for (auto& g : b->groups) {
    auto& V = [&]() -> Vecs<T>& {
      if constexpr (std::is_same<T, double>::value) return g.f64; else return g.f32;
    }();
    precond<T>(g.mesh.get(), V.v[1].p, V.v[2].p, pc, s);
    seg_dot<T, T>(b, g, V.v[1].p, V.v[2].p, s);
  }
  seg_final(b, b->sc.p, 0, 2, s);
  for (auto& g : b->groups) {
    auto& V = [&]() -> Vecs<T>& {
      if constexpr (std::is_same<T, double>::value) return g.f64; else return g.f32;
    }();
    if (g.chunk_ids.empty()) continue;
    hipLaunchKernelGGL((seg_update_p_kernel<T>), dim3((unsigned)g.chunk_ids.size()), dim3(256), 0, s, V.v[3].p,
                       V.v[2].p, g.d_chunk_ids.p, b->d_chunks.p, b->sc.p);
  }
  SEM_HIP(hipGetLastError());
}

template <typename T>
hipGraphExec_t capture_iteration(sem_batch b, int pc) {
  if (!b->cap) SEM_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  for (auto& g : b->groups) g.mesh->direct_coarse = true;
  hipGraph_t graph = nullptr;
  SEM_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  try {
    batched_iteration<T>(b, pc, b->cap);
  } catch (...) {
    (void)hipStreamEndCapture(b->cap, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto& g : b->groups) g.mesh->direct_coarse = false;
    throw;
  }
  SEM_HIP(hipStreamEndCapture(b->cap, &graph));
  for (auto& g : b->groups) g.mesh->direct_coarse = false;
  hipGraphExec_t exec = nullptr;
  hipError_t err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (err != hipSuccess) throw Error{SEM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(err)};
  return exec;
}

double read_active(sem_batch b, hipStream_t s) {
  double v = 0.0;
  SEM_HIP(hipMemcpyAsync(&v, b->nactive.p, sizeof(double), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  return v;
}

// PCG on all instances: x, r given (r = rhs), returns the batched iterations
// performed.  restart: the scalars (tolerances, active flags, counters) come
// from seg_restart_kernel instead of a fresh start from ||r||.
template <typename T>
int batched_pcg(sem_batch b, double rtol, int max_iter, int pc, int check_every, hipStream_t s,
                bool restart = false) {
  if (!restart) {
    // per-instance ||r||^2 -> scalars, tolerance, active flags
    for (auto& g : b->groups) {
      auto& V = [&]() -> Vecs<T>& {
        if constexpr (std::is_same<T, double>::value) return g.f64; else return g.f32;
      }();
      seg_dot<T, T>(b, g, V.v[1].p, V.v[1].p, s);
    }
    seg_final(b, b->sc.p, kRr, 0, s);
    hipLaunchKernelGGL(seg_init_kernel, dim3(1), dim3(64), 0, s, b->sc.p, (const double*)b->sc.p, (int)kRr, b->n,
                       rtol * rtol);
  }
  for (auto& g : b->groups) {
    auto& V = [&]() -> Vecs<T>& {
      if constexpr (std::is_same<T, double>::value) return g.f64; else return g.f32;
    }();
    precond<T>(g.mesh.get(), V.v[1].p, V.v[2].p, pc, s);
    hipLaunchKernelGGL((copy_vec_kernel<T>), dim3(grid_for(g.mesh->T.n_global)), dim3(256), 0, s, V.v[3].p,
                       (const T*)V.v[2].p, g.mesh->T.n_global);
    seg_dot<T, T>(b, g, V.v[1].p, V.v[2].p, s);
  }
  seg_final(b, b->sc.p, kRz, 0, s);
  SEM_HIP(hipGetLastError());
  hipGraphExec_t& exec = std::is_same<T, double>::value ? b->it64 : b->it32;
  if (!exec || b->graph_pc != pc) {
    if (b->it64) (void)hipGraphExecDestroy(b->it64);
    if (b->it32) (void)hipGraphExecDestroy(b->it32);
    b->it64 = b->it32 = nullptr;
    b->graph_pc = pc;
    exec = capture_iteration<T>(b, pc);
  }
  int k = 0;
  while (k < max_iter) {
    SEM_HIP(hipGraphLaunch(exec, s));
    ++k;
    if (k % check_every == 0 || k == max_iter) {
      if (read_active(b, s) == 0.0) break;
    }
  }
  return k;
}

void copy_in(sem_batch b, const double* const* src, int slot, hipStream_t s) {
  for (auto& r : b->runs)
    SEM_HIP(hipMemcpyAsync(b->groups[r.group].f64.v[slot].p + r.dst, src[r.inst] + r.src, r.len * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
}

void copy_out(sem_batch b, double* const* dst, int slot, hipStream_t s) {
  for (auto& r : b->runs)
    SEM_HIP(hipMemcpyAsync(dst[r.inst] + r.src, b->groups[r.group].f64.v[slot].p + r.dst, r.len * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
}

}  // namespace

extern "C" {

int sem_batch_setup(int n, const double* const* vtx, const int64_t* n_vtx, const int64_t* const* hex,
                    const int64_t* n_hex, const int* order, const sem_setup_opts* opts, sem_batch* out) {
  return guarded_call([&]() -> int {
    if (!out || n <= 0 || !vtx || !n_vtx || !hex || !n_hex || !order) throw Error{SEM_EINVAL, "batch arguments"};
    *out = nullptr;
    sem_setup_opts d;
    sem_default_setup_opts(&d);
    if (!opts) opts = &d;
    if (opts->host_only) throw Error{SEM_EUNSUPPORTED, "a batch needs a device"};
    auto B = std::make_unique<sem_batch_s>();
    B->n = n;
    B->ng.assign(n, 0);
    std::vector<int> orders;
    for (int i = 0; i < n; ++i) {
      if (order[i] < 2 || order[i] > 15) throw Error{SEM_EUNSUPPORTED, "order must be in 2..15"};
      if (!vtx[i] || !hex[i] || n_vtx[i] <= 0 || n_hex[i] <= 0) throw Error{SEM_EINVAL, "empty instance"};
      orders.push_back(order[i]);
    }
    std::sort(orders.begin(), orders.end());
    orders.erase(std::unique(orders.begin(), orders.end()), orders.end());
    for (int N : orders) {
      Group g;
      g.N = N;
      std::vector<double> V;
      std::vector<int64_t> H;
      for (int i = 0; i < n; ++i) {
        if (order[i] != N) continue;
        const int64_t voff = (int64_t)V.size() / 3;
        V.insert(V.end(), vtx[i], vtx[i] + 3 * n_vtx[i]);
        for (int64_t x = 0; x < 8 * n_hex[i]; ++x) {
          if (hex[i][x] < 0 || hex[i][x] >= n_vtx[i]) throw Error{SEM_EINVAL, "hexahedron vertex id out of range"};
          H.push_back(hex[i][x] + voff);
        }
        g.inst.push_back(i);
      }
      g.mesh.reset(create_mesh(V.data(), (int64_t)V.size() / 3, H.data(), (int64_t)H.size() / 8, N, opts));
      B->groups.push_back(std::move(g));
    }
    // instance <-> union maps: vertices, edges, faces, interiors
    for (size_t gi = 0; gi < B->groups.size(); ++gi) {
      Group& g = B->groups[gi];
      const HostTables& U = g.mesh->T;
      const int64_t m = g.N - 1;
      int64_t vo = 0, eo = 0, fo = 0, io = 0;
      for (int i : g.inst) {
        // the instance's own class sizes, from its referenced vertices and topology
        std::vector<char> used(n_vtx[i], 0);
        for (int64_t x = 0; x < 8 * n_hex[i]; ++x) used[hex[i][x]] = 1;
        int64_t Vi = 0;
        for (char c : used) Vi += c;
        // edges and faces of the instance = union entities of its elements
        std::vector<int64_t> eds, fcs;
        int64_t ebase = 0, fbase = 0;
        for (int j : g.inst) {
          if (j == i) break;
          ebase += n_hex[j];
        }
        (void)fbase;
        std::vector<char> eu, fu;
        int64_t nE = 0, nF = 0;
        {
          // count distinct edge / face ranks of this instance's elements in the union
          std::vector<int64_t> er, fr;
          for (int64_t e = ebase; e < ebase + n_hex[i]; ++e) {
            for (int cz = 0; cz < 3; ++cz)
              for (int cy = 0; cy < 3; ++cy)
                for (int cx = 0; cx < 3; ++cx) {
                  const int nb = (cx != 1) + (cy != 1) + (cz != 1);
                  if (nb != 2 && nb != 1) continue;
                  const int64_t gid = gid_of(U, e, cx == 2 ? g.N : (cx == 1 ? 1 : 0), cy == 2 ? g.N : (cy == 1 ? 1 : 0),
                                             cz == 2 ? g.N : (cz == 1 ? 1 : 0));
                  if (nb == 2)
                    er.push_back((gid - U.base_e) / m);
                  else
                    fr.push_back((gid - U.base_f) / (m * m));
                }
          }
          std::sort(er.begin(), er.end());
          er.erase(std::unique(er.begin(), er.end()), er.end());
          std::sort(fr.begin(), fr.end());
          fr.erase(std::unique(fr.begin(), fr.end()), fr.end());
          nE = (int64_t)er.size();
          nF = (int64_t)fr.size();
          if (nE && (er.front() != eo || er.back() != eo + nE - 1)) throw Error{SEM_EMESH, "batch edge map"};
          if (nF && (fr.front() != fo || fr.back() != fo + nF - 1)) throw Error{SEM_EMESH, "batch face map"};
        }
        const int64_t Ei = n_hex[i];
        const int64_t ng = Vi + nE * m + nF * m * m + Ei * m * m * m;
        B->ng[i] = ng;
        B->runs.push_back(Run{i, (int)gi, 0, vo, Vi});
        B->runs.push_back(Run{i, (int)gi, Vi, U.base_e + eo * m, nE * m});
        B->runs.push_back(Run{i, (int)gi, Vi + nE * m, U.base_f + fo * m * m, nF * m * m});
        B->runs.push_back(Run{i, (int)gi, Vi + nE * m + nF * m * m, U.base_i + io * m * m * m, Ei * m * m * m});
        vo += Vi;
        eo += nE;
        fo += nF;
        io += Ei;
      }
      if (vo != U.V || eo != U.n_edges || fo != U.n_faces || io != U.E) throw Error{SEM_EMESH, "batch maps"};
    }
    // reduction chunks, ordered by instance
    B->inst_chunk_off.assign(n + 1, 0);
    std::vector<std::vector<Chunk>> per(n);
    for (auto& r : B->runs)
      for (int64_t q = 0; q < r.len; q += kChunk)
        per[r.inst].push_back(Chunk{r.dst + q, r.dst + std::min(r.len, q + kChunk), r.inst, r.group});
    for (int i = 0; i < n; ++i) {
      for (auto& c : per[i]) B->chunks.push_back(c);
      B->inst_chunk_off[i + 1] = (int32_t)B->chunks.size();
    }
    for (size_t c = 0; c < B->chunks.size(); ++c) B->groups[B->chunks[c].pad].chunk_ids.push_back((int32_t)c);
    SEM_HIP(hipSetDevice(opts->device));
    B->d_chunks.upload(B->chunks.data(), B->chunks.size());
    B->d_inst_chunk_off.upload(B->inst_chunk_off.data(), B->inst_chunk_off.size());
    for (auto& g : B->groups) {
      g.d_chunk_ids.upload(g.chunk_ids.data(), g.chunk_ids.size());
      const int64_t ngu = g.mesh->T.n_global;
      for (auto& v : g.f64.v) v.alloc(ngu);
      if (opts->build_fp32)
        for (int q = 0; q < 5; ++q) g.f32.v[q].alloc(ngu);
    }
    B->part.alloc(std::max<size_t>(1, B->chunks.size()));
    B->sc.alloc((size_t)n * kScal);
    B->sc_outer.alloc((size_t)n * kScal);
    B->nactive.alloc(1);
    *out = B.release();
    return SEM_OK;
  });
}

int sem_batch_destroy(sem_batch b) {
  if (!b) return SEM_OK;
  (void)hipDeviceSynchronize();
  delete b;
  return SEM_OK;
}

int sem_batch_sizes(sem_batch b, int64_t* n_global) {
  if (!b || !n_global) return SEM_EINVAL;
  for (int i = 0; i < b->n; ++i) n_global[i] = b->ng[i];
  return SEM_OK;
}

int sem_batch_solve(sem_batch b, const double* const* b_dev, double* const* x_dev, const sem_solve_opts* o,
                    sem_solve_stats* st, void* stream) {
  if (!b || !b_dev || !x_dev) return SEM_EINVAL;
  sem_solve_opts d;
  sem_default_solve_opts(&d);
  if (!o) o = &d;
  if (o->pc < 0 || o->pc > 3 || o->max_iter < 0 || !(o->rtol >= 0.0)) return SEM_EINVAL;
  for (int i = 0; i < b->n; ++i)
    if (!b_dev[i] || !x_dev[i]) return SEM_EINVAL;
  return guarded_call([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    const int check = std::max(1, o->check_every);
    const bool refined = o->mode == SEM_SOLVE_FP32_REFINED;
    if (refined && !b->groups.front().f32.v[0].p) throw Error{SEM_EUNSUPPORTED, "batch built without FP32 copies"};
    if (o->use_x0) throw Error{SEM_EUNSUPPORTED, "batched solves start from x = 0"};
    // b -> union slot 5 (zero on the Dirichlet set); x = 0
    copy_in(b, b_dev, 5, s);
    for (auto& g : b->groups) {
      hipLaunchKernelGGL(mask_vec_kernel, dim3(grid_for(g.mesh->T.n_global)), dim3(256), 0, s, g.f64.v[5].p,
                         (const uint8_t*)g.mesh->dir.p, g.mesh->T.n_global);
      hipLaunchKernelGGL((fill_vec_kernel<double>), dim3(grid_for(g.mesh->T.n_global)), dim3(256), 0, s,
                         g.f64.v[0].p, 0.0, g.mesh->T.n_global);
    }
    std::vector<int> iters(b->n, 0), outer(b->n, 0);
    std::vector<double> host_sc((size_t)b->n * kScal), host_out((size_t)b->n * kScal);
    if (!refined) {
      for (auto& g : b->groups)
        hipLaunchKernelGGL((copy_vec_kernel<double>), dim3(grid_for(g.mesh->T.n_global)), dim3(256), 0, s,
                           g.f64.v[1].p, (const double*)g.f64.v[5].p, g.mesh->T.n_global);
      int total = batched_pcg<double>(b, o->rtol, o->max_iter, o->pc, check, s);
      // the recursive residual can drift below the true one: b - A x per
      // instance, and PCG again from it for the instances still above their
      // tolerance (as the single solve does)
      for (;;) {
        for (auto& g : b->groups) {
          apply_A<double>(g.mesh.get(), g.f64.v[0].p, g.f64.v[4].p, s);
          if (!g.chunk_ids.empty())
            hipLaunchKernelGGL(seg_residual_kernel, dim3((unsigned)g.chunk_ids.size()), dim3(256), 0, s, g.f64.v[1].p,
                               (const double*)g.f64.v[5].p, (const double*)g.f64.v[4].p, g.d_chunk_ids.p,
                               b->d_chunks.p, b->part.p);
        }
        hipLaunchKernelGGL(seg_restart_kernel, dim3(1), dim3(64), 0, s, (const double*)b->part.p,
                           (const int32_t*)b->d_inst_chunk_off.p, b->sc.p, b->n, b->nactive.p);
        SEM_HIP(hipGetLastError());
        if (read_active(b, s) == 0.0 || total >= o->max_iter) break;
        total += batched_pcg<double>(b, o->rtol, o->max_iter - total, o->pc, check, s, true);
      }
      SEM_HIP(hipMemcpyAsync(host_sc.data(), b->sc.p, host_sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      SEM_HIP(hipStreamSynchronize(s));
      for (int i = 0; i < b->n; ++i) {
        iters[i] = (int)host_sc[(size_t)i * kScal + kIters];
        outer[i] = (int)host_sc[(size_t)i * kScal + kRestarts];
      }
    } else {
      // outer: r = b - A x in FP64 per instance; inner: FP32 batched PCG on r / ||r||
      for (int it = 0; it <= o->max_outer; ++it) {
        for (auto& g : b->groups) {
          apply_A<double>(g.mesh.get(), g.f64.v[0].p, g.f64.v[4].p, s);
          if (!g.chunk_ids.empty())
            hipLaunchKernelGGL(seg_residual_kernel, dim3((unsigned)g.chunk_ids.size()), dim3(256), 0, s, g.f64.v[1].p,
                               (const double*)g.f64.v[5].p, (const double*)g.f64.v[4].p, g.d_chunk_ids.p,
                               b->d_chunks.p, b->part.p);
        }
        seg_final(b, b->sc_outer.p, kRr, 0, s);
        if (it == 0) {
          // ||b||^2 = ||r||^2 at x = 0: sets each instance's tolerance
          hipLaunchKernelGGL(seg_init_kernel, dim3(1), dim3(64), 0, s, b->sc_outer.p, (const double*)b->sc_outer.p,
                             (int)kRr, b->n, o->rtol * o->rtol);
        } else {
          // refreshed residuals: stop the instances that meet their tolerance
          hipLaunchKernelGGL(seg_final_kernel, dim3(1), dim3(64), 0, s, b->part.p, b->d_inst_chunk_off.p,
                             b->sc_outer.p, b->n, 0, 3, b->nactive.p);
        }
        SEM_HIP(hipMemcpyAsync(host_out.data(), b->sc_outer.p, host_out.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        SEM_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int i = 0; i < b->n; ++i) any |= host_out[(size_t)i * kScal + kActive] != 0.0;
        if (!any || it == o->max_outer) break;
        for (int i = 0; i < b->n; ++i)
          if (host_out[(size_t)i * kScal + kActive] != 0.0) outer[i]++;
        hipLaunchKernelGGL(seg_norm_kernel, dim3(1), dim3(64), 0, s, b->sc_outer.p, b->n, (int)kRr);
        for (auto& g : b->groups) {
          if (g.chunk_ids.empty()) continue;
          hipLaunchKernelGGL((seg_scale_kernel<float, double>), dim3((unsigned)g.chunk_ids.size()), dim3(256), 0, s,
                             g.f32.v[1].p, (const double*)g.f64.v[1].p, g.d_chunk_ids.p, b->d_chunks.p,
                             (const double*)b->sc_outer.p, 1);
          hipLaunchKernelGGL((fill_vec_kernel<float>), dim3(grid_for(g.mesh->T.n_global)), dim3(256), 0, s,
                             g.f32.v[0].p, 0.0f, g.mesh->T.n_global);
        }
        batched_pcg<float>(b, o->inner_rtol, o->max_iter, o->pc, check, s);
        SEM_HIP(hipMemcpyAsync(host_sc.data(), b->sc.p, host_sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        SEM_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < b->n; ++i)
          if (host_out[(size_t)i * kScal + kActive] != 0.0) iters[i] += (int)host_sc[(size_t)i * kScal + kIters];
        for (auto& g : b->groups) {
          if (g.chunk_ids.empty()) continue;
          hipLaunchKernelGGL(seg_correct_kernel, dim3((unsigned)g.chunk_ids.size()), dim3(256), 0, s, g.f64.v[0].p,
                             (const float*)g.f32.v[0].p, g.d_chunk_ids.p, b->d_chunks.p,
                             (const double*)b->sc_outer.p);
        }
      }
      host_sc = host_out;
    }
    copy_out(b, x_dev, 0, s);
    SEM_HIP(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int status = SEM_OK;
    for (int i = 0; i < b->n; ++i) {
      const double* S = &host_sc[(size_t)i * kScal];
      const double rel = S[kBb] > 0.0 ? std::sqrt(S[kRr] / S[kBb]) : 0.0;
      const bool flag = S[kFlag] != 0.0;
      const bool conv = S[kBb] == 0.0 || S[kRr] <= S[kTol2];
      if (st) {
        st[i].iterations = iters[i];
        st[i].outer_iterations = outer[i];
        st[i].rel_residual = rel;
        st[i].solve_ms = ms;
        st[i].history_len = 0;
      }
      if (flag)
        status = SEM_EBREAKDOWN;
      else if (!conv && status == SEM_OK)
        status = SEM_ENOCONV;
    }
    if (status == SEM_EBREAKDOWN) set_error("PCG breakdown in a batched instance");
    if (status == SEM_ENOCONV) set_error("a batched instance did not reach its tolerance");
    return status;
  });
}

}  // extern "C"
