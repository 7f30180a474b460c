// HIP kernels of the spectral-element solver for gfx950 (wave64, LDS-staged).
// Included once, by sem_device.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sem_internal.h"

namespace sem {

// elements per workgroup of the operator kernel: about 128 lanes per group
template <int N>
constexpr int ax_epb() {
  return (64 / ((N + 1) * (N + 1))) > 0 ? (64 / ((N + 1) * (N + 1))) : 1;
}

__device__ __forceinline__ void unpack_coef(int32_t code, int& ai, int& aj, int& ak) {
  ai = (int32_t)((uint32_t)code << 22) >> 22;
  aj = (int32_t)((uint32_t)code << 12) >> 22;
  ak = (int32_t)((uint32_t)code << 2) >> 22;
}

__device__ __forceinline__ int node_class(int x, int N) { return x == 0 ? 0 : (x == N ? 2 : 1); }

// Constant coefficients of the model problem c u - div(kappa grad u) = s
// (eq. (pde)): the operator is kappa times the stiffness action plus c times
// the mass term.  With GLL quadrature the element mass is diagonal, m_{ijk;e}
// at each node (Section 2.4), so its assembly is the lumped mass m_N: the
// kernels add c m_N u_N where each global node's value is written.
// With one kappa_e and c_e per element (Algorithm 2), the element kernel
// applies them to its own local values instead: kappa_e r + c_e m_{ijk;e} u.
template <typename T>
struct OpCoef {
  T kap, cm;
  const T* mN;  // lumped mass [n_global]; read only when cm != 0
  int scaled;   // constant coefficients other than kappa = 1, c = 0
  const T* ke;  // per element: kappa_e [E] (NULL: constant coefficients)
  const T* ce;  // per element: c_e [E]
  const T* mL;  // per element: local mass m_{ijk;e} [E][(N+1)^3], read where c_e != 0
  const T* kn;  // per node: kappa_{ijk;e} [E][(N+1)^3], read by the kernel that rebuilds G
                // (the stored factors carry kappa already); NULL otherwise
};

template <typename T>
__device__ __forceinline__ T op_value(const OpCoef<T>& oc, T stiff, int64_t g, T ug) {
  if (!oc.scaled) return stiff;
  T v = oc.kap * stiff;
  if (oc.cm != T(0)) v += oc.cm * oc.mN[g] * ug;
  return v;
}

// element e's kappa_e, c_e (1, 0 without per-element coefficients), read
// once per element before its results are stored
template <typename T>
struct ElemCoef {
  T k, c;
};

template <typename T>
__device__ __forceinline__ ElemCoef<T> elem_coef(const OpCoef<T>& oc, int64_t e) {
  if (oc.ke == nullptr) return ElemCoef<T>{T(1), T(0)};
  return ElemCoef<T>{oc.ke[e], oc.ce[e]};
}

// local value of element e at local node `loc` with per-element coefficients
template <typename T>
__device__ __forceinline__ T elem_value(const OpCoef<T>& oc, const ElemCoef<T>& ec, int64_t e, int64_t nloc, int loc,
                                        T stiff, T ul) {
  if (oc.ke == nullptr) return stiff;
  T v = ec.k * stiff;
  if (ec.c != T(0)) v += ec.c * oc.mL[e * nloc + loc] * ul;
  return v;
}

// ---------------------------------------------------------------------------
// Operator kernel, eq. (R) / Algorithm 2.  One (N+1)^2-lane group per element:
// lane (i,j) keeps the k-pencil of u and of the result in registers, the
// xi/eta contractions go through one LDS plane at a time.  Global ids come
// from the element's entity records (scatter of eq. (scatter) fused into the
// load); interior results go straight to y, shared-node results to the work
// array w that the gather kernel sums.
// ---------------------------------------------------------------------------
// value a[k] of a register array for a wave-uniform runtime index k
template <typename T, int M>
__device__ __forceinline__ T pick(const T (&a)[M], int k) {
  T r = a[0];
#pragma unroll
  for (int m = 1; m < M; ++m) r = (m == k) ? a[m] : r;
  return r;
}

// Sum of v over a workgroup of NT lanes in a fixed order (deterministic):
// wave shuffles when NT is a multiple of 64, else a tree in LDS (red[NT]).
// Every lane of the workgroup must call it; lane 0 gets the result.
template <int NT>
__device__ __forceinline__ double group_sum(double v, double* red) {
  const int tid = threadIdx.x;
  if constexpr (NT % 64 == 0) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
      for (int q = 0; q < NT / 64; ++q) s += red[q];
    return s;
  } else {
    constexpr int P2 = NT >= 512 ? 512 : NT >= 256 ? 256 : NT >= 128 ? 128 : NT >= 64 ? 64 : NT >= 32 ? 32 : NT >= 16 ? 16 : 8;
    red[tid] = v;
    __syncthreads();
    if (tid < NT - P2) red[tid] += red[tid + P2];
    __syncthreads();
    for (int h = P2 / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    return red[0];
  }
}

// global id and work slot of lane (i, j)'s node in plane k, from the records
struct NodeAddr {
  int g, w, flags;
};

__device__ __forceinline__ NodeAddr node_addr(const int32_t* __restrict__ rec, int64_t e, int cx, int cy, int k,
                                              int i, int j, int N) {
  const int32_t* r = rec + ((e * kClasses + cx + 3 * cy + 9 * node_class(k, N)) * kRecInts);
  int ai, aj, ak;
  unpack_coef(r[1], ai, aj, ak);
  const int off = ai * i + aj * j + ak * k;
  return NodeAddr{r[0] + off, r[2] + off, r[3]};
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b on XCD b % 8):
// give each XCD one contiguous run of the traversal order so that elements
// that share faces, edges and vertices meet in the same L2.
__device__ __forceinline__ int64_t xcd_position(int64_t b, int64_t nlogical) {
  const int64_t per = (nlogical + 7) / 8;
  return (b & 7) * per + (b >> 3);
}

inline int64_t xcd_grid(int64_t nlogical) { return ((nlogical + 7) / 8) * 8; }

// GEO = false: the factors G are read from memory (6 per node).  GEO = true:
// they are rebuilt at every node from the element's 8 vertices (the r' kernel
// of Section 5.1 and Table 3, which trades the factor stream for arithmetic): the columns of
// the Jacobian of the trilinear map, c0 = dx/dxi etc., their cross products
// a0 = c1 x c2, a1 = c2 x c0, a2 = c0 x c1 (the rows of det J . J^-1), and
// G_ab = rho_i rho_j rho_k (a_a . a_b) / det J with det J = c0 . a0, the same
// rho rho rho |J| (J^T J)^-1 as the stored factors.  In that case G points to
// the vertex coordinates [E][8][3] and tq to the GLL points and weights [2][N+1].
// KN (with GEO): kappa per node (oc.kn) scales the rebuilt factors at its node;
// the element's values are staged in LDS next to u.
// 1/d for a positive, normal d: hardware reciprocal refined by Newton steps
// (two in FP64, one in FP32): within about an ulp of the rounded quotient
__device__ __forceinline__ double recip_pos(double d) {
  double y = __builtin_amdgcn_rcp(d);
  y = __builtin_fma(y, __builtin_fma(-d, y, 1.0), y);
  return __builtin_fma(y, __builtin_fma(-d, y, 1.0), y);
}

__device__ __forceinline__ float recip_pos(float d) {
  const float y = __builtin_amdgcn_rcpf(d);
  return __builtin_fmaf(y, __builtin_fmaf(-d, y, 1.0f), y);
}

template <int N, typename T, int EPB, bool GEO = false, bool KN = false>
__global__ void __launch_bounds__(EPB*(N + 1) * (N + 1))
__attribute__((amdgpu_waves_per_eu(N <= 9 ? (GEO && sizeof(T) == 8 ? 3 : 4) : 1, 8)))
ax_kernel(const T* __restrict__ u, T* __restrict__ y, T* __restrict__ w, const T* __restrict__ G,
          const int32_t* __restrict__ rec, const T* __restrict__ Dg, const uint8_t* __restrict__ dir,
          const int32_t* __restrict__ order, int64_t E, double* __restrict__ dpart, const T* __restrict__ tq,
          OpCoef<T> oc) {
  constexpr int n1 = N + 1, P = n1 * n1, NN = P * n1;
  __shared__ T sD[P];
  __shared__ double sRed[EPB * P];
  __shared__ T sU[EPB][NN];  // the element's gathered u, all planes
  __shared__ T sA[EPB][P];
  __shared__ T sB[EPB][P];
  __shared__ T sK[KN ? EPB : 1][KN ? NN : 1];  // KN: the element's kappa per node
  const int tid = threadIdx.x;
  const int le = tid / P, ij = tid - le * P;
  const int i = ij % n1, j = ij / n1;
  const int64_t pos = xcd_position(blockIdx.x, (E + EPB - 1) / EPB) * EPB + le;
  const bool valid = pos < E;
  const int64_t e = valid ? order[pos] : 0;
  const int cx = node_class(i, N), cy = node_class(j, N);
  // The lane's k-pencil crosses three entity records (k = 0, interior k,
  // k = N).  Loads go out in dependency order with no wait between them:
  // records, then the factors of plane 0, then all u values, then D.
  const int4* rp = reinterpret_cast<const int4*>(rec) + e * kClasses + cx + 3 * cy;
  const int4 r0 = rp[0], r1 = rp[9], r2 = rp[18];
  // factors of plane k in registers, plane k+1 prefetched during plane k
  const T* Ge = G + (GEO ? e * 24 : e * 6 * NN + ij);
  T g0 = 0, g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0;
  // GEO: the lane's k-independent parts of the Jacobian columns,
  // c0 = f0(zeta) P0 + f1(zeta) P1, c1 = f0(zeta) Q0 + f1(zeta) Q1, c2 = C2
  T P0[3], P1[3], Q0[3], Q1[3], C2[3], rij = 0;
  if constexpr (GEO) {
    const T ti = tq[i], tj = tq[j];
    const T f0i = T(0.5) * (T(1) - ti), f1i = T(0.5) * (T(1) + ti);
    const T f0j = T(0.5) * (T(1) - tj), f1j = T(0.5) * (T(1) + tj);
    rij = tq[n1 + i] * tq[n1 + j];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      // x(a, b, c) = Ge[(a + 2 b + 4 c) * 3 + q]
      P0[q] = T(0.5) * ((Ge[1 * 3 + q] - Ge[0 * 3 + q]) * f0j + (Ge[3 * 3 + q] - Ge[2 * 3 + q]) * f1j);
      P1[q] = T(0.5) * ((Ge[5 * 3 + q] - Ge[4 * 3 + q]) * f0j + (Ge[7 * 3 + q] - Ge[6 * 3 + q]) * f1j);
      Q0[q] = T(0.5) * ((Ge[2 * 3 + q] - Ge[0 * 3 + q]) * f0i + (Ge[3 * 3 + q] - Ge[1 * 3 + q]) * f1i);
      Q1[q] = T(0.5) * ((Ge[6 * 3 + q] - Ge[4 * 3 + q]) * f0i + (Ge[7 * 3 + q] - Ge[5 * 3 + q]) * f1i);
      C2[q] = T(0.5) * ((Ge[4 * 3 + q] - Ge[0 * 3 + q]) * f0i * f0j + (Ge[5 * 3 + q] - Ge[1 * 3 + q]) * f1i * f0j +
                        (Ge[6 * 3 + q] - Ge[2 * 3 + q]) * f0i * f1j + (Ge[7 * 3 + q] - Ge[3 * 3 + q]) * f1i * f1j);
    }
  } else {
    g0 = Ge[0 * NN];
    g1 = Ge[1 * NN];
    g2 = Ge[2 * NN];
    g3 = Ge[3 * NN];
    g4 = Ge[4 * NN];
    g5 = Ge[5 * NN];
  }
  T rw[n1];
  T uv[n1];  // the lane's own pencil of u (GEO: also used for the zeta derivative)
  {
#pragma unroll
    for (int k = 0; k < n1; ++k) {
      const int4 r = k == 0 ? r0 : (k == N ? r2 : r1);
      int ai, aj, ak;
      unpack_coef(r.y, ai, aj, ak);
      uv[k] = u[r.x + ai * i + aj * j + ak * k];
    }
    for (int x = tid; x < P; x += EPB * P) sD[x] = Dg[x];
#pragma unroll
    for (int k = 0; k < n1; ++k) {
      sU[le][k * P + ij] = valid ? uv[k] : T(0);
      rw[k] = T(0);
    }
    if constexpr (KN) {
#pragma unroll
      for (int k = 0; k < n1; ++k) sK[le][k * P + ij] = valid ? oc.kn[e * NN + k * P + ij] : T(1);
    }
  }
  __syncthreads();
  // FP64 rebuilt-factor form: the lane's two columns of D stay in registers
  // (fewer LDS reads for the transposed contractions; the other forms keep
  // their register budget for the factor stream)
  constexpr bool kDc = GEO && sizeof(T) == 8;
  T Dci[kDc ? n1 : 1], Dcj[kDc ? n1 : 1];
  if constexpr (kDc) {
#pragma unroll
    for (int m = 0; m < n1; ++m) {
      Dci[m] = sD[m * n1 + i];
      Dcj[m] = sD[m * n1 + j];
    }
  }
#pragma unroll 1
  for (int k = 0; k < n1; ++k) {
    T h0 = 0, h1 = 0, h2 = 0, h3 = 0, h4 = 0, h5 = 0;
    if constexpr (GEO) {
      const T tk = tq[k];  // wave-uniform
      const T f0k = T(0.5) * (T(1) - tk), f1k = T(0.5) * (T(1) + tk);
      T c0[3], c1[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        c0[q] = f0k * P0[q] + f1k * P1[q];
        c1[q] = f0k * Q0[q] + f1k * Q1[q];
      }
      const T a0x = c1[1] * C2[2] - c1[2] * C2[1], a0y = c1[2] * C2[0] - c1[0] * C2[2], a0z = c1[0] * C2[1] - c1[1] * C2[0];
      const T a1x = C2[1] * c0[2] - C2[2] * c0[1], a1y = C2[2] * c0[0] - C2[0] * c0[2], a1z = C2[0] * c0[1] - C2[1] * c0[0];
      const T a2x = c0[1] * c1[2] - c0[2] * c1[1], a2y = c0[2] * c1[0] - c0[0] * c1[2], a2z = c0[0] * c1[1] - c0[1] * c1[0];
      const T det = c0[0] * a0x + c0[1] * a0y + c0[2] * a0z;
      T sc = rij * tq[n1 + k] * recip_pos(det);
      if constexpr (KN) sc *= sK[le][k * P + ij];  // kappa at the node (eq. (R))
      g0 = sc * (a0x * a0x + a0y * a0y + a0z * a0z);
      g1 = sc * (a0x * a1x + a0y * a1y + a0z * a1z);
      g2 = sc * (a0x * a2x + a0y * a2y + a0z * a2z);
      g3 = sc * (a1x * a1x + a1y * a1y + a1z * a1z);
      g4 = sc * (a1x * a2x + a1y * a2y + a1z * a2z);
      g5 = sc * (a2x * a2x + a2y * a2y + a2z * a2z);
    } else {
      const T* Gn = Ge + (k + 1 < n1 ? k + 1 : 0) * P;
      h0 = Gn[0 * NN];
      h1 = Gn[1 * NN];
      h2 = Gn[2 * NN];
      h3 = Gn[3 * NN];
      h4 = Gn[4 * NN];
      h5 = Gn[5 * NN];
    }
    const T* Dk = Dg + k * n1;  // wave-uniform: scalar loads
    const T* su = &sU[le][k * P];
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int m = 0; m < n1; ++m) {
      ur += sD[i * n1 + m] * su[j * n1 + m];
      us += sD[j * n1 + m] * su[m * n1 + i];
      ut += Dk[m] * (GEO ? uv[m] : sU[le][m * P + ij]);
    }
    const T A = g0 * ur + g1 * us + g2 * ut;
    const T B = g1 * ur + g3 * us + g4 * ut;
    const T C = g2 * ur + g4 * us + g5 * ut;
    sA[le][ij] = A;
    sB[le][ij] = B;
#pragma unroll
    for (int m = 0; m < n1; ++m) rw[m] += Dk[m] * C;
    __syncthreads();
    T acc = 0;
#pragma unroll
    for (int m = 0; m < n1; ++m) {
      T dmi, dmj;
      if constexpr (kDc) {
        dmi = Dci[m];
        dmj = Dcj[m];
      } else {
        dmi = sD[m * n1 + i];
        dmj = sD[m * n1 + j];
      }
      acc += dmi * sA[le][j * n1 + m] + dmj * sB[le][m * n1 + i];
    }
#pragma unroll
    for (int m = 0; m < n1; ++m) rw[m] = (m == k) ? rw[m] + acc : rw[m];
    __syncthreads();
    if constexpr (!GEO) {
      g0 = h0;
      g1 = h1;
      g2 = h2;
      g3 = h3;
      g4 = h4;
      g5 = h5;
    }
  }
  // interior results straight to y, shared ones to the work array; with dpart,
  // this workgroup's share of u . y over the interior nodes
  double dacc = 0.0;
  if (valid) {
    const bool masked_interior = rec[(e * kClasses + kInteriorClass) * kRecInts + 3] & kFlagMaskedInterior;
    const ElemCoef<T> ec = elem_coef(oc, e);
#pragma unroll
    for (int k = 0; k < n1; ++k) {
      const int4 r = k == 0 ? r0 : (k == N ? r2 : r1);
      int ai, aj, ak;
      unpack_coef(r.y, ai, aj, ak);
      const int off = ai * i + aj * j + ak * k;
      const T uk = ((r.w & kFlagInterior) || oc.ke != nullptr) ? sU[le][k * P + ij] : T(0);
      const T v = elem_value(oc, ec, e, NN, k * P + ij, rw[k], uk);
      if (r.w & kFlagInterior) {
        const T yv = (masked_interior && dir[r.x + off]) ? T(0) : op_value(oc, v, r.x + off, uk);
        y[r.x + off] = yv;
        dacc += (double)uk * (double)yv;
      } else {
        w[r.z + off] = v;
      }
    }
  }
  if (dpart != nullptr) {
    const double t = group_sum<EPB * P>(dacc, sRed);
    if (tid == 0) dpart[blockIdx.x] = t;
  }
}


// ---------------------------------------------------------------------------
// One 1D contraction of a line of n1 = N + 1 values by a matrix A with
// A[N-q][N-m] = -A[q][m] (the GLL derivative matrix D and D^T: the points are
// symmetric about 0).  With e_m = x_m + x_{N-m} and o_m = x_m - x_{N-m}
// (m < H = n1/2), the outputs q and N-q are E + O and O - E, E = sum_m
// Ap[q][m] e_m (+ A[q][H] x_H for odd n1), O = sum_m Am[q][m] o_m, so a line
// costs H (n1 + 1) multiply-adds instead of n1^2.  tb: rows q < H of
// [Ap[q][0..H-1], A[q][H] (odd n1), Am[q][0..H-1]], then for odd n1 the middle
// output's Am[H][0..H-1] (read with wave-uniform addresses).  ld(m) reads
// entry m of the line, st(q, v) writes output q; every read comes first, so
// the output may overwrite the line.
// Whether the line-phase operator kernel contracts its lines by output pairs:
// everywhere but the FP64 kernels up to N = 9, which run at the 128-VGPR limit
// of 4 waves per SIMD and measure faster with the row-by-row form (at 56^3,
// N = 7: 0.628-0.636 ms against 0.635-0.651 ms; at N = 15 the pairs take
// FP64 from 0.330 to 0.306 ms and FP32 from 0.171 to 0.151 ms).
template <int N, typename T>
constexpr bool line_pairs_on() {
  return !(N <= 9 && sizeof(T) == 8);
}

// Whether the pencil's nodes k and N-k are processed together (the zeta
// derivative and the zeta part of D^T C by output pairs as well): from N = 10,
// where the kernel has registers to spare (N = 15: 0.303-0.308 -> 0.288-0.289 ms
// FP64, 0.150-0.154 -> 0.139 ms FP32); at N = 7 FP32 it measured 2-3% slower.
template <int N, typename T>
constexpr bool zeta_pairs_on() {
  return line_pairs_on<N, T>() && N >= 10;
}

template <int n1>
constexpr int dsplit_size() {
  return (n1 / 2) * (2 * (n1 / 2) + n1 % 2) + (n1 % 2) * (n1 / 2);
}

template <int n1, typename T, typename Ld, typename St>
__device__ __forceinline__ void line_pairs(const T* __restrict__ tb, Ld ld, St st) {
  constexpr int H = n1 / 2, OD = n1 % 2, RW = 2 * H + OD;
  T e[H], o[H], xm = T(0);
#pragma unroll
  for (int m = 0; m < H; ++m) {
    const T l = ld(m), r = ld(n1 - 1 - m);
    e[m] = l + r;
    o[m] = l - r;
  }
  if constexpr (OD) xm = ld(H);
#pragma unroll 1
  for (int q = 0; q < H; ++q) {
    const T* row = tb + q * RW;
    T E = 0, O = 0;
#pragma unroll
    for (int m = 0; m < H; ++m) E += row[m] * e[m];
    if constexpr (OD) E += row[H] * xm;
#pragma unroll
    for (int m = 0; m < H; ++m) O += row[H + OD + m] * o[m];
    st(q, E + O);
    st(n1 - 1 - q, O - E);
  }
  if constexpr (OD) {
    const T* row = tb + H * RW;
    T O = 0;
#pragma unroll
    for (int m = 0; m < H; ++m) O += row[m] * o[m];
    st(H, O);
  }
}

// ---------------------------------------------------------------------------
// Operator kernel by line phases, eq. (R) / Algorithm 2.  Each 1D contraction
// is done by lanes that own whole lines of the element, so the derivative
// matrix is wave-uniform (scalar registers) and every line is read from LDS
// once per contraction instead of once per output node:
//   eta lines    (lane (i, k)):  u_s = D u along eta          -> Z
//   xi lines     (lane (j, k)):  u_r = D u along xi, in place -> X
//   pencils      (lane (i, j)):  u_t = D u along zeta in registers; the factors
//                G (stored, or rebuilt from the vertices); A -> X, B -> Z in
//                place; the zeta part of the transposed sum D^T C in registers
//   xi, eta lines: D^T A along xi in place in X, D^T B along eta in place in Z
//   pencils:     result = zeta part + X + Z at the lane's nodes
// Two padded LDS buffers per element (line stride N + 2, plane stride
// (N + 1)(N + 2)); lanes of one element read distinct banks along all three
// directions.  Same arguments, results and epilogue as ax_kernel.
// ---------------------------------------------------------------------------
template <int N, typename T, int EPB, bool GEO = false, bool KN = false>
__global__ void __launch_bounds__(EPB*(N + 1) * (N + 1))
__attribute__((amdgpu_waves_per_eu(N <= 9 ? 4 : 1, 8)))
ax_line_kernel(const T* __restrict__ u, T* __restrict__ y, T* __restrict__ w, const T* __restrict__ G,
               const int32_t* __restrict__ rec, const T* __restrict__ Dg, const uint8_t* __restrict__ dir,
               const int32_t* __restrict__ order, int64_t E, double* __restrict__ dpart, const T* __restrict__ tq,
               OpCoef<T> oc) {
  constexpr int n1 = N + 1, P = n1 * n1, NN = P * n1;
  constexpr int LS = n1 + 1, PS = n1 * LS, BS = n1 * PS;
  constexpr bool PAIRS = line_pairs_on<N, T>(), ZPAIRS = zeta_pairs_on<N, T>();
  __shared__ T sX[EPB][BS];
  __shared__ T sZ[EPB][BS];
  __shared__ double sRed[EPB * P];
  const int tid = threadIdx.x;
  const int le = tid / P, ij = tid - le * P;
  const int a = ij % n1, b = ij / n1;  // pencil (i, j) = (a, b); lines (., k = b)
  const int64_t pos = xcd_position(blockIdx.x, (E + EPB - 1) / EPB) * EPB + le;
  const bool valid = pos < E;
  const int64_t e = valid ? order[pos] : 0;
  const int cx = node_class(a, N), cy = node_class(b, N);
  const int4* rp = reinterpret_cast<const int4*>(rec) + e * kClasses + cx + 3 * cy;
  const int4 r0 = rp[0], r1 = rp[9], r2 = rp[18];
  const T* Ge = G + (GEO ? e * 24 : e * 6 * NN + ij);
  // Rebuilt factors: along the lane's pencil (i, j) the Jacobian columns are
  // dx/dxi = f0(t) P0 + f1(t) P1, dx/deta = f0(t) Q0 + f1(t) Q1 (f0,1 = (1 -+ t)/2)
  // and dx/dzeta = C2 (no t), so the cofactor rows a0 = dx/deta x C2 and
  // a1 = C2 x dx/dxi are linear in t and a2 = dx/dxi x dx/deta is quadratic:
  // a0 = A0 + t A1, a1 = B0 + t B1, a2 = Z0 + t (Z1 + t Z2), and
  // |J| = a2 . C2 = d0 + t (d1 + t d2).
  T A0[3], A1[3], B0[3], B1[3], Z0[3], Z1[3], Z2[3], d0 = 0, d1 = 0, d2 = 0, rij = 0;
  if constexpr (GEO) {
    const T ti = tq[a], tj = tq[b];
    const T f0i = T(0.5) * (T(1) - ti), f1i = T(0.5) * (T(1) + ti);
    const T f0j = T(0.5) * (T(1) - tj), f1j = T(0.5) * (T(1) + tj);
    rij = tq[n1 + a] * tq[n1 + b];
    T P0[3], P1[3], Q0[3], Q1[3], C2[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      P0[q] = T(0.5) * ((Ge[1 * 3 + q] - Ge[0 * 3 + q]) * f0j + (Ge[3 * 3 + q] - Ge[2 * 3 + q]) * f1j);
      P1[q] = T(0.5) * ((Ge[5 * 3 + q] - Ge[4 * 3 + q]) * f0j + (Ge[7 * 3 + q] - Ge[6 * 3 + q]) * f1j);
      Q0[q] = T(0.5) * ((Ge[2 * 3 + q] - Ge[0 * 3 + q]) * f0i + (Ge[3 * 3 + q] - Ge[1 * 3 + q]) * f1i);
      Q1[q] = T(0.5) * ((Ge[6 * 3 + q] - Ge[4 * 3 + q]) * f0i + (Ge[7 * 3 + q] - Ge[5 * 3 + q]) * f1i);
      C2[q] = T(0.5) * ((Ge[4 * 3 + q] - Ge[0 * 3 + q]) * f0i * f0j + (Ge[5 * 3 + q] - Ge[1 * 3 + q]) * f1i * f0j +
                        (Ge[6 * 3 + q] - Ge[2 * 3 + q]) * f0i * f1j + (Ge[7 * 3 + q] - Ge[3 * 3 + q]) * f1i * f1j);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int q1 = (q + 1) % 3, q2 = (q + 2) % 3;
      const T x0 = Q0[q1] * C2[q2] - Q0[q2] * C2[q1], x1 = Q1[q1] * C2[q2] - Q1[q2] * C2[q1];
      const T y0 = C2[q1] * P0[q2] - C2[q2] * P0[q1], y1 = C2[q1] * P1[q2] - C2[q2] * P1[q1];
      const T z00 = P0[q1] * Q0[q2] - P0[q2] * Q0[q1], z11 = P1[q1] * Q1[q2] - P1[q2] * Q1[q1];
      const T z01 = (P0[q1] * Q1[q2] - P0[q2] * Q1[q1]) + (P1[q1] * Q0[q2] - P1[q2] * Q0[q1]);
      A0[q] = T(0.5) * (x0 + x1);
      A1[q] = T(0.5) * (x1 - x0);
      B0[q] = T(0.5) * (y0 + y1);
      B1[q] = T(0.5) * (y1 - y0);
      Z0[q] = T(0.25) * (z00 + z01 + z11);
      Z1[q] = T(0.5) * (z11 - z00);
      Z2[q] = T(0.25) * (z00 - z01 + z11);
    }
    d0 = Z0[0] * C2[0] + Z0[1] * C2[1] + Z0[2] * C2[2];
    d1 = Z1[0] * C2[0] + Z1[1] * C2[1] + Z1[2] * C2[2];
    d2 = Z2[0] * C2[0] + Z2[1] * C2[1] + Z2[2] * C2[2];
  }
  T uv[n1];
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    const int4 r = k == 0 ? r0 : (k == N ? r2 : r1);
    int ai, aj, ak;
    unpack_coef(r.y, ai, aj, ak);
    uv[k] = valid ? u[r.x + ai * a + aj * b + ak * k] : T(0);
  }
  T kv[KN ? n1 : 1];
  if constexpr (KN) {
#pragma unroll
    for (int k = 0; k < n1; ++k) kv[k] = valid ? oc.kn[e * NN + k * P + ij] : T(1);
  }
  T* X = sX[le];
  T* Z = sZ[le];
#pragma unroll
  for (int k = 0; k < n1; ++k) X[k * PS + b * LS + a] = uv[k];
  __syncthreads();
  // Line contractions: by output pairs (line_pairs, with the even/odd split of
  // D and of D^T stored after D), or row by row with the full D (the form
  // that keeps more independent accumulators; see line_pairs_on); the line
  // sits in registers.
  const T* Dsp = Dg + n1 * n1;             // D
  const T* DTsp = Dsp + dsplit_size<n1>();  // D^T
  if constexpr (PAIRS) {
    // eta lines: lane (i = a, k = b)
    line_pairs<n1, T>(Dsp, [&](int m) { return X[b * PS + m * LS + a]; },
                      [&](int q, T v) { Z[b * PS + q * LS + a] = v; });
    __syncthreads();
    // xi lines: lane (j = a, k = b), in place
    line_pairs<n1, T>(Dsp, [&](int m) { return X[b * PS + a * LS + m]; },
                      [&](int q, T v) { X[b * PS + a * LS + q] = v; });
    __syncthreads();
  } else {
    // Forward contractions loop over the output index q with row q of D in
    // scalar registers (one row live at a time).
    {  // eta lines: lane (i = a, k = b)
      T v[n1];
#pragma unroll
      for (int m = 0; m < n1; ++m) v[m] = X[b * PS + m * LS + a];
#pragma unroll 1
      for (int q = 0; q < n1; ++q) {
        const T* Dq = Dg + q * n1;
        T s = 0;
#pragma unroll
        for (int m = 0; m < n1; ++m) s += Dq[m] * v[m];
        Z[b * PS + q * LS + a] = s;
      }
    }
    __syncthreads();
    {  // xi lines: lane (j = a, k = b), in place
      T v[n1];
#pragma unroll
      for (int m = 0; m < n1; ++m) v[m] = X[b * PS + a * LS + m];
#pragma unroll 1
      for (int q = 0; q < n1; ++q) {
        const T* Dq = Dg + q * n1;
        T s = 0;
#pragma unroll
        for (int m = 0; m < n1; ++m) s += Dq[m] * v[m];
        X[b * PS + a * LS + q] = s;
      }
    }
    __syncthreads();
  }
  T rw[n1];
#pragma unroll
  for (int k = 0; k < n1; ++k) rw[k] = T(0);
  if constexpr (ZPAIRS) {
    // nodes k and N-k of the pencil together: their zeta derivatives are one
    // output pair of line_pairs on u, and the zeta part of D^T C takes
    // C_k - C_{N-k} against the even part of row k of D and C_k + C_{N-k}
    // against the odd part (rw_m = SE_m + SO_m, rw_{N-m} = SE_m - SO_m)
    constexpr int H = n1 / 2, OD = n1 % 2, RW = 2 * H + OD;
    T ue[H], uo[H], SE[H], SO[H], SM = T(0);
#pragma unroll
    for (int m = 0; m < H; ++m) {
      ue[m] = uv[m] + uv[N - m];
      uo[m] = uv[m] - uv[N - m];
      SE[m] = SO[m] = T(0);
    }
    // A and B of node k to X and Z in place; returns C
    auto node = [&](int k, T ut) -> T {
      const int o = k * PS + b * LS + a;
      const T ur = X[o], us = Z[o];
      T A, B, C;
      if constexpr (GEO) {
        const T tk = tq[k];
        const T a0x = A0[0] + tk * A1[0], a0y = A0[1] + tk * A1[1], a0z = A0[2] + tk * A1[2];
        const T a1x = B0[0] + tk * B1[0], a1y = B0[1] + tk * B1[1], a1z = B0[2] + tk * B1[2];
        const T a2x = Z0[0] + tk * (Z1[0] + tk * Z2[0]), a2y = Z0[1] + tk * (Z1[1] + tk * Z2[1]),
                a2z = Z0[2] + tk * (Z1[2] + tk * Z2[2]);
        const T det = d0 + tk * (d1 + tk * d2);
        T sc = rij * tq[n1 + k] * recip_pos(det);
        if constexpr (KN) sc *= pick(kv, k);  // kappa at the node (eq. (R))
        // G = sc M M^T (M: rows a0, a1, a2): (A, B, C) = sc M (M^T grad u)
        const T vx = ur * a0x + us * a1x + ut * a2x, vy = ur * a0y + us * a1y + ut * a2y,
                vz = ur * a0z + us * a1z + ut * a2z;
        A = sc * (a0x * vx + a0y * vy + a0z * vz);
        B = sc * (a1x * vx + a1y * vy + a1z * vz);
        C = sc * (a2x * vx + a2y * vy + a2z * vz);
      } else {
        const T* Gk = Ge + k * P;
        const T g0 = Gk[0 * NN], g1 = Gk[1 * NN], g2 = Gk[2 * NN], g3 = Gk[3 * NN], g4 = Gk[4 * NN], g5 = Gk[5 * NN];
        A = g0 * ur + g1 * us + g2 * ut;
        B = g1 * ur + g3 * us + g4 * ut;
        C = g2 * ur + g4 * us + g5 * ut;
      }
      X[o] = A;
      Z[o] = B;
      return C;
    };
#pragma unroll 1
    for (int k = 0; k < H; ++k) {
      const T* row = Dsp + k * RW;  // wave-uniform: scalar loads
      T E = 0, O = 0;
#pragma unroll
      for (int m = 0; m < H; ++m) E += row[m] * ue[m];
      if constexpr (OD) E += row[H] * uv[H];
#pragma unroll
      for (int m = 0; m < H; ++m) O += row[H + OD + m] * uo[m];
      const T C1 = node(k, E + O), C2 = node(N - k, O - E);
      const T cd = C1 - C2, cs = C1 + C2;
#pragma unroll
      for (int m = 0; m < H; ++m) {
        SE[m] += row[m] * cd;
        SO[m] += row[H + OD + m] * cs;
      }
      if constexpr (OD) SM += row[H] * cd;
    }
    if constexpr (OD) {  // the middle node (its row of D is odd)
      const T* row = Dsp + H * RW;
      T O = 0;
#pragma unroll
      for (int m = 0; m < H; ++m) O += row[m] * uo[m];
      const T C = node(H, O);
#pragma unroll
      for (int m = 0; m < H; ++m) SO[m] += row[m] * C;
      rw[H] = SM;
    }
#pragma unroll
    for (int m = 0; m < H; ++m) {
      rw[m] = SE[m] + SO[m];
      rw[N - m] = SE[m] - SO[m];
    }
  } else {
#pragma unroll 1
    for (int k = 0; k < n1; ++k) {
      const T* Dk = Dg + k * n1;  // wave-uniform: scalar loads
      const int o = k * PS + b * LS + a;
      const T ur = X[o], us = Z[o];
      T ut = 0;
#pragma unroll
      for (int m = 0; m < n1; ++m) ut += Dk[m] * uv[m];
      T A, B, C;
      if constexpr (GEO) {
        const T tk = tq[k];
        const T a0x = A0[0] + tk * A1[0], a0y = A0[1] + tk * A1[1], a0z = A0[2] + tk * A1[2];
        const T a1x = B0[0] + tk * B1[0], a1y = B0[1] + tk * B1[1], a1z = B0[2] + tk * B1[2];
        const T a2x = Z0[0] + tk * (Z1[0] + tk * Z2[0]), a2y = Z0[1] + tk * (Z1[1] + tk * Z2[1]),
                a2z = Z0[2] + tk * (Z1[2] + tk * Z2[2]);
        const T det = d0 + tk * (d1 + tk * d2);
        T sc = rij * tq[n1 + k] * recip_pos(det);
        if constexpr (KN) sc *= pick(kv, k);  // kappa at the node (eq. (R))
        // G = sc M M^T (M: rows a0, a1, a2): (A, B, C) = sc M (M^T grad u)
        const T vx = ur * a0x + us * a1x + ut * a2x, vy = ur * a0y + us * a1y + ut * a2y,
                vz = ur * a0z + us * a1z + ut * a2z;
        A = sc * (a0x * vx + a0y * vy + a0z * vz);
        B = sc * (a1x * vx + a1y * vy + a1z * vz);
        C = sc * (a2x * vx + a2y * vy + a2z * vz);
      } else {
        const T* Gk = Ge + k * P;
        const T g0 = Gk[0 * NN], g1 = Gk[1 * NN], g2 = Gk[2 * NN], g3 = Gk[3 * NN], g4 = Gk[4 * NN], g5 = Gk[5 * NN];
        A = g0 * ur + g1 * us + g2 * ut;
        B = g1 * ur + g3 * us + g4 * ut;
        C = g2 * ur + g4 * us + g5 * ut;
      }
      X[o] = A;
      Z[o] = B;
#pragma unroll
      for (int m = 0; m < n1; ++m) rw[m] += Dk[m] * C;
    }
  }
  __syncthreads();
  // transposed xi lines (lane (j = a, k = b)) and eta lines (lane (i = a, k = b)), in place
  if constexpr (PAIRS) {
    line_pairs<n1, T>(DTsp, [&](int m) { return X[b * PS + a * LS + m]; },
                      [&](int q, T v) { X[b * PS + a * LS + q] = v; });
    line_pairs<n1, T>(DTsp, [&](int m) { return Z[b * PS + m * LS + a]; },
                      [&](int q, T v) { Z[b * PS + q * LS + a] = v; });
  } else {
    // loop over the input index m: row m of D in scalar registers scales line
    // entry m into all outputs; the results overwrite the line after the loop
    T sx[n1], sz[n1];
#pragma unroll
    for (int q = 0; q < n1; ++q) sx[q] = sz[q] = T(0);
#pragma unroll 1
    for (int m = 0; m < n1; ++m) {
      const T* Dm = Dg + m * n1;
      const T vx = X[b * PS + a * LS + m], vz = Z[b * PS + m * LS + a];
#pragma unroll
      for (int q = 0; q < n1; ++q) {
        sx[q] += Dm[q] * vx;
        sz[q] += Dm[q] * vz;
      }
    }
#pragma unroll
    for (int q = 0; q < n1; ++q) {
      X[b * PS + a * LS + q] = sx[q];
      Z[b * PS + q * LS + a] = sz[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < n1; ++k) rw[k] += X[k * PS + b * LS + a] + Z[k * PS + b * LS + a];
  double dacc = 0.0;
  if (valid) {
    const bool masked_interior = rec[(e * kClasses + kInteriorClass) * kRecInts + 3] & kFlagMaskedInterior;
    const ElemCoef<T> ec = elem_coef(oc, e);
    // the pencil's records read again (cached) rather than kept live through the contractions
    int64_t ro = e * kClasses + cx + 3 * cy;
    asm volatile("" : "+v"(ro));
    const int4* rq = reinterpret_cast<const int4*>(rec) + ro;
    const int4 q0 = rq[0], q1 = rq[9], q2 = rq[18];
#pragma unroll
    for (int k = 0; k < n1; ++k) {
      const int4 r = k == 0 ? q0 : (k == N ? q2 : q1);
      int ai, aj, ak;
      unpack_coef(r.y, ai, aj, ak);
      const int off = ai * a + aj * b + ak * k;
      const T uk = uv[k];
      const T v = elem_value(oc, ec, e, NN, k * P + ij, rw[k], uk);
      if (r.w & kFlagInterior) {
        const T yv = (masked_interior && dir[r.x + off]) ? T(0) : op_value(oc, v, r.x + off, uk);
        y[r.x + off] = yv;
        dacc += (double)uk * (double)yv;
      } else {
        w[r.z + off] = v;
      }
    }
  }
  if (dpart != nullptr) {
    const double t = group_sum<EPB * P>(dacc, sRed);
    if (tid == 0) dpart[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Operator at N = 15 on matrix cores (v_mfma_f64_16x16x4f64 in FP64,
// v_mfma_f32_16x16x4_f32 in FP32: the same operand layout).  One
// workgroup of four waves per element (16^3 nodes).  MFMA operand layout for
// a 16x16 product with K = 4: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and receives D[4r + l/16][l%16] (FP64) or D[4(l/16) + r][l%16] (FP32) in
// accumulator register r = 0..3.
//   1. zeta derivative  UT = D (16x16) x U (16 x 256 columns (j,i)), 4 tiles per wave
//   2. per plane k (4 planes per wave): UR = U_k D^T, US = D U_k, the factors
//      G at the lane's 4 nodes, A, B, C; then W_k = A_k D + D^T B_k
//   3. zeta transpose  W += D^T (16x16) x C (16 x 256), 4 tiles per wave, and the
//      results go to y (element interiors) or the work array (shared nodes).
// D is held in registers in both operand layouts (4 + 4 values per lane).
typedef double sem_d4 __attribute__((ext_vector_type(4)));
typedef float sem_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma4;
template <> struct Mfma4<double> {
  typedef sem_d4 V;
  static __device__ __forceinline__ V fma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct Mfma4<float> {
  typedef sem_f4 V;
  static __device__ __forceinline__ V fma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

template <typename T>

__global__ void __launch_bounds__(256)
ax_mfma15_kernel(const T* __restrict__ u, T* __restrict__ y, T* __restrict__ w,
                 const T* __restrict__ G, const int32_t* __restrict__ rec, const T* __restrict__ Dg,
                 const uint8_t* __restrict__ dir, const int32_t* __restrict__ order, int64_t E,
                 double* __restrict__ dpart, OpCoef<T> oc) {
  typedef typename Mfma4<T>::V V;
  constexpr int N = 15, n1 = 16, P = 256, NN = 4096;
  __shared__ T sU[NN];        // u, later the xi/eta part of the result
  __shared__ T sT[NN];        // zeta derivative of u, later C
  __shared__ __attribute__((aligned(16))) T sS[4][2][P];  // per-wave A_k, B_k; at the end the reduction
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int lr = l & 15, lq = l >> 4;
  // row of the 16x16 result held in accumulator register r: interleaved in FP64
  // (4r + l/16), blocked in FP32 (4(l/16) + r)
  auto orow = [lq](int r) { return std::is_same<T, double>::value ? 4 * r + lq : 4 * lq + r; };
  const int64_t pos = xcd_position(blockIdx.x, E);
  if (pos >= E) {  // whole workgroup
    if (dpart != nullptr && tid == 0) dpart[blockIdx.x] = 0.0;
    return;
  }
  const int64_t e = order[pos];
  // gather: lane tid owns the k-pencil of node (i, j) = (tid % 16, tid / 16)
  {
    const int i0 = tid & 15, j0 = tid >> 4;
    const int cx = node_class(i0, N), cy = node_class(j0, N);
    const int4* rp = reinterpret_cast<const int4*>(rec) + e * kClasses + cx + 3 * cy;
    const int4 r0 = rp[0], r1 = rp[9], r2 = rp[18];
    T uv[n1];
#pragma unroll
    for (int k = 0; k < n1; ++k) {
      const int4 r = k == 0 ? r0 : (k == N ? r2 : r1);
      int ai, aj, ak;
      unpack_coef(r.y, ai, aj, ak);
      uv[k] = u[r.x + ai * i0 + aj * j0 + ak * k];
    }
#pragma unroll
    for (int k = 0; k < n1; ++k) sU[k * P + tid] = uv[k];
  }
  T DA[4], DB[4];  // DA[s] = D[lr][4s+lq] (A layout of D), DB[s] = D[4s+lq][lr] (B layout)
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    DA[s] = Dg[lr * n1 + 4 * s + lq];
    DB[s] = Dg[(4 * s + lq) * n1 + lr];
  }
  __syncthreads();
  // 1. UT[k'][col] = sum_k D[k'][k] U[k][col]
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = wave * 4 + q;
    V acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = Mfma4<T>::fma(DA[s], sU[(4 * s + lq) * P + t * 16 + lr], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) sT[orow(r) * P + t * 16 + lr] = acc[r];
  }
  __syncthreads();
  // 2. planes
  const T* Ge = G + e * 6 * NN;
  V W[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = wave * 4 + q;
    const T* Uk = sU + k * P;
    V ur = {0, 0, 0, 0}, us = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      ur = Mfma4<T>::fma(Uk[lr * n1 + 4 * s + lq], DA[s], ur);  // U_k D^T
      us = Mfma4<T>::fma(DA[s], Uk[(4 * s + lq) * n1 + lr], us);  // D U_k
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int node = k * P + orow(r) * n1 + lr;
      const T ut = sT[node];
      const T g0 = Ge[0 * NN + node], g1 = Ge[1 * NN + node], g2 = Ge[2 * NN + node];
      const T g3 = Ge[3 * NN + node], g4 = Ge[4 * NN + node], g5 = Ge[5 * NN + node];
      const T A = g0 * ur[r] + g1 * us[r] + g2 * ut;
      const T B = g1 * ur[r] + g3 * us[r] + g4 * ut;
      const T C = g2 * ur[r] + g4 * us[r] + g5 * ut;
      sS[wave][0][orow(r) * n1 + lr] = A;
      sS[wave][1][orow(r) * n1 + lr] = B;
      sT[node] = C;  // plane k of the zeta derivative is no longer needed
    }
    __syncthreads();
    V wk = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      wk = Mfma4<T>::fma(sS[wave][0][lr * n1 + 4 * s + lq], DB[s], wk);  // A_k D
      wk = Mfma4<T>::fma(DB[s], sS[wave][1][(4 * s + lq) * n1 + lr], wk);  // D^T B_k
    }
    W[q] = wk;
    __syncthreads();
  }
  // xi/eta part of the result into sU (u is no longer read)
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) sU[(wave * 4 + q) * P + orow(r) * n1 + lr] = W[q][r];
  __syncthreads();
  // 3. zeta transpose and output: tile t = row j of every plane
  const bool masked_interior = rec[(e * kClasses + kInteriorClass) * kRecInts + 3] & kFlagMaskedInterior;
  const ElemCoef<T> ec = elem_coef(oc, e);
  double dacc = 0.0;  // share of u . y over interior nodes, with dpart
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = wave * 4 + q;
    V acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = Mfma4<T>::fma(DB[s], sT[(4 * s + lq) * P + t * 16 + lr], acc);
    const int j = t, i = lr, cx = node_class(i, N), cy = node_class(j, N);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = orow(r);
      const NodeAddr a = node_addr(rec, e, cx, cy, k, i, j, N);
      const T ug = (dpart != nullptr || oc.scaled || oc.ke != nullptr) ? u[a.g] : T(0);
      const T v = elem_value(oc, ec, e, NN, k * P + j * n1 + i, acc[r] + sU[k * P + j * n1 + i], ug);
      if (a.flags & kFlagInterior) {
        const T yv = (masked_interior && dir[a.g]) ? T(0) : op_value(oc, v, a.g, ug);
        y[a.g] = yv;
        if (dpart != nullptr) dacc += (double)ug * (double)yv;
      } else {
        w[a.w] = v;
      }
    }
  }
  if (dpart != nullptr) {
    __syncthreads();  // sS is reused for the reduction (FP64: 2 x 80 KB fills the CU's LDS exactly)
    const double tsum = group_sum<256>(dacc, reinterpret_cast<double*>(&sS[0][0][0]));
    if (tid == 0) dpart[blockIdx.x] = tsum;
  }
}

// ---------------------------------------------------------------------------
// Gather of the shared nodes (eq. (gather)): one lane per shared global node,
// copies summed in ascending element order, Dirichlet nodes zeroed.  As the
// operator's last step (oc.scaled) it also applies kappa and the mass term at
// the shared nodes of u; as the preconditioner's assembly it only sums.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
gs_kernel(T* __restrict__ y, const T* __restrict__ w, const int32_t* __restrict__ vinc_off,
          const int32_t* __restrict__ einc_off, const uint8_t* __restrict__ fcount,
          const uint8_t* __restrict__ dir, int64_t V, int64_t base_f, int64_t base_i, int m,
          int64_t wedge_off, int64_t wvert_off, const T* __restrict__ pd, double* __restrict__ dpart,
          OpCoef<T> oc, const T* __restrict__ u) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0;
  if (g < base_i) {
    // every load of the node issued before any is used (node ids fit in 32 bits)
    const uint8_t dg = dir[g];
    const T pg = dpart != nullptr ? pd[g] : T(0);
    T s = 0;
    if (g >= base_f) {  // face node (most shared nodes): both slots read, the second kept on interior faces
      const uint32_t mm = (uint32_t)m * (uint32_t)m, q = (uint32_t)(g - base_f), f = q / mm, r = q - f * mm;
      const T s0 = w[2 * (int64_t)f * mm + r], s1 = w[(2 * (int64_t)f + 1) * mm + r];
      s = fcount[f] == 2 ? s0 + s1 : s0;
    } else if (g < V) {
      for (int32_t q = vinc_off[g]; q < vinc_off[g + 1]; ++q) s += w[wvert_off + q];
    } else {
      const uint32_t q = (uint32_t)(g - V), ed = q / (uint32_t)m, r = q - ed * (uint32_t)m;
      for (int32_t x = einc_off[ed]; x < einc_off[ed + 1]; ++x) s += w[wedge_off + (int64_t)x * m + r];
    }
    const T yv = dg ? T(0) : op_value(oc, s, g, oc.scaled ? u[g] : T(0));
    y[g] = yv;
    if (dpart != nullptr) d = (double)pg * (double)yv;
  }
  // with dpart: this workgroup's share of pd . y over the shared nodes
  if (dpart != nullptr) {
    __shared__ double red[256 / 64];
    const double t = group_sum<256>(d, red);
    if (threadIdx.x == 0) dpart[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Fine patch solve, eq. (z), one workgroup per subdomain.  The (N+3)^3 patch
// is gathered through I^p into LDS; each of the six 1D contractions is done
// by lanes that own a whole pencil in registers (one LDS read and one write
// per node and pass); the diagonal scaling 1/(kappa 4 (lambda_a/h_x^2 +
// lambda_b/h_y^2 + lambda_c/h_z^2) + c) is fused into the zeta pass.  The
// correction at the element's own nodes goes to zc; the slots outside the
// element go to the consumer layout of the element that holds them (zx).
// ---------------------------------------------------------------------------
// Patches per workgroup: each patch has m^2 pencils (m = N + 3), one per
// lane in each pass; several patches share a workgroup so that the lanes in use
// come close to a multiple of 64 (N = 7: 5 x 100 of 512), within ~64 KB of LDS
// in FP64.
template <int N>
constexpr int fdm_ppb() {
  return N == 2 ? 5 : N == 3 ? 7 : N == 4 ? 5 : N == 6 ? 3 : N == 7 ? 5 : N == 9 ? 3 : N == 10 ? 3 : N == 11 ? 2 : 1;
}

template <int N>
constexpr int fdm_threads() {
  return ((fdm_ppb<N>() * (N + 3) * (N + 3) + 63) / 64) * 64;
}

// One 1D pass of the fast diagonalisation on a lane's pencil.  The extended
// pencil is symmetric under a -> m-1-a, so every column of S is even or odd:
// with ho = m/2 pairs (a, m-1-a) and he = m - ho even columns, the pencil's
// transform takes the pair sums x_a + x_{m-1-a} against the even columns and
// the differences against the odd ones (about half the products of a full
// m x m pass).  Transformed coefficients sit in the order (even columns
// ascending, odd columns ascending).  Sp holds, for a < ho, row a as
// S[a][even j] (j < he) then S[a][odd j] (j < ho), and for odd m the middle
// row S[ho][even j]; rows are read with wave-uniform addresses (scalar loads
// feeding the FMAs) in a rolled loop, so S is not hoisted into registers.
//   pencil_St: out = S^T x     (x in LDS, stride apart)
//   pencil_S:  y = scale S v    (y in LDS)
template <int m, typename T>
__device__ __forceinline__ void pencil_St(const T* __restrict__ Sp, const T* x, int stride, T (&out)[m]) {
  constexpr int ho = m / 2, he = m - ho;
#pragma unroll
  for (int b = 0; b < m; ++b) out[b] = T(0);
#pragma unroll 1
  for (int a = 0; a < ho; ++a) {
    const T xl = x[a * stride], xr = x[(m - 1 - a) * stride];
    const T ps = xl + xr, ms = xl - xr;
    const T* sr = Sp + a * m;
#pragma unroll
    for (int j = 0; j < he; ++j) out[j] += sr[j] * ps;
#pragma unroll
    for (int j = 0; j < ho; ++j) out[he + j] += sr[he + j] * ms;
  }
  if constexpr (m % 2 == 1) {
    const T xc = x[ho * stride];
    const T* sr = Sp + ho * m;
#pragma unroll
    for (int j = 0; j < he; ++j) out[j] += sr[j] * xc;
  }
}

template <int m, typename T>
__device__ __forceinline__ void pencil_S(const T* __restrict__ Sp, const T (&v)[m], T* y, int stride, T scale) {
  constexpr int ho = m / 2, he = m - ho;
#pragma unroll 1
  for (int a = 0; a < ho; ++a) {
    const T* sr = Sp + a * m;
    T ev = T(0), od = T(0);
#pragma unroll
    for (int j = 0; j < he; ++j) ev += sr[j] * v[j];
#pragma unroll
    for (int j = 0; j < ho; ++j) od += sr[he + j] * v[he + j];
    y[a * stride] = (ev + od) * scale;
    y[(m - 1 - a) * stride] = (ev - od) * scale;
  }
  if constexpr (m % 2 == 1) {
    const T* sr = Sp + ho * m;
    T ev = T(0);
#pragma unroll
    for (int j = 0; j < he; ++j) ev += sr[j] * v[j];
    y[ho * stride] = ev * scale;
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(fdm_threads<N>()) __attribute__((amdgpu_waves_per_eu(N <= 8 ? 8 : 4, 8)))
fdm_kernel(const T* __restrict__ r, T* __restrict__ zc, T* __restrict__ zx, const int32_t* __restrict__ ip,
           const int32_t* __restrict__ xdest, const T* __restrict__ S,
           const T* __restrict__ lam, const T* __restrict__ hg, const int32_t* __restrict__ order, int64_t E,
           T kap, T cm, const T* __restrict__ ke, const T* __restrict__ ce) {
  constexpr int m = N + 3, MM = m * m, MMM = MM * m, PPB = fdm_ppb<N>(), NT = fdm_threads<N>();
  constexpr int NN = (N + 1) * (N + 1) * (N + 1), NX = MMM - NN, R = (PPB * MMM + NT - 1) / NT;
  __shared__ T X[PPB * MMM];
  __shared__ T sL[m];
  __shared__ int64_t sE[PPB];  // element of each patch slot, -1 past the end
  const int tid = threadIdx.x;
  const int64_t pos0 = xcd_position(blockIdx.x, (E + PPB - 1) / PPB) * PPB;
  if (pos0 >= E) return;  // whole workgroup
  if (tid < PPB) sE[tid] = pos0 + tid < E ? (int64_t)order[pos0 + tid] : -1;
  if (tid < m) sL[tid] = lam[tid];
  __syncthreads();
  {
    // all index loads, then all residual loads, then the LDS stores
    int32_t gi[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int x = tid + q * NT, lp = min(x / MMM, PPB - 1);
      const int64_t e = x < PPB * MMM ? sE[lp] : -1;
      gi[q] = e >= 0 ? ip[e * MMM + (x - lp * MMM)] : -1;
    }
    T rv[R];
#pragma unroll
    for (int q = 0; q < R; ++q) rv[q] = r[gi[q] >= 0 ? gi[q] : 0];
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (tid + q * NT < PPB * MMM) X[tid + q * NT] = gi[q] >= 0 ? rv[q] : T(0);
  }
  __syncthreads();
  const bool act = tid < PPB * MM;
  const int lp = act ? tid / MM : 0, pl = tid - lp * MM;
  const int p0 = pl % m, p1 = pl / m;
  const int64_t e = act && sE[lp] >= 0 ? sE[lp] : 0;  // slots past the end run on zeros
  T* Xp = X + lp * MMM;
  T v[m], o[m];
  // pass 1: xi, S^T   (lane owns row (b = p0, c = p1))
  if (act) {
    T* row = Xp + p1 * MM + p0 * m;
    pencil_St<m, T>(S, row, 1, o);
#pragma unroll
    for (int a = 0; a < m; ++a) row[a] = o[a];
  }
  __syncthreads();
  // pass 2: eta, S^T  (lane owns column (a = p0, c = p1))
  if (act) {
    T* col = Xp + p1 * MM + p0;
    pencil_St<m, T>(S, col, m, o);
#pragma unroll
    for (int b = 0; b < m; ++b) col[b * m] = o[b];
  }
  __syncthreads();
  // pass 3: zeta, S^T, diagonal, S  (lane owns pencil (a = p0, b = p1))
  if (act) {
    const T hx = hg[e * 3 + 0], hy = hg[e * 3 + 1], hz = hg[e * 3 + 2];
    const T ihx2 = T(4) / (hx * hx), ihy2 = T(4) / (hy * hy), ihz2 = T(4) / (hz * hz);
    T kp = kap, c0 = cm;
    if (ke != nullptr) {  // the subdomain's own element's coefficients
      kp = ke[e];
      c0 = ce[e];
    }
    T* pen = Xp + p1 * m + p0;
    const T dab = sL[p0] * ihx2 + sL[p1] * ihy2;
    pencil_St<m, T>(S, pen, MM, o);
#pragma unroll
    for (int c = 0; c < m; ++c) o[c] = o[c] * recip_pos(kp * (dab + sL[c] * ihz2) + c0);
    pencil_S<m, T>(S, o, pen, MM, T(1));
  }
  __syncthreads();
  // pass 4: eta, S
  if (act) {
    T* col = Xp + p1 * MM + p0;
#pragma unroll
    for (int b = 0; b < m; ++b) v[b] = col[b * m];
    pencil_S<m, T>(S, v, col, m, T(1));
  }
  __syncthreads();
  // pass 5: xi, S, and the volume factor 8/(hx hy hz)
  if (act) {
    T* row = Xp + p1 * MM + p0 * m;
    const T vscale = T(8) / (hg[e * 3 + 0] * hg[e * 3 + 1] * hg[e * 3 + 2]);
#pragma unroll
    for (int a = 0; a < m; ++a) v[a] = row[a];
    pencil_S<m, T>(S, v, row, 1, vscale);
  }
  __syncthreads();
  // Results out, driven by the destination: the element's own nodes to zc in
  // element-local order (consecutive lanes, consecutive addresses), then the
  // slots outside the element in their ordinal order, grouped by entity (6
  // face planes of (N+1)^2, the lower of the other two axes fastest; 12 edge
  // lines of N+1, edge 4 axis + side_lo + 2 side_hi; 8 corners), so that a
  // wave's stores land in one neighbour's consumer block; xdest is read with
  // consecutive addresses and NULL slots are dropped.
  {
    constexpr int n1 = N + 1, P1 = n1 * n1;
    // the lane's slots are recomputed here rather than kept live (in
    // registers) from the gather through the five passes
    int ts = tid;
    asm volatile("" : "+v"(ts));
    constexpr int RC = (PPB * NN + NT - 1) / NT, RO = (PPB * NX + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      const int x = ts + q * NT;
      if (x >= PPB * NN) break;
      const int lq = x / NN, t = x - lq * NN;
      const int i = t % n1, j = (t / n1) % n1, k = t / P1;
      const int64_t eq = sE[lq];
      if (eq >= 0) zc[eq * NN + t] = X[lq * MMM + (i + 1) + m * (j + 1) + MM * (k + 1)];
    }
    int32_t dq[RO];
#pragma unroll
    for (int q = 0; q < RO; ++q) {
      const int x = ts + q * NT, lq = min(x / NX, PPB - 1);
      dq[q] = (x < PPB * NX && sE[lq] >= 0) ? xdest[sE[lq] * NX + (x - lq * NX)] : -1;
    }
#pragma unroll
    for (int q = 0; q < RO; ++q) {
      if (dq[q] < 0) continue;
      const int x = ts + q * NT, lq = x / NX, o = x - lq * NX;
      int ca, cb, cc;  // slot coordinates (a, b, c)
      if (o < 6 * P1) {
        const int f = o / P1, t = o - f * P1, d = f >> 1, s = (f & 1) ? m - 1 : 0;
        const int u = 1 + t % n1, v = 1 + t / n1;
        ca = d == 0 ? s : u;
        cb = d == 1 ? s : (d == 0 ? u : v);
        cc = d == 2 ? s : v;
      } else if (o < 6 * P1 + 12 * n1) {
        const int y = o - 6 * P1, id = y / n1, ax = id >> 2, t = 1 + y % n1;
        const int slo = (id & 1) ? m - 1 : 0, shi = (id & 2) ? m - 1 : 0;
        ca = ax == 0 ? t : slo;
        cb = ax == 1 ? t : (ax == 0 ? slo : shi);
        cc = ax == 2 ? t : shi;
      } else {
        const int id = o - 6 * P1 - 12 * n1;
        ca = (id & 1) ? m - 1 : 0;
        cb = (id & 2) ? m - 1 : 0;
        cc = (id & 4) ? m - 1 : 0;
      }
      zx[dq[q]] = X[lq * MMM + ca + m * cb + MM * cc];
    }
  }
}

// ---------------------------------------------------------------------------
// Sum of the patch corrections and the coarse interpolation, element by element
// (the preconditioner's result before assembly).  Lane (i, j) of element e
// walks its k-pencil: the patch of e itself (zc) plus the corrections that the
// neighbouring patches left in e's consumer layout (zx: planes one layer in
// from each face, lines one layer in from both faces of each edge, corner
// points), then I Z at the nodes e owns.  Element interiors go straight to z
// (Dirichlet zeroed), shared nodes to the work array for gs_kernel.  With
// dpart, each workgroup also leaves its share of rd . z over the interior
// nodes (the gather adds the shared nodes' share), so that PCG's r . z needs
// no pass of its own.
// ---------------------------------------------------------------------------
template <int N, typename T, int EPB>
__global__ void __launch_bounds__(EPB*(N + 1) * (N + 1))
schwarz_sum_kernel(T* __restrict__ z, T* __restrict__ w, const T* __restrict__ zc, const T* __restrict__ zx,
                   const int32_t* __restrict__ rec, const uint8_t* __restrict__ dir,
                   const int32_t* __restrict__ order, int64_t E, int use_fine, const double* __restrict__ Zv,
                   const double* __restrict__ phi, const T* __restrict__ rd, double* __restrict__ dpart) {
  constexpr int n1 = N + 1, P = n1 * n1, NN = P * n1;
  constexpr int NX = (N + 3) * (N + 3) * (N + 3) - NN;
  constexpr int F0 = 0, E0 = 6 * P, C0 = 6 * P + 12 * n1;
  constexpr int RX = (NX + P - 1) / P;
  __shared__ T sX[EPB][NX];  // the element's consumer layout, staged with coalesced loads
  __shared__ double sPhi[2 * n1];
  __shared__ double sRed[EPB * P];
  const int tid = threadIdx.x;
  const int le = tid / P, ij = tid - le * P;
  const int i = ij % n1, j = ij / n1;
  const int64_t pos = xcd_position(blockIdx.x, (E + EPB - 1) / EPB) * EPB + le;
  const bool valid = pos < E;
  const int64_t e = valid ? order[pos] : 0;
  const int cx = node_class(i, N), cy = node_class(j, N);
  const int4* rp = reinterpret_cast<const int4*>(rec) + e * kClasses + cx + 3 * cy;
  const int4 r0 = rp[0], r1 = rp[9], r2 = rp[18];
  const bool masked_interior = rec[(e * kClasses + kInteriorClass) * kRecInts + 3] & kFlagMaskedInterior;
  T cv[n1];
  if (use_fine) {
    const T* ze = zc + e * NN;
    const T* xe = zx + e * NX;
    T xv[RX];
#pragma unroll
    for (int q = 0; q < RX; ++q) xv[q] = (ij + q * P < NX) ? xe[ij + q * P] : T(0);
#pragma unroll
    for (int k = 0; k < n1; ++k) cv[k] = ze[ij + P * k];
#pragma unroll
    for (int q = 0; q < RX; ++q)
      if (ij + q * P < NX) sX[le][ij + q * P] = xv[q];
  }
  // with dpart: rd at the lane's interior nodes (1 <= k < N), loaded ahead of
  // the sum so that the loop's loads do not wait one by one
  const bool int_ij = (r1.w & kFlagInterior) != 0;
  T rdk[n1];
  if (dpart != nullptr && valid && int_ij) {
    int ai, aj, ak;
    unpack_coef(r1.y, ai, aj, ak);
#pragma unroll
    for (int k = 1; k < N; ++k) rdk[k] = rd[r1.x + ai * i + aj * j + ak * k];
  }
  double zv[8];
  if (Zv != nullptr) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cls = 2 * (c & 1) + 6 * ((c >> 1) & 1) + 18 * (c >> 2);
      zv[c] = Zv[rec[(e * kClasses + cls) * kRecInts]];
    }
    for (int x = tid; x < 2 * n1; x += EPB * P) sPhi[x] = phi[x];
  }
  __syncthreads();
  // I Z at (i, j, k) = Phi_0(t_k) zk0 + Phi_1(t_k) zk1, with zk0 / zk1 the
  // bilinear interpolation in (i, j) of the vertex values on the faces k = 0 / N
  double zk0 = 0.0, zk1 = 0.0;
  if (Zv != nullptr) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double wij = sPhi[(c & 1) * n1 + i] * sPhi[(c >> 1) * n1 + j];
      zk0 += wij * zv[c];
      zk1 += wij * zv[c + 4];
    }
  }
  const T* xs = sX[le];
  const bool li0 = i == 1, li1 = i == N - 1, lj0 = j == 1, lj1 = j == N - 1;
  double dacc = 0.0;  // with dpart: this workgroup's share of rd . z over the interior nodes
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    if (!valid) break;
    const bool lk0 = k == 1, lk1 = k == N - 1;
    T v = 0;
    if (use_fine) {
      v = cv[k];
      if (li0) v += xs[F0 + 0 * P + j + n1 * k];
      if (li1) v += xs[F0 + 1 * P + j + n1 * k];
      if (lj0) v += xs[F0 + 2 * P + i + n1 * k];
      if (lj1) v += xs[F0 + 3 * P + i + n1 * k];
      if (lk0) v += xs[F0 + 4 * P + i + n1 * j];
      if (lk1) v += xs[F0 + 5 * P + i + n1 * j];
      // edge lines along x (sides of y, z), along y (sides of x, z), along z (sides of x, y)
      if (lj0 && lk0) v += xs[E0 + (0 + 0 + 0) * n1 + i];
      if (lj1 && lk0) v += xs[E0 + (0 + 1 + 0) * n1 + i];
      if (lj0 && lk1) v += xs[E0 + (0 + 0 + 2) * n1 + i];
      if (lj1 && lk1) v += xs[E0 + (0 + 1 + 2) * n1 + i];
      if (li0 && lk0) v += xs[E0 + (4 + 0 + 0) * n1 + j];
      if (li1 && lk0) v += xs[E0 + (4 + 1 + 0) * n1 + j];
      if (li0 && lk1) v += xs[E0 + (4 + 0 + 2) * n1 + j];
      if (li1 && lk1) v += xs[E0 + (4 + 1 + 2) * n1 + j];
      if (li0 && lj0) v += xs[E0 + (8 + 0 + 0) * n1 + k];
      if (li1 && lj0) v += xs[E0 + (8 + 1 + 0) * n1 + k];
      if (li0 && lj1) v += xs[E0 + (8 + 0 + 2) * n1 + k];
      if (li1 && lj1) v += xs[E0 + (8 + 1 + 2) * n1 + k];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const bool si = (c & 1) ? li1 : li0, sj = ((c >> 1) & 1) ? lj1 : lj0, sk = (c >> 2) ? lk1 : lk0;
        if (si && sj && sk) v += xs[C0 + c];
      }
    }
    const int4 rr = k == 0 ? r0 : (k == N ? r2 : r1);
    if (Zv != nullptr && (rr.w & kFlagOwned)) v += (T)(sPhi[k] * zk0 + sPhi[n1 + k] * zk1);
    int ai, aj, ak;
    unpack_coef(rr.y, ai, aj, ak);
    const int off = ai * i + aj * j + ak * k;
    if (rr.w & kFlagInterior) {
      const T zv = (masked_interior && dir[rr.x + off]) ? T(0) : v;
      z[rr.x + off] = zv;
      if (dpart != nullptr && k > 0 && k < N) dacc += (double)rdk[k] * (double)zv;
    } else {
      w[rr.z + off] = v;
    }
  }
  if (dpart != nullptr) {
    const double t = group_sum<EPB * P>(dacc, sRed);
    if (tid == 0) dpart[blockIdx.x] = t;
  }
}

// Coarse restriction, per element: R_e[IJK] = sum over the nodes this element
// owns of Phi_I(t_i) Phi_J(t_j) Phi_K(t_k) r_N  (= (I^T r) once gathered).
template <int N, typename T>
__global__ void __launch_bounds__((N + 1) * (N + 1))
restrict_kernel(const T* __restrict__ r, double* __restrict__ Re, const int32_t* __restrict__ rec,
                const double* __restrict__ phi, const int32_t* __restrict__ order, int64_t E) {
  constexpr int n1 = N + 1, P = n1 * n1;
  __shared__ double red[8][P + 1];  // padded: the eight summing lanes read eight distinct banks
  __shared__ double sPhi[2 * n1];
  const int tid = threadIdx.x;
  const int i = tid % n1, j = tid / n1;
  const int64_t pos = xcd_position(blockIdx.x, E);
  if (pos >= E) return;  // whole workgroup
  for (int x = tid; x < 2 * n1; x += P) sPhi[x] = phi[x];
  const int64_t e = order[pos];
  const int cx = node_class(i, N), cy = node_class(j, N);
  // the three records of the lane's k-pencil, then all its residual values
  const int4* rp = reinterpret_cast<const int4*>(rec) + e * kClasses + cx + 3 * cy;
  const int4 r0 = rp[0], r1 = rp[9], r2 = rp[18];
  T rv[n1];  // loaded only where the element owns the node (each global node once)
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    const int4 rr = k == 0 ? r0 : (k == N ? r2 : r1);
    int ai, aj, ak;
    unpack_coef(rr.y, ai, aj, ak);
    rv[k] = (rr.w & kFlagOwned) ? r[rr.x + ai * i + aj * j + ak * k] : T(0);
  }
  __syncthreads();
  // the lane's share of corner c: Phi_ci(t_i) Phi_cj(t_j) sum_k Phi_ck(t_k) r_k
  double sk0 = 0.0, sk1 = 0.0;
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    const int4 rr = k == 0 ? r0 : (k == N ? r2 : r1);
    if (rr.w & kFlagOwned) {
      const double v = (double)rv[k];
      sk0 += sPhi[k] * v;
      sk1 += sPhi[n1 + k] * v;
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c)
    red[c][tid] = sPhi[(c & 1) * n1 + i] * sPhi[((c >> 1) & 1) * n1 + j] * ((c >> 2) ? sk1 : sk0);
  __syncthreads();
  if (tid < 8) {
    // four interleaved partial sums, combined in a fixed order
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int x = 0;
    for (; x + 3 < P; x += 4) {
      s0 += red[tid][x];
      s1 += red[tid][x + 1];
      s2 += red[tid][x + 2];
      s3 += red[tid][x + 3];
    }
    for (; x < P; ++x) s0 += red[tid][x];
    Re[e * 8 + tid] = (s0 + s1) + (s2 + s3);
  }
}

// r -= alpha w at the nodes each element owns (each global node once), with
// the element's part of the coarse restriction of the updated r (as
// restrict_kernel: Re[e][IJK] = sum over the owned nodes of
// Phi_I(t_i) Phi_J(t_j) Phi_K(t_k) r_N) and of r . r (dpart[block], 0 for
// the padding blocks).  Lets the coarse chain start right after the update
// of r, before the patch solves.
template <int N, typename T>
__global__ void __launch_bounds__((N + 1) * (N + 1))
update_r_restrict_kernel(T* __restrict__ r, const T* __restrict__ w, const double* __restrict__ sc,
                         double* __restrict__ Re, double* __restrict__ dpart, const int32_t* __restrict__ rec,
                         const double* __restrict__ phi, const int32_t* __restrict__ order, int64_t E) {
  constexpr int n1 = N + 1, P = n1 * n1;
  __shared__ double red[9][P + 1];  // padded rows: the summing lanes read distinct banks
  __shared__ double sPhi[2 * n1];
  const int tid = threadIdx.x;
  const int i = tid % n1, j = tid / n1;
  const int64_t pos = xcd_position(blockIdx.x, E);
  const bool valid = pos < E;
  const int64_t e = valid ? order[pos] : 0;
  for (int x = tid; x < 2 * n1; x += P) sPhi[x] = phi[x];
  const int cx = node_class(i, N), cy = node_class(j, N);
  const int4* rp = reinterpret_cast<const int4*>(rec) + e * kClasses + cx + 3 * cy;
  const int4 r0 = rp[0], r1 = rp[9], r2 = rp[18];
  const T al = (T)sc[2];
  T rv[n1], wv[n1];
  int32_t gk[n1];  // global node ids fit in 32 bits
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    const int4 rr = k == 0 ? r0 : (k == N ? r2 : r1);
    int ai, aj, ak;
    unpack_coef(rr.y, ai, aj, ak);
    const bool own = valid && (rr.w & kFlagOwned);
    gk[k] = own ? rr.x + ai * i + aj * j + ak * k : -1;
    rv[k] = own ? r[gk[k]] : T(0);
    wv[k] = own ? w[gk[k]] : T(0);
  }
  __syncthreads();
  // restriction as in restrict_kernel: two k-sums per lane, corner weights at the end
  double sk0 = 0.0, sk1 = 0.0, rsq = 0.0;
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    if (gk[k] < 0) continue;
    const T rn = rv[k] - al * wv[k];
    r[gk[k]] = rn;
    const double v = (double)rn;
    rsq += v * v;
    sk0 += sPhi[k] * v;
    sk1 += sPhi[n1 + k] * v;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c)
    red[c][tid] = sPhi[(c & 1) * n1 + i] * sPhi[((c >> 1) & 1) * n1 + j] * ((c >> 2) ? sk1 : sk0);
  red[8][tid] = rsq;
  __syncthreads();
  if (tid < 9) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int x = 0;
    for (; x + 3 < P; x += 4) {
      s0 += red[tid][x];
      s1 += red[tid][x + 1];
      s2 += red[tid][x + 2];
      s3 += red[tid][x + 3];
    }
    for (; x < P; ++x) s0 += red[tid][x];
    const double t = (s0 + s1) + (s2 + s3);
    if (tid == 8)
      dpart[blockIdx.x] = t;
    else if (valid)
      Re[e * 8 + tid] = t;
  }
}

// coarse residual on the free vertices (coarse order): sum of the element parts
__global__ void __launch_bounds__(256)
restrict_gather_kernel(double* __restrict__ R, const double* __restrict__ Re, const int32_t* __restrict__ vinc_off,
                       const int32_t* __restrict__ vinc_ec, const int32_t* __restrict__ cidx, int64_t V) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int32_t c = cidx[v];
  if (c < 0) return;
  // four incidences in flight at a time; the sum still runs in list order
  const int32_t q1 = vinc_off[v + 1];
  int32_t q = vinc_off[v];
  double s = 0.0;
  for (; q + 4 <= q1; q += 4) {
    const int32_t a0 = vinc_ec[q], a1 = vinc_ec[q + 1], a2 = vinc_ec[q + 2], a3 = vinc_ec[q + 3];
    const double b0 = Re[a0], b1 = Re[a1], b2 = Re[a2], b3 = Re[a3];
    s += b0;
    s += b1;
    s += b2;
    s += b3;
  }
  for (; q < q1; ++q) s += Re[vinc_ec[q]];
  R[c] = s;
}

// Nested-dissection solve of the coarse system, node by node in height order.
//   forward, height h (leaves first), node t with own rows I and boundary B:
//     y_I = R_I - (contributions W_d y_d of the descendants d with I in B_d)
//     Z_I = S_t^-1 y_I,   c_t = W_t y_I        (one stacked product [S^-1; W] y)
//   backward, height h (roots first):
//     X_I = Z_I - W_t^T X_B
// All rows are independent within a height; sums run in a fixed order.

// y_i = R_i - sum of the contributions listed for row i: 8 lanes per row,
// lane t taking every 8th entry from t, then a fixed shuffle tree
__global__ void __launch_bounds__(256)
coarse_assemble_kernel(double* __restrict__ Y, const double* __restrict__ R, const double* __restrict__ cvec,
                       const int32_t* __restrict__ ct_off, const int32_t* __restrict__ ct_pos,
                       const int32_t* __restrict__ items, int64_t n) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t x = gid >> 3;
  const int sub = (int)(gid & 7);
  if (x >= n) return;  // whole 8-lane groups leave together
  const int32_t i = items[x];
  double s = 0.0;
  for (int32_t q = ct_off[i] + sub; q < ct_off[i + 1]; q += 8) s += cvec[ct_pos[q]];
  s += __shfl_xor(s, 4, 8);
  s += __shfl_xor(s, 2, 8);
  s += __shfl_xor(s, 1, 8);
  if (sub == 0) Y[i] = R[i] - s;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Tiled sweeps: one workgroup (4 waves) per tile of rows of one node.  Not
// split: a tile of 4 RW consecutive rows, wave w taking rows r + w RW ..
// r + w RW + RW - 1, each lane its columns c = lane + 64 j.  Split (rows
// longer than 1024): a tile of RW rows shared by the 4 waves, wave w taking
// the column blocks c = 64 w + lane + 256 j, the 4 partial sums of a row
// added in wave order through LDS.  The vector the rows are dotted with (y_I
// forward, x_B backward) passes through LDS in chunks of kCoarseStage entries
// (a multiple of 256), each staged once per tile; sums run in ascending c
// within a lane, then a wave sum per row.
constexpr int kCoarseStage = 1024;

// the wave's RW dot products against the staged vector; returns them summed over the wave (lane 0 holds them)
template <int RW, bool SPLIT>
__device__ __forceinline__ void coarse_tile_dots(const double* const (&rp)[RW], double (&acc)[RW], int len,
                                                 const double* __restrict__ stage_src,
                                                 const int32_t* __restrict__ gather_idx, double* sv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cfirst = SPLIT ? 64 * wave + lane : lane, cstep = SPLIT ? 256 : 64;
  for (int c0 = 0; c0 < len; c0 += kCoarseStage) {
    const int cn = min(kCoarseStage, len - c0);
    __syncthreads();  // the previous chunk is consumed
    for (int c = threadIdx.x; c < cn; c += 256)
      sv[c] = gather_idx != nullptr ? stage_src[gather_idx[c0 + c]] : stage_src[c0 + c];
    __syncthreads();
#pragma unroll 2
    for (int c = cfirst; c < cn; c += cstep) {
      const double vc = sv[c];
#pragma unroll
      for (int i = 0; i < RW; ++i) acc[i] += rp[i][c0 + c] * vc;
    }
  }
}

// row sums of a tile: not split, each wave's own rows; split, the 4 waves'
// partial sums of the shared rows in wave order (thread 0 holds them)
template <int RW, bool SPLIT>
__device__ __forceinline__ void coarse_tile_reduce(double (&acc)[RW], double (*sp)[RW]) {
#pragma unroll
  for (int i = 0; i < RW; ++i) acc[i] = wave_sum(acc[i]);
  if constexpr (SPLIT) {
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int i = 0; i < RW; ++i) sp[threadIdx.x >> 6][i] = acc[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
      for (int i = 0; i < RW; ++i) acc[i] = ((sp[0][i] + sp[1][i]) + sp[2][i]) + sp[3][i];
  }
}

// forward, large nodes: rows of [S^-1; W] (row-major, s columns); rows < s
// give Z, the others the node's contribution
template <int RW, bool SPLIT>
__global__ void __launch_bounds__(256)
coarse_fwd_kernel(double* __restrict__ Z, double* __restrict__ cvec, const double* __restrict__ Y,
                  const double* __restrict__ pool, const FrontNode* __restrict__ nodes,
                  const RowItem* __restrict__ tiles) {
  __shared__ double sv[kCoarseStage];
  __shared__ double sp[4][RW];
  const RowItem ti = tiles[blockIdx.x];
  const FrontNode nd = nodes[ti.node];
  const int s = nd.s, f = nd.s + nd.b;
  const int r0 = SPLIT ? ti.row : ti.row + (threadIdx.x >> 6) * RW;
  const double* rp[RW];
  double acc[RW];
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    rp[i] = pool + nd.fwd + (int64_t)min(r0 + i, f - 1) * s;  // rows past the node: read, not stored
    acc[i] = 0.0;
  }
  coarse_tile_dots<RW, SPLIT>(rp, acc, s, Y + nd.off, nullptr, sv);
  coarse_tile_reduce<RW, SPLIT>(acc, sp);
  if (SPLIT ? threadIdx.x == 0 : (threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < RW; ++i) {
      const int r = r0 + i;
      if (r >= f) break;
      if (r < s)
        Z[nd.off + r] = acc[i];
      else
        cvec[nd.coff + r - s] = acc[i];
    }
}

// value of v held by lane l (l wave-uniform)
__device__ __forceinline__ double lane_value(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l), hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// small nodes (s <= 128): one lane per row of [S^-1; W] (column-major,
// leading dimension s + b), 64-row chunks; y sits in two registers per lane
// and is broadcast with readlane; matrix loads go out eight at a time.  Each
// wave assembles the node's y itself (lane i: y_i = R_i minus the listed
// contributions of the descendants, in list order), so heights with only
// small nodes need no assembly launch.
__global__ void __launch_bounds__(256)
coarse_fwd_small_kernel(double* __restrict__ Z, double* __restrict__ cvec, const double* __restrict__ R,
                        const int32_t* __restrict__ ct_off, const int32_t* __restrict__ ct_pos,
                        const double* __restrict__ pool, const FrontNode* __restrict__ nodes,
                        const RowItem* __restrict__ items, int64_t n) {
  const int64_t it = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  const int lane = threadIdx.x & 63;
  if (it >= n) return;  // whole wave
  const RowItem ri = items[it];
  const FrontNode nd = nodes[ri.node];
  const int f = nd.s + nd.b, s = nd.s;
  const int rho = ri.row * 64 + lane;
  const int rr = rho < f ? rho : f - 1;
  const double* M = pool + nd.fwd + rr;
  auto y_row = [&](int64_t g) {  // assembled y of coarse row g (contributions written by earlier launches)
    double a = 0.0;
    for (int32_t q = ct_off[g]; q < ct_off[g + 1]; ++q) a += cvec[ct_pos[q]];
    return R[g] - a;
  };
  const double y0 = lane < s ? y_row(nd.off + lane) : 0.0;
  const double y1 = lane + 64 < s ? y_row(nd.off + lane + 64) : 0.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < s; c0 += 8) {
    double mv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) mv[u] = M[(int64_t)(c0 + u < s ? c0 + u : s - 1) * f];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + u;
      if (c < s) acc[u & 3] += mv[u] * lane_value(c < 64 ? y0 : y1, c & 63);
    }
  }
  const double v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  if (rho < s)
    Z[nd.off + rho] = v;
  else if (rho < f)
    cvec[nd.coff + rho - s] = v;
}

// backward: rows of W^T (row-major, b columns), one per own column c of a
// node: X_c = Z_c - (W^T)_c . X_B (X_B final from the ancestors' launches)
template <int RW, bool SPLIT>
__global__ void __launch_bounds__(256)
coarse_bwd_kernel(double* __restrict__ X, const double* __restrict__ Z, const double* __restrict__ pool,
                  const int32_t* __restrict__ fb_idx, const FrontNode* __restrict__ nodes,
                  const RowItem* __restrict__ tiles) {
  __shared__ double sv[kCoarseStage];
  __shared__ double sp[4][RW];
  const RowItem ti = tiles[blockIdx.x];
  const FrontNode nd = nodes[ti.node];
  const int s = nd.s, b = nd.b;
  const int r0 = SPLIT ? ti.row : ti.row + (threadIdx.x >> 6) * RW;
  const double* rp[RW];
  double acc[RW];
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    rp[i] = pool + nd.bwd + (int64_t)min(r0 + i, s - 1) * b;
    acc[i] = 0.0;
  }
  coarse_tile_dots<RW, SPLIT>(rp, acc, b, X, fb_idx + nd.bidx, sv);
  coarse_tile_reduce<RW, SPLIT>(acc, sp);
  if (SPLIT ? threadIdx.x == 0 : (threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < RW; ++i) {
      const int r = r0 + i;
      if (r >= s) break;
      X[nd.off + r] = Z[nd.off + r] - acc[i];
    }
}

// ---------------------------------------------------------------------------
// Aggregation AMG with a K-cycle on the coarse system (Section 4.1, "Algebraic
// multigrid"): CSR matrices per level (columns ascending), damped Jacobi with
// wd = omega / a_ii, restriction by aggregate sums (members ascending),
// prolongation by injection.  All scalars of the flexible-CG steps stay on the
// device, so a whole cycle can be captured in a graph.
// ---------------------------------------------------------------------------
// Jacobi sweep from zero and its residual in one pass: x = wd .* b,
// r = b - A x (x at the neighbours formed on the fly)
__global__ void __launch_bounds__(256)
amg_presmooth_kernel(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ b,
                     const double* __restrict__ wd, const int32_t* __restrict__ off, const int32_t* __restrict__ col,
                     const double* __restrict__ val, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int32_t q = off[i]; q < off[i + 1]; ++q) {
    const int32_t j = col[q];
    acc += val[q] * (wd[j] * b[j]);
  }
  x[i] = wd[i] * b[i];
  r[i] = b[i] - acc;
}

// w = A v
__global__ void __launch_bounds__(256)
amg_spmv_kernel(double* __restrict__ w, const double* __restrict__ v, const int32_t* __restrict__ off,
                const int32_t* __restrict__ col, const double* __restrict__ val, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int32_t q = off[i]; q < off[i + 1]; ++q) acc += val[q] * v[col[q]];
  w[i] = acc;
}

// B[a] = sum of r over the members of aggregate a
__global__ void __launch_bounds__(256)
amg_restrict_kernel(double* __restrict__ B, const double* __restrict__ r, const int32_t* __restrict__ moff,
                    const int32_t* __restrict__ mem, int64_t nc) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nc) return;
  double acc = 0.0;
  for (int32_t q = moff[a]; q < moff[a + 1]; ++q) acc += r[mem[q]];
  B[a] = acc;
}

// t = x + X[agg]  (coarse correction by injection)
__global__ void __launch_bounds__(256)
amg_prolong_kernel(double* __restrict__ t, const double* __restrict__ x, const double* __restrict__ X,
                   const int32_t* __restrict__ agg, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = x[i] + X[agg[i]];
}

// x = t + wd .* (b - A t)  (Jacobi sweep after the coarse correction)
__global__ void __launch_bounds__(256)
amg_post_kernel(double* __restrict__ x, const double* __restrict__ t, const double* __restrict__ b,
                const int32_t* __restrict__ off, const int32_t* __restrict__ col, const double* __restrict__ val,
                const double* __restrict__ wd, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int32_t q = off[i]; q < off[i + 1]; ++q) acc += val[q] * t[col[q]];
  x[i] = t[i] + wd[i] * (b[i] - acc);
}

// sc[idx + k] = a . b_k over n entries for the K vectors b_0..b_{K-1} (K <= 3),
// one workgroup, fixed summation order
template <int K>
__global__ void __launch_bounds__(1024)
amg_dots_kernel(double* __restrict__ sc, int idx, const double* __restrict__ a, const double* __restrict__ b0,
                const double* __restrict__ b1, const double* __restrict__ b2, int64_t n) {
  __shared__ double red[1024 / 64];
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double ai = a[i];
    acc[0] += ai * b0[i];
    if constexpr (K > 1) acc[1] += ai * b1[i];
    if constexpr (K > 2) acc[2] += ai * b2[i];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double t = group_sum<1024>(acc[k], red);
    if (threadIdx.x == 0) sc[idx + k] = t;
    __syncthreads();  // red is reused by the next sum
  }
}

// r2 = b - (rho / a1) w   with sc = {rho, a1, ...}
__global__ void __launch_bounds__(256)
amg_r2_kernel(double* __restrict__ r2, const double* __restrict__ b, const double* __restrict__ w,
              const double* __restrict__ sc, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r2[i] = b[i] - (sc[0] / sc[1]) * w[i];
}

// two flexible-CG steps combined: x = (rho/a1) v + (a2/den) (v2 - (g/a1) v),
// den = be - g^2/a1, with sc = {rho, a1, g, be, a2}
__global__ void __launch_bounds__(256)
amg_combine_kernel(double* __restrict__ x, const double* __restrict__ v, const double* __restrict__ v2,
                   const double* __restrict__ sc, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double rho = sc[0], a1 = sc[1], g = sc[2], be = sc[3], a2 = sc[4];
  const double den = be - g * g / a1;
  x[i] = (rho / a1) * v[i] + (a2 / den) * (v2[i] - (g / a1) * v[i]);
}

// x = Ainv b, dense row-major n x n; one wave per row
__global__ void __launch_bounds__(256)
amg_gemv_kernel(double* __restrict__ x, const double* __restrict__ Ainv, const double* __restrict__ b, int64_t n) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;  // whole wave
  double acc = 0.0;
  for (int64_t k = lane; k < n; k += 64) acc += Ainv[row * n + k] * b[k];
  acc = wave_sum(acc);
  if (lane == 0) x[row] = acc;
}

// level-0 right-hand side from the coarse residual (nested-dissection order)
__global__ void __launch_bounds__(256)
amg_in_kernel(double* __restrict__ B0, const double* __restrict__ R, const int32_t* __restrict__ nd_of, int64_t n) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) B0[q] = R[nd_of[q]];
}

// vertex-indexed result (0 on Dirichlet vertices) from the level-0 solution
__global__ void __launch_bounds__(256)
amg_out_kernel(double* __restrict__ Zv, const double* __restrict__ X0, const int32_t* __restrict__ cidx,
               const int32_t* __restrict__ pos, int64_t V) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int32_t c = cidx[v];
  Zv[v] = c >= 0 ? X0[pos[c]] : 0.0;
}

// vertex-indexed coarse solution (0 on Dirichlet vertices)
__global__ void __launch_bounds__(256)
coarse_scatter_kernel(double* __restrict__ Zv, const double* __restrict__ X, const int32_t* __restrict__ cidx,
                      int64_t V) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int32_t c = cidx[v];
  Zv[v] = c >= 0 ? X[c] : 0.0;
}

__global__ void __launch_bounds__(256)
coarse_gather_vertex_kernel(double* __restrict__ Rlev, const double* __restrict__ Rv, const int32_t* __restrict__ cidx,
                            int64_t V) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int32_t c = cidx[v];
  if (c >= 0) Rlev[c] = Rv[v];
}

// --- set-up of the coarse fronts (column-major f x f front F, leading dimension f)
// copy the lower triangle of the leading n x n block to the upper one
__global__ void symmetrize_kernel(double* __restrict__ A, int64_t n, int64_t ld) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n * n) return;
  const int64_t r = x % n, c = x / n;
  if (r < c) A[r + c * ld] = A[c + r * ld];
}

// F_IB = F_BI^T: F[c, s + k] = F[s + k, c] for c < s, k < b
__global__ void front_transpose_kernel(double* __restrict__ F, int64_t f, int64_t s, int64_t b) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= s * b) return;
  const int64_t c = x % s, k = x / s;
  F[c + (s + k) * f] = F[(s + k) + c * f];
}

// extend-add of a child's update matrix U (b x b, leading dimension b) into F
__global__ void front_extend_add_kernel(double* __restrict__ F, int64_t f, const double* __restrict__ U, int64_t b,
                                        const int32_t* __restrict__ map) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= b * b) return;
  const int64_t i = x % b, j = x / b;
  F[map[i] + (int64_t)map[j] * f] += U[x];
}

// ---------------------------------------------------------------------------
// PCG vector kernels (Algorithm 1).  Reductions are two-pass with a fixed
// grid and a fixed tree order, so results are reproducible run to run.
// Scalars live on the device: sc[0] = z^T r, sc[1] = p^T w, sc[2] = alpha,
// sc[3] = beta, sc[4] = r^T r, sc[5] = scratch, sc[6] = breakdown flag.
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// two consecutive entries as one 16-byte (double) or 8-byte (float) access
template <typename T>
struct Pair2;
template <>
struct Pair2<double> {
  typedef double2 type;
};
template <>
struct Pair2<float> {
  typedef float2 type;
};


__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += sh[q];
  return s;
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(kRedThreads)
dot_partial_kernel(const TA* __restrict__ a, const TB* __restrict__ b, double* __restrict__ part, int64_t n,
                   int pairs) {
  __shared__ double sh[kRedThreads / 64];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double s = 0.0;
  if (pairs) {
    typedef typename Pair2<TA>::type A2;
    typedef typename Pair2<TB>::type B2;
    const A2* a2 = reinterpret_cast<const A2*>(a);
    const B2* b2 = reinterpret_cast<const B2*>(b);
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n / 2; x += stride) {
      const A2 av = a2[x];
      const B2 bv = b2[x];
      s += (double)av.x * (double)bv.x;
      s += (double)av.y * (double)bv.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) s += (double)a[n - 1] * (double)b[n - 1];
  } else {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride)
      s += (double)a[x] * (double)b[x];
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// mode 0: sc[dst] = sum;  mode 1: alpha = sc[0] / sum (p^T w);  mode 2: beta = sum / sc[0], sc[0] = sum
__global__ void __launch_bounds__(kRedThreads)
dot_final_kernel(const double* __restrict__ part, double* __restrict__ sc, int nparts, int dst, int mode) {
  __shared__ double sh[kRedThreads / 64];
  double s = 0.0;
  for (int x = threadIdx.x; x < nparts; x += blockDim.x) s += part[x];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    sc[dst] = s;
    if (mode == 1) {
      const double a = sc[0] / s;
      if (!(s > 0.0) || !isfinite(a)) sc[6] = 1.0;
      sc[2] = a;
    } else if (mode == 2) {
      const double bta = s / sc[0];
      if (!isfinite(bta)) sc[6] = 1.0;
      sc[3] = bta;
      sc[0] = s;
    }
  }
}

// first stage of a reduction over many partial sums: block b sums the
// partials [b * chunk, (b + 1) * chunk) in a fixed order
__global__ void __launch_bounds__(kRedThreads)
sum_chunks_kernel(const double* __restrict__ in, double* __restrict__ out, int64_t n, int64_t chunk) {
  __shared__ double sh[kRedThreads / 64];
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
  double s = 0.0;
  for (int64_t x = b0 + threadIdx.x; x < b1; x += blockDim.x) s += in[x];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// r -= alpha w; partial sums of r^T r (the matching x update is deferred to
// update_px_kernel, which reads p anyway)
// With `pairs`, entries go two at a time (all pointers 16-byte aligned, a
// single odd tail entry handled by thread 0 of block 0).
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
update_r_kernel(T* __restrict__ r, const T* __restrict__ w, const double* __restrict__ sc, double* __restrict__ part,
                int64_t n, int pairs) {
  __shared__ double sh[kRedThreads / 64];
  typedef typename Pair2<T>::type T2;
  const T al = (T)sc[2];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double s = 0.0;
  if (pairs) {
    T2* r2 = reinterpret_cast<T2*>(r);
    const T2* w2 = reinterpret_cast<const T2*>(w);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n / 2; q += stride) {
      const T2 rv = r2[q], wv = w2[q];
      T2 rn;
      rn.x = rv.x - al * wv.x;
      rn.y = rv.y - al * wv.y;
      r2[q] = rn;
      s += (double)rn.x * (double)rn.x;
      s += (double)rn.y * (double)rn.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
      const T rn = r[n - 1] - al * w[n - 1];
      r[n - 1] = rn;
      s += (double)rn * (double)rn;
    }
  } else {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
      const T rn = r[q] - al * w[q];
      r[q] = rn;
      s += (double)rn * (double)rn;
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x += alpha p (this iteration's alpha); p = z + beta p.  Nothing once the
// breakdown flag is set (x keeps its last finite iterate).
template <typename T>
__global__ void __launch_bounds__(256)
update_px_kernel(T* __restrict__ x, T* __restrict__ p, const T* __restrict__ z, const double* __restrict__ sc,
                 int64_t n, int pairs) {
  if (sc[6] != 0.0) return;  // whole grid
  typedef typename Pair2<T>::type T2;
  const T al = (T)sc[2];
  const T beta = (T)sc[3];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (pairs) {
    T2* x2 = reinterpret_cast<T2*>(x);
    T2* p2 = reinterpret_cast<T2*>(p);
    const T2* z2 = reinterpret_cast<const T2*>(z);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n / 2; q += stride) {
      const T2 pq = p2[q], zq = z2[q];
      T2 xq = x2[q], pn;
      xq.x += al * pq.x;
      xq.y += al * pq.y;
      pn.x = zq.x + beta * pq.x;
      pn.y = zq.y + beta * pq.y;
      x2[q] = xq;
      p2[q] = pn;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
      const T pq = p[n - 1];
      x[n - 1] += al * pq;
      p[n - 1] = z[n - 1] + beta * pq;
    }
  } else {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
      const T pq = p[q];
      x[q] += al * pq;
      p[q] = z[q] + beta * pq;
    }
  }
}

// x += alpha p (the last iteration's deferred update; nothing after a breakdown)
template <typename T>
__global__ void __launch_bounds__(256)
update_x_kernel(T* __restrict__ x, const T* __restrict__ p, const double* __restrict__ sc, int64_t n) {
  if (sc[6] != 0.0) return;  // whole grid
  const T al = (T)sc[2];
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    x[q] += al * p[q];
}

template <typename TD, typename TS>
__global__ void __launch_bounds__(256) copy_kernel(TD* __restrict__ d, const TS* __restrict__ s, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    d[q] = (TD)s[q];
}

// Bandwidth probes (copy, triad, read) over n doubles as double2 pairs with a
// grid-stride loop: the on-device ceiling that the streaming kernels of the
// solver are compared with.  n is even and the pointers are 16-byte aligned.
__global__ void __launch_bounds__(256) stream_copy_kernel(double2* __restrict__ b, const double2* __restrict__ a,
                                                          int64_t n2) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n2; q += (int64_t)gridDim.x * blockDim.x)
    b[q] = a[q];
}

__global__ void __launch_bounds__(256) stream_triad_kernel(double2* __restrict__ c, const double2* __restrict__ a,
                                                           const double2* __restrict__ b, double s, int64_t n2) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n2; q += (int64_t)gridDim.x * blockDim.x) {
    const double2 x = a[q], y = b[q];
    c[q] = make_double2(x.x + s * y.x, x.y + s * y.y);
  }
}

__global__ void __launch_bounds__(256) stream_read_kernel(const double2* __restrict__ a, int64_t n2,
                                                          double* __restrict__ part) {
  double v = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n2; q += (int64_t)gridDim.x * blockDim.x) {
    const double2 x = a[q];
    v += x.x + x.y;
  }
  __shared__ double red[4];
  const double t = group_sum<256>(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Right-hand side of one backward Euler step of the heat equation (Section
// 6.2): b_N = m_N (u_N / dt + q_N) on free nodes, 0 on Dirichlet nodes
// (q = NULL: no source).
__global__ void __launch_bounds__(256)
heat_rhs_kernel(double* __restrict__ b, const double* __restrict__ u, const double* __restrict__ q,
                const double* __restrict__ mN, const uint8_t* __restrict__ dir, double dt, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) b[g] = dir[g] ? 0.0 : mN[g] * (u[g] / dt + (q != nullptr ? q[g] : 0.0));
}

template <typename T>
__global__ void __launch_bounds__(256) fill_kernel(T* __restrict__ d, T v, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    d[q] = v;
}

// r = b - Ax (FP64) on the free nodes, 0 on the Dirichlet set (Ax = NULL:
// r = b there), with partial sums of r^T r
__global__ void __launch_bounds__(kRedThreads)
residual_kernel(double* __restrict__ r, const double* __restrict__ b, const double* __restrict__ Ax,
                const uint8_t* __restrict__ dir, double* __restrict__ part, int64_t n) {
  __shared__ double sh[kRedThreads / 64];
  double s = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const double v = dir[q] ? 0.0 : b[q] - (Ax != nullptr ? Ax[q] : 0.0);
    r[q] = v;
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// f32 = (float)(r64 * scale)
__global__ void __launch_bounds__(256)
scale_to_f32_kernel(float* __restrict__ d, const double* __restrict__ s, double scale, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    d[q] = (float)(s[q] * scale);
}

// x64 += scale * d32
__global__ void __launch_bounds__(256)
axpy_f32_kernel(double* __restrict__ x, const float* __restrict__ d, double scale, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    x[q] += scale * (double)d[q];
}

}  // namespace sem
