// Host-side set-up of the spectral-element discretisation (runs once per mesh).
//
//  * 1D reference data: GLL points and weights, derivative matrix (Section 2.1),
//    extended 1D pencil and its generalised eigenbasis (Section 4.2).
//  * Canonical global numbering as per-element affine "entity records" and
//    the gather structure of eq. (gather) (Section 2.2).
//  * Geometric factors, weighted mass, lumped mass (Sections 2.3-2.4).
//  * Overlapping patch table I^p and its inverse (Section 4.2).
//  * Order-1 coarse matrix on the free vertices with a BFS level ordering that
//    makes it block tridiagonal (Section 4.1).
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>

#include "sem_internal.h"

namespace sem {

namespace {

// run f(begin, end) over [0, n) on the host cores
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::max(1u, std::min(hw, 32u));
  if (n < 4096 || nt == 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back(f, b, e);
  }
  for (auto& x : th) x.join();
}

// Legendre P_{n-1}(x), P_n(x) by the three-term recurrence
void legendre_pair(int n, double x, double& pnm1, double& pn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    pnm1 = 0.0;
    pn = 1.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pnm1 = p0;
  pn = p1;
}

// symmetric eigen-decomposition by cyclic Jacobi rotations: A = Q diag(w) Q^T
void jacobi_eigen(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& Q) {
  Q.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
  // ascending eigenvalues
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a] < w[b]; });
  std::vector<double> w2(n), Q2(n * n);
  for (int c = 0; c < n; ++c) {
    w2[c] = w[ord[c]];
    for (int r = 0; r < n; ++r) Q2[r * n + c] = Q[r * n + ord[c]];
  }
  w = w2;
  Q = Q2;
}

inline int corner_pos(int a, int b, int c) { return a + 2 * b + 4 * c; }

struct EdgeKey {
  int64_t lo, hi;
  int64_t e;
  int le;
};

struct FaceKey {
  int64_t v[4];
  int64_t e;
  int lf;
};

}  // namespace

// ---------------------------------------------------------------------------
// 1D reference data
// ---------------------------------------------------------------------------
void build_reference(HostTables& T, int N) {
  T.N = N;
  T.n1 = N + 1;
  T.np = N + 3;
  const int n1 = N + 1;
  T.t.assign(n1, 0.0);
  T.rho.assign(n1, 0.0);
  T.t[0] = -1.0;
  T.t[N] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int i = 1; i < N; ++i) {
    // Newton on P_N'(x) = 0 from the Chebyshev-Gauss-Lobatto guess; P_N' and
    // P_N'' from the recurrence identity and Legendre's equation.
    double x = -std::cos(pi * i / N);
    for (int it = 0; it < 100; ++it) {
      double pm1, p;
      legendre_pair(N, x, pm1, p);
      double dp = N * (pm1 - x * p) / (1.0 - x * x);
      double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
      double dx = dp / d2p;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    T.t[i] = x;
  }
  std::vector<double> PN(n1);
  for (int i = 0; i < n1; ++i) {
    double pm1, p;
    legendre_pair(N, T.t[i], pm1, p);
    PN[i] = p;
    T.rho[i] = 2.0 / (N * (N + 1.0) * p * p);
  }
  // D[i][j] = phi_j'(t_i), closed form for GLL Lagrange interpolants
  T.D.assign(n1 * n1, 0.0);
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      if (i != j)
        T.D[i * n1 + j] = PN[i] / (PN[j] * (T.t[i] - T.t[j]));
      else if (i == 0)
        T.D[i * n1 + j] = -N * (N + 1.0) / 4.0;
      else if (i == N)
        T.D[i * n1 + j] = N * (N + 1.0) / 4.0;
    }
  // extended pencil (nodes -1..N+1 at positions 0..N+2): element block, plus the
  // neighbours' two nodes nearest each end vertex; d = D^T diag(rho) D
  const int np = N + 3;
  std::vector<double> d(n1 * n1, 0.0);
  for (int a = 0; a < n1; ++a)
    for (int b = 0; b < n1; ++b) {
      double s = 0.0;
      for (int m = 0; m < n1; ++m) s += T.D[m * n1 + a] * T.D[m * n1 + b] * T.rho[m];
      d[a * n1 + b] = s;
    }
  std::vector<double> K(np * np, 0.0), M(np, 0.0);
  for (int a = 0; a < n1; ++a) {
    M[a + 1] += T.rho[a];
    for (int b = 0; b < n1; ++b) K[(a + 1) * np + (b + 1)] += d[a * n1 + b];
  }
  const int L[2] = {N - 1, N};  // left neighbour nodes -> positions 0, 1
  const int R[2] = {0, 1};      // right neighbour nodes -> positions N+1, N+2
  for (int a = 0; a < 2; ++a) {
    M[a] += T.rho[L[a]];
    M[N + 1 + a] += T.rho[R[a]];
    for (int b = 0; b < 2; ++b) {
      K[a * np + b] += d[L[a] * n1 + L[b]];
      K[(N + 1 + a) * np + (N + 1 + b)] += d[R[a] * n1 + R[b]];
    }
  }
  // K S = M S Lambda, S^T M S = I:  C = M^{-1/2} K M^{-1/2} = Q Lambda Q^T, S = M^{-1/2} Q.
  // The pencil is symmetric under the reflection a -> np-1-a (rho and D are), so
  // C splits into blocks on the even vectors (e_a + e_{np-1-a})/sqrt 2 (and the
  // middle e_a when np is odd) and the odd ones (e_a - e_{np-1-a})/sqrt 2: each
  // eigenvector is even or odd, and a 1D pass needs only half of S.  Each block
  // is diagonalised on its own, so that the parity holds exactly.
  std::vector<double> C(np * np);
  for (int a = 0; a < np; ++a)
    for (int b = 0; b < np; ++b) C[a * np + b] = K[a * np + b] / std::sqrt(M[a] * M[b]);
  const int ho = np / 2, he = np - ho;
  const double r2 = 1.0 / std::sqrt(2.0);
  auto half_vec = [&](int a, int sign, std::vector<double>& v) {  // basis vector a of one block
    v.assign(np, 0.0);
    if (a < ho) {
      v[a] = r2;
      v[np - 1 - a] = sign * r2;
    } else {
      v[a] = 1.0;  // the middle node (np odd, even block)
    }
  };
  auto block = [&](int n, int sign, std::vector<double>& lam, std::vector<double>& Q) {
    std::vector<double> B(n * n), va, vb;
    for (int a = 0; a < n; ++a) {
      half_vec(a, sign, va);
      for (int b = 0; b < n; ++b) {
        half_vec(b, sign, vb);
        double s = 0.0;
        for (int x = 0; x < np; ++x)
          for (int y = 0; y < np; ++y) s += va[x] * C[x * np + y] * vb[y];
        B[a * n + b] = s;
      }
    }
    jacobi_eigen(n, B, lam, Q);
  };
  std::vector<double> le, lo, Qe, Qo;
  block(he, +1, le, Qe);
  block(ho, -1, lo, Qo);
  // packed basis: row a < ho holds S[a][even j] (j < he) then S[a][odd j]
  // (j < ho); rows np-1-a follow by parity (+ even, - odd).  For odd np a last
  // row holds the middle node's S[ho][even j].  Eigenvalues in the same order:
  // the even ones ascending, then the odd ones.
  T.S.assign((size_t)ho * np + (np % 2 ? he : 0), 0.0);
  for (int a = 0; a < ho; ++a) {
    const double w = r2 / std::sqrt(M[a]);
    for (int j = 0; j < he; ++j) T.S[a * np + j] = Qe[a * he + j] * w;
    for (int j = 0; j < ho; ++j) T.S[a * np + he + j] = Qo[a * ho + j] * w;
  }
  if (np % 2)
    for (int j = 0; j < he; ++j) T.S[ho * np + j] = Qe[ho * he + j] / std::sqrt(M[ho]);
  T.lam = le;
  T.lam.insert(T.lam.end(), lo.begin(), lo.end());
}

// ---------------------------------------------------------------------------
// numbering
// ---------------------------------------------------------------------------
static const int kFaceAxis[6] = {0, 0, 1, 1, 2, 2};
static const int kFaceSide[6] = {0, 1, 0, 1, 0, 1};

static void tangential(int d, int& t1, int& t2) {
  t1 = (d == 0) ? 1 : 0;
  t2 = (d == 2) ? 1 : 2;
}

int64_t gid_of(const HostTables& T, int64_t e, int i, int j, int k) {
  const int N = T.N;
  int cx = i == 0 ? 0 : (i == N ? 2 : 1);
  int cy = j == 0 ? 0 : (j == N ? 2 : 1);
  int cz = k == 0 ? 0 : (k == N ? 2 : 1);
  const int32_t* r = &T.rec[((size_t)e * kClasses + cx + 3 * cy + 9 * cz) * kRecInts];
  int32_t code = r[1];
  int ai = (int32_t)((uint32_t)code << 22) >> 22;
  int aj = (int32_t)((uint32_t)code << 12) >> 22;
  int ak = (int32_t)((uint32_t)code << 2) >> 22;
  return (int64_t)r[0] + ai * i + aj * j + ak * k;
}

void build_numbering(HostTables& T, const int64_t* hex, int64_t n_hex, int64_t n_vtx) {
  const int N = T.N, n1 = T.n1;
  const int64_t E = n_hex;
  T.E = E;
  T.n_local = E * n1 * n1 * n1;
  for (int64_t x = 0; x < E * 8; ++x)
    if (hex[x] < 0 || hex[x] >= n_vtx) throw Error{SEM_EINVAL, "hexahedron vertex id out of range"};
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < 8; ++a)
      for (int b = a + 1; b < 8; ++b)
        if (hex[e * 8 + a] == hex[e * 8 + b]) throw Error{SEM_EMESH, "hexahedron repeats a vertex"};

  // vertices: referenced ids in ascending order
  std::vector<int64_t> vrank(n_vtx, -1);
  for (int64_t x = 0; x < E * 8; ++x) vrank[hex[x]] = 0;
  int64_t V = 0;
  for (int64_t v = 0; v < n_vtx; ++v)
    if (vrank[v] == 0) vrank[v] = V++;
  T.V = V;

  // edges: local edge le = 4 d + 2 b2 + b1 runs along axis d from corner bit 0 to 1
  std::vector<EdgeKey> ek(E * 12);
  for (int64_t e = 0; e < E; ++e)
    for (int d = 0; d < 3; ++d)
      for (int b2 = 0; b2 < 2; ++b2)
        for (int b1 = 0; b1 < 2; ++b1) {
          int t1, t2;
          tangential(d, t1, t2);
          int c0[3], c1[3];
          c0[d] = 0;
          c0[t1] = b1;
          c0[t2] = b2;
          c1[d] = 1;
          c1[t1] = b1;
          c1[t2] = b2;
          int64_t va = hex[e * 8 + corner_pos(c0[0], c0[1], c0[2])];
          int64_t vb = hex[e * 8 + corner_pos(c1[0], c1[1], c1[2])];
          int le = 4 * d + 2 * b2 + b1;
          ek[e * 12 + le] = EdgeKey{std::min(va, vb), std::max(va, vb), e, le};
        }
  std::vector<int64_t> edge_rank(E * 12), edge_inc(E * 12);
  {
    std::vector<int64_t> ord(E * 12);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
      const EdgeKey &x = ek[a], &y = ek[b];
      if (x.lo != y.lo) return x.lo < y.lo;
      if (x.hi != y.hi) return x.hi < y.hi;
      return x.e < y.e;
    });
    int64_t r = -1;
    T.einc_off.clear();
    for (int64_t p = 0; p < (int64_t)ord.size(); ++p) {
      const EdgeKey& x = ek[ord[p]];
      if (p == 0 || x.lo != ek[ord[p - 1]].lo || x.hi != ek[ord[p - 1]].hi) {
        ++r;
        T.einc_off.push_back((int32_t)p);
      }
      edge_rank[ord[p]] = r;
      edge_inc[ord[p]] = p;
    }
    T.n_edges = r + 1;
    T.einc_off.push_back((int32_t)ord.size());
  }

  // faces: local face lf = 2 d + s, corners listed by (s1 along t1, s2 along t2)
  std::vector<FaceKey> fk(E * 6);
  std::vector<int64_t> fv(E * 6 * 4);  // [e][lf][s1 + 2 s2]
  for (int64_t e = 0; e < E; ++e)
    for (int lf = 0; lf < 6; ++lf) {
      int d = kFaceAxis[lf], s = kFaceSide[lf], t1, t2;
      tangential(d, t1, t2);
      FaceKey key;
      for (int s2 = 0; s2 < 2; ++s2)
        for (int s1 = 0; s1 < 2; ++s1) {
          int c[3];
          c[d] = s;
          c[t1] = s1;
          c[t2] = s2;
          int64_t v = hex[e * 8 + corner_pos(c[0], c[1], c[2])];
          fv[(e * 6 + lf) * 4 + s1 + 2 * s2] = v;
          key.v[s1 + 2 * s2] = v;
        }
      std::sort(key.v, key.v + 4);
      key.e = e;
      key.lf = lf;
      fk[e * 6 + lf] = key;
    }
  std::vector<int64_t> face_rank(E * 6);
  std::vector<int> face_side(E * 6);
  T.face_nbr.assign(E * 12, -1);
  {
    std::vector<int64_t> ord(E * 6);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
      const FaceKey &x = fk[a], &y = fk[b];
      for (int q = 0; q < 4; ++q)
        if (x.v[q] != y.v[q]) return x.v[q] < y.v[q];
      return x.e < y.e;
    });
    int64_t r = -1;
    int side = 0;
    T.fcount.clear();
    for (int64_t p = 0; p < (int64_t)ord.size(); ++p) {
      const FaceKey& x = fk[ord[p]];
      bool fresh = p == 0 || !std::equal(x.v, x.v + 4, fk[ord[p - 1]].v);
      if (fresh) {
        ++r;
        side = 0;
        T.fcount.push_back(1);
      } else {
        ++side;
        if (side >= 2) throw Error{SEM_EMESH, "a face is shared by more than two hexahedra"};
        T.fcount.back() = 2;
        const FaceKey& y = fk[ord[p - 1]];
        T.face_nbr[(x.e * 6 + x.lf) * 2 + 0] = (int32_t)y.e;
        T.face_nbr[(x.e * 6 + x.lf) * 2 + 1] = y.lf;
        T.face_nbr[(y.e * 6 + y.lf) * 2 + 0] = (int32_t)x.e;
        T.face_nbr[(y.e * 6 + y.lf) * 2 + 1] = x.lf;
      }
      face_rank[ord[p]] = r;
      face_side[ord[p]] = side;
    }
    T.n_faces = r + 1;
  }

  // vertex incidences, sorted by (vertex, element)
  std::vector<int64_t> vert_inc(E * 8);
  {
    std::vector<int64_t> cnt(V + 1, 0);
    for (int64_t x = 0; x < E * 8; ++x) cnt[vrank[hex[x]] + 1]++;
    for (int64_t v = 0; v < V; ++v) cnt[v + 1] += cnt[v];
    T.vinc_off.assign(cnt.begin(), cnt.end());
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < E; ++e)  // element-major sweep keeps elements ascending
      for (int a = 0; a < 8; ++a) vert_inc[e * 8 + a] = fill[vrank[hex[e * 8 + a]]]++;
  }

  const int64_t m = N - 1;
  T.base_e = V;
  T.base_f = V + T.n_edges * m;
  T.base_i = T.base_f + T.n_faces * m * m;
  T.n_global = T.base_i + E * m * m * m;
  if (T.n_global >= (int64_t)INT32_MAX || T.n_local >= (int64_t)INT32_MAX)
    throw Error{SEM_EUNSUPPORTED, "mesh too large for 32-bit node ids"};
  T.wedge_off = 2 * T.n_faces * m * m;
  T.wvert_off = T.wedge_off + (int64_t)E * 12 * m;
  T.w_size = T.wvert_off + (int64_t)E * 8;

  // entity records
  T.rec.assign((size_t)E * kClasses * kRecInts, 0);
  for (int64_t e = 0; e < E; ++e) {
    for (int cz = 0; cz < 3; ++cz)
      for (int cy = 0; cy < 3; ++cy)
        for (int cx = 0; cx < 3; ++cx) {
          int cls[3] = {cx, cy, cz};
          int32_t* r = &T.rec[((size_t)e * kClasses + cx + 3 * cy + 9 * cz) * kRecInts];
          int nb = (cx != 1) + (cy != 1) + (cz != 1);
          int64_t gbase = 0, wbase = 0;
          int coef[3] = {0, 0, 0};
          int flags = 0;
          if (nb == 3) {  // vertex
            int p = corner_pos(cx / 2, cy / 2, cz / 2);
            gbase = vrank[hex[e * 8 + p]];
            int64_t inc = vert_inc[e * 8 + p];
            wbase = T.wvert_off + inc;
            if (inc == T.vinc_off[gbase]) flags |= kFlagOwned;
          } else if (nb == 2) {  // edge along the axis whose class is 1
            int d = cx == 1 ? 0 : (cy == 1 ? 1 : 2);
            int t1, t2;
            tangential(d, t1, t2);
            int le = 4 * d + 2 * (cls[t2] / 2) + (cls[t1] / 2);
            const EdgeKey& k = ek[e * 12 + le];
            int c0[3];
            c0[d] = 0;
            c0[t1] = cls[t1] / 2;
            c0[t2] = cls[t2] / 2;
            int64_t va = hex[e * 8 + corner_pos(c0[0], c0[1], c0[2])];
            bool fwd = va == k.lo;
            int64_t ed = edge_rank[e * 12 + le];
            int64_t inc = edge_inc[e * 12 + le];
            int64_t g0 = T.base_e + ed * m;
            if (fwd) {
              gbase = g0 - 1;
              coef[d] = 1;
            } else {
              gbase = g0 + N - 1;
              coef[d] = -1;
            }
            wbase = gbase - g0 + T.wedge_off + inc * m;
            if (inc == T.einc_off[ed]) flags |= kFlagOwned;
          } else if (nb == 1) {  // face normal to the axis whose class is not 1
            int d = cx != 1 ? 0 : (cy != 1 ? 1 : 2);
            int s = cls[d] / 2;
            int lf = 2 * d + s;
            int t1, t2;
            tangential(d, t1, t2);
            const int64_t* f4 = &fv[(e * 6 + lf) * 4];
            int w0 = (int)(std::min_element(f4, f4 + 4) - f4);
            int s1_0 = w0 % 2, s2_0 = w0 / 2;
            int64_t nb1 = f4[(1 - s1_0) + 2 * s2_0], nb2 = f4[s1_0 + 2 * (1 - s2_0)];
            int sg1 = s1_0 ? -1 : 1, c1 = s1_0 ? N : 0;
            int sg2 = s2_0 ? -1 : 1, c2 = s2_0 ? N : 0;
            int64_t f = face_rank[e * 6 + lf];
            int64_t g0 = T.base_f + f * m * m;
            if (nb1 < nb2) {  // p along t1
              coef[t1] = sg1;
              coef[t2] = (int)m * sg2;
              gbase = g0 - N + m * c2 + c1;
            } else {
              coef[t1] = (int)m * sg1;
              coef[t2] = sg2;
              gbase = g0 - N + m * c1 + c2;
            }
            int sd = face_side[e * 6 + lf];
            wbase = gbase - g0 + (2 * f + sd) * m * m;
            if (sd == 0) flags |= kFlagOwned;
          } else {  // interior
            gbase = T.base_i + e * m * m * m - 1 - m - m * m;
            coef[0] = 1;
            coef[1] = (int)m;
            coef[2] = (int)(m * m);
            wbase = -1;
            flags |= kFlagOwned | kFlagInterior;
          }
          r[0] = (int32_t)gbase;
          r[1] = pack_coef(coef[0], coef[1], coef[2]);
          r[2] = (int32_t)wbase;
          r[3] = flags;
        }
  }

  // default Dirichlet set: every node of a face owned by one hexahedron
  T.dir.assign(T.n_global, 0);
  for (int64_t e = 0; e < E; ++e)
    for (int lf = 0; lf < 6; ++lf) {
      if (T.face_nbr[(e * 6 + lf) * 2] >= 0) continue;
      int d = kFaceAxis[lf], s = kFaceSide[lf], t1, t2;
      tangential(d, t1, t2);
      for (int b = 0; b <= N; ++b)
        for (int a = 0; a <= N; ++a) {
          int x[3];
          x[d] = s * N;
          x[t1] = a;
          x[t2] = b;
          T.dir[gid_of(T, e, x[0], x[1], x[2])] = 1;
        }
    }

  update_interior_mask_flags(T);

  // first local copy of every global node
  T.owner.assign(T.n_global, -1);
  for (int64_t e = 0; e < E; ++e)
    for (int k = 0; k <= N; ++k)
      for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) {
          int64_t g = gid_of(T, e, i, j, k);
          if (T.owner[g] < 0) T.owner[g] = (int32_t)(e * n1 * n1 * n1 + i + n1 * (j + n1 * k));
        }
}

// flag elements whose interior holds a Dirichlet node (never the case for the
// topological boundary): only those need the mask on their direct writes
void update_interior_mask_flags(HostTables& T) {
  const int N = T.N;
  for (int64_t e = 0; e < T.E; ++e) {
    int32_t* r = &T.rec[((size_t)e * kClasses + kInteriorClass) * kRecInts];
    bool any = false;
    for (int k = 1; k < N && !any; ++k)
      for (int j = 1; j < N && !any; ++j)
        for (int i = 1; i < N; ++i)
          if (T.dir[gid_of(T, e, i, j, k)]) {
            any = true;
            break;
          }
    r[3] = any ? (r[3] | kFlagMaskedInterior) : (r[3] & ~kFlagMaskedInterior);
  }
}

void export_l2g(const HostTables& T, int32_t* l2g) {
  const int n1 = T.n1;
  parallel_for(T.E, [&](int64_t b, int64_t e1) {
    for (int64_t e = b; e < e1; ++e)
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i)
            l2g[e * n1 * n1 * n1 + i + n1 * (j + n1 * k)] = (int32_t)gid_of(T, e, i, j, k);
  });
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
void build_geometry(HostTables& T, const double* vtx, const int64_t* hex) {
  const int N = T.N, n1 = T.n1;
  const int64_t E = T.E, nn = (int64_t)n1 * n1 * n1;
  T.G.assign((size_t)E * 6 * nn, 0.0);
  T.X8.assign((size_t)E * 24, 0.0);
  T.mass.assign((size_t)E * nn, 0.0);
  T.h.assign((size_t)E * 3, 0.0);
  std::vector<double> xl((size_t)E * nn * 3);
  std::vector<int> bad(std::max<unsigned>(1, std::thread::hardware_concurrency()) * 0 + 1, 0);
  std::vector<char> badel(E, 0);
  const std::vector<double>& t = T.t;
  parallel_for(E, [&](int64_t b0, int64_t b1) {
    for (int64_t e = b0; e < b1; ++e) {
      double X[8][3];
      for (int p = 0; p < 8; ++p)
        for (int r = 0; r < 3; ++r) X[p][r] = T.X8[(size_t)e * 24 + p * 3 + r] = vtx[hex[e * 8 + p] * 3 + r];
      // box sizes: mean length of the four edges parallel to each reference axis
      for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int q = 0; q < 4; ++q) {
          int u = q & 1, v = q >> 1;
          int c0[3], c1[3];
          int t1, t2;
          tangential(d, t1, t2);
          c0[d] = 0;
          c1[d] = 1;
          c0[t1] = c1[t1] = u;
          c0[t2] = c1[t2] = v;
          const double* a = X[corner_pos(c0[0], c0[1], c0[2])];
          const double* bb = X[corner_pos(c1[0], c1[1], c1[2])];
          s += std::sqrt((a[0] - bb[0]) * (a[0] - bb[0]) + (a[1] - bb[1]) * (a[1] - bb[1]) +
                         (a[2] - bb[2]) * (a[2] - bb[2]));
        }
        T.h[e * 3 + d] = 0.25 * s;
      }
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            const double xi = t[i], eta = t[j], zeta = t[k];
            const double f[2][3] = {{0.5 * (1 - xi), 0.5 * (1 - eta), 0.5 * (1 - zeta)},
                                    {0.5 * (1 + xi), 0.5 * (1 + eta), 0.5 * (1 + zeta)}};
            const double df[2] = {-0.5, 0.5};
            double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, x[3] = {0, 0, 0};
            for (int c = 0; c < 2; ++c)
              for (int bb = 0; bb < 2; ++bb)
                for (int a = 0; a < 2; ++a) {
                  const double* P = X[corner_pos(a, bb, c)];
                  double w0 = df[a] * f[bb][1] * f[c][2];
                  double w1 = f[a][0] * df[bb] * f[c][2];
                  double w2 = f[a][0] * f[bb][1] * df[c];
                  double w3 = f[a][0] * f[bb][1] * f[c][2];
                  for (int r = 0; r < 3; ++r) {
                    J[r][0] += P[r] * w0;
                    J[r][1] += P[r] * w1;
                    J[r][2] += P[r] * w2;
                    x[r] += P[r] * w3;
                  }
                }
            double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            if (!(det > 0.0)) badel[e] = 1;
            // M = J^T J and its inverse by cofactors
            double Mt[3][3];
            for (int a = 0; a < 3; ++a)
              for (int c = 0; c < 3; ++c) Mt[a][c] = J[0][a] * J[0][c] + J[1][a] * J[1][c] + J[2][a] * J[2][c];
            double c00 = Mt[1][1] * Mt[2][2] - Mt[1][2] * Mt[2][1];
            double c01 = Mt[0][2] * Mt[2][1] - Mt[0][1] * Mt[2][2];
            double c02 = Mt[0][1] * Mt[1][2] - Mt[0][2] * Mt[1][1];
            double c11 = Mt[0][0] * Mt[2][2] - Mt[0][2] * Mt[2][0];
            double c12 = Mt[0][2] * Mt[1][0] - Mt[0][0] * Mt[1][2];
            double c22 = Mt[0][0] * Mt[1][1] - Mt[0][1] * Mt[1][0];
            double detM = Mt[0][0] * c00 + Mt[0][1] * (Mt[1][2] * Mt[2][0] - Mt[1][0] * Mt[2][2]) +
                          Mt[0][2] * (Mt[1][0] * Mt[2][1] - Mt[1][1] * Mt[2][0]);
            double w = T.rho[i] * T.rho[j] * T.rho[k] * det;
            double sc = w / detM;
            int64_t node = i + n1 * (j + n1 * k);
            double* G = &T.G[(size_t)e * 6 * nn];
            G[0 * nn + node] = sc * c00;
            G[1 * nn + node] = sc * c01;
            G[2 * nn + node] = sc * c02;
            G[3 * nn + node] = sc * c11;
            G[4 * nn + node] = sc * c12;
            G[5 * nn + node] = sc * c22;
            T.mass[e * nn + node] = w;
            for (int r = 0; r < 3; ++r) xl[(e * nn + node) * 3 + r] = x[r];
          }
    }
  });
  for (int64_t e = 0; e < E; ++e)
    if (badel[e]) throw Error{SEM_EMESH, "inverted or degenerate hexahedron (|J| <= 0 at a GLL node)"};
  // traversal order: Morton (Z-order) key of the element centroids, 21 bits per axis
  {
    std::vector<double> cen((size_t)E * 3, 0.0);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t e = 0; e < E; ++e)
      for (int r = 0; r < 3; ++r) {
        double c = 0.0;
        for (int p = 0; p < 8; ++p) c += vtx[hex[e * 8 + p] * 3 + r];
        c *= 0.125;
        cen[e * 3 + r] = c;
        lo[r] = std::min(lo[r], c);
        hi[r] = std::max(hi[r], c);
      }
    std::vector<std::pair<uint64_t, int32_t>> key(E);
    for (int64_t e = 0; e < E; ++e) {
      uint64_t m = 0;
      for (int r = 0; r < 3; ++r) {
        const double span = hi[r] > lo[r] ? hi[r] - lo[r] : 1.0;
        const uint32_t q = (uint32_t)std::min(2097151.0, (cen[e * 3 + r] - lo[r]) / span * 2097151.0);
        for (int bit = 0; bit < 21; ++bit) m |= (uint64_t)((q >> bit) & 1u) << (3 * bit + r);
      }
      key[e] = {m, (int32_t)e};
    }
    std::sort(key.begin(), key.end());
    T.order.resize(E);
    for (int64_t e = 0; e < E; ++e) T.order[e] = key[e].second;
  }
  // lumped mass: copies summed in ascending local index; coordinates of the first copy
  T.mN.assign(T.n_global, 0.0);
  T.xN.assign(T.n_global * 3, 0.0);
  for (int64_t e = 0; e < E; ++e)
    for (int k = 0; k <= N; ++k)
      for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) {
          int64_t g = gid_of(T, e, i, j, k);
          int64_t node = i + n1 * (j + n1 * k);
          T.mN[g] += T.mass[e * nn + node];
        }
  for (int64_t g = 0; g < T.n_global; ++g)
    for (int r = 0; r < 3; ++r) T.xN[g * 3 + r] = xl[(size_t)T.owner[g] * 3 + r];
  (void)bad;
}

// ---------------------------------------------------------------------------
// overlapping patches
// ---------------------------------------------------------------------------
namespace {
struct FaceMap {
  int perm[3], sign[3], off[3];
};

// Patch slot (a + m b + m^2 c, m = N + 3) of outside ordinal o, grouped by the
// entity of the element the slot lies across: 6 face planes of (N+1)^2 (face
// 2d + side, the lower of the other two axes fastest), 12 edge lines of N+1
// (edge 4 axis + side_lo + 2 side_hi, position along the axis), 8 corners
// (side_x + 2 side_y + 4 side_z).  The patch solve derives the same slot in
// closed form when it writes the outside slots in ordinal order.
int outside_patch_slot(int N, int o) {
  const int m = N + 3, n1 = N + 1, P1 = n1 * n1;
  int c[3];
  if (o < 6 * P1) {
    const int f = o / P1, t = o - f * P1, d = f >> 1;
    const int lo = d == 0 ? 1 : 0, hi = d == 2 ? 1 : 2;
    c[d] = (f & 1) ? m - 1 : 0;
    c[lo] = 1 + t % n1;
    c[hi] = 1 + t / n1;
  } else if (o < 6 * P1 + 12 * n1) {
    const int q = o - 6 * P1, id = q / n1, ax = id >> 2;
    const int lo = ax == 0 ? 1 : 0, hi = ax == 2 ? 1 : 2;
    c[ax] = 1 + q % n1;
    c[lo] = (id & 1) ? m - 1 : 0;
    c[hi] = (id & 2) ? m - 1 : 0;
  } else {
    const int id = o - 6 * P1 - 12 * n1;
    c[0] = (id & 1) ? m - 1 : 0;
    c[1] = (id & 2) ? m - 1 : 0;
    c[2] = (id & 4) ? m - 1 : 0;
  }
  return c[0] + m * (c[1] + m * c[2]);
}
}  // namespace

void build_patches(HostTables& T, const int64_t* hex) {
  const int N = T.N, np = T.np;
  const int64_t E = T.E, pp = (int64_t)np * np * np;
  // affine maps across every interior face: y[perm[d]] = sign[d] x[d] + off[d]
  std::vector<FaceMap> fmap(E * 6);
  auto lattice = [&](int p, int* c) {
    c[0] = (p & 1) * N;
    c[1] = ((p >> 1) & 1) * N;
    c[2] = ((p >> 2) & 1) * N;
  };
  for (int64_t e = 0; e < E; ++e)
    for (int lf = 0; lf < 6; ++lf) {
      int64_t e2 = T.face_nbr[(e * 6 + lf) * 2];
      if (e2 < 0) continue;
      int lf2 = T.face_nbr[(e * 6 + lf) * 2 + 1];
      int d = kFaceAxis[lf], s = kFaceSide[lf], d2 = kFaceAxis[lf2], s2 = kFaceSide[lf2];
      FaceMap fm;
      auto pos_in_e2 = [&](int64_t v) {
        for (int p = 0; p < 8; ++p)
          if (hex[e2 * 8 + p] == v) return p;
        return -1;
      };
      int base[3] = {0, 0, 0};
      base[d] = s;
      int y0[3];
      lattice(pos_in_e2(hex[e * 8 + corner_pos(base[0], base[1], base[2])]), y0);
      int t1, t2;
      tangential(d, t1, t2);
      for (int tt : {t1, t2}) {
        int c1[3] = {base[0], base[1], base[2]};
        c1[tt] = 1;
        int y1[3];
        lattice(pos_in_e2(hex[e * 8 + corner_pos(c1[0], c1[1], c1[2])]), y1);
        for (int ax = 0; ax < 3; ++ax)
          if (y1[ax] != y0[ax]) {
            fm.perm[tt] = ax;
            fm.sign[tt] = (y1[ax] - y0[ax]) / N;
            fm.off[tt] = y0[ax];
          }
      }
      fm.perm[d] = d2;
      fm.sign[d] = (s == s2) ? -1 : 1;
      fm.off[d] = (s == 0 && s2 == 0) ? 0 : (s == 0 ? N : (s2 == 0 ? -N : 2 * N));
      fmap[e * 6 + lf] = fm;
    }
  auto edge_valence = [&](int64_t va, int64_t vb, int64_t e) {
    // number of hexahedra sharing mesh edge (va, vb): the incidence list of the
    // edge is found from element e's own local edge
    for (int d = 0; d < 3; ++d)
      for (int b2 = 0; b2 < 2; ++b2)
        for (int b1 = 0; b1 < 2; ++b1) {
          int t1, t2;
          tangential(d, t1, t2);
          int c0[3], c1[3];
          c0[d] = 0;
          c1[d] = 1;
          c0[t1] = c1[t1] = b1;
          c0[t2] = c1[t2] = b2;
          int64_t a = hex[e * 8 + corner_pos(c0[0], c0[1], c0[2])];
          int64_t b = hex[e * 8 + corner_pos(c1[0], c1[1], c1[2])];
          if ((a == va && b == vb) || (a == vb && b == va)) {
            int64_t g = gid_of(T, e, c0[0] * N + (d == 0), c0[1] * N + (d == 1), c0[2] * N + (d == 2));
            int64_t ed = (g - T.base_e) / (N - 1);
            return T.einc_off[ed + 1] - T.einc_off[ed];
          }
        }
    return 0;
  };
  T.ip.assign((size_t)E * pp, -1);
  // patch slots outside the element: ordinal among them, or -(local index)-1 inside
  const int n1 = N + 1;
  const int64_t nx = pp - (int64_t)n1 * n1 * n1;
  T.nx = nx;
  T.xord.assign(pp, 0);
  for (int c = 1; c <= N + 1; ++c)
    for (int b = 1; b <= N + 1; ++b)
      for (int a = 1; a <= N + 1; ++a)
        T.xord[a + np * (b + np * c)] = -((a - 1) + n1 * ((b - 1) + n1 * (c - 1))) - 1;
  for (int32_t o = 0; o < (int32_t)nx; ++o) T.xord[outside_patch_slot(N, o)] = o;
  // consumer slot of an outside patch slot: the element it lands in receives it
  // in its own frame, at one layer in from the face / edge / corner it shares
  // with the patch's element
  T.xdest.assign((size_t)E * nx, -1);
  const int64_t fplane = (int64_t)n1 * n1;
  auto other_axes = [](int d, int& lo, int& hi) {
    lo = d == 0 ? 1 : 0;
    hi = d == 2 ? 1 : 2;
  };
  auto local_corner = [&](int64_t e, int64_t v) {
    for (int q = 0; q < 8; ++q)
      if (hex[e * 8 + q] == v) return q;
    return -1;
  };
  auto layer1 = [&](int v, int side) { return v == (side ? N - 1 : 1); };
  std::atomic<bool> off_layer{false};
  parallel_for(E, [&](int64_t b0, int64_t b1) {
    for (int64_t s = b0; s < b1; ++s) {
      for (int c = 0; c < np; ++c)
        for (int b = 0; b < np; ++b)
          for (int a = 0; a < np; ++a) {
            int x[3] = {a - 1, b - 1, c - 1};
            int nout = 0;
            int corner[3];
            for (int d = 0; d < 3; ++d) {
              bool o = x[d] < 0 || x[d] > N;
              nout += o;
              corner[d] = x[d] < 0 ? 0 : 1;
            }
            if (nout == 2) {
              int dfree = (x[0] >= 0 && x[0] <= N) ? 0 : ((x[1] >= 0 && x[1] <= N) ? 1 : 2);
              int c0[3] = {corner[0], corner[1], corner[2]}, c1[3] = {corner[0], corner[1], corner[2]};
              c0[dfree] = 0;
              c1[dfree] = 1;
              if (edge_valence(hex[s * 8 + corner_pos(c0[0], c0[1], c0[2])],
                               hex[s * 8 + corner_pos(c1[0], c1[1], c1[2])], s) != 4)
                continue;
            } else if (nout == 3) {
              int64_t v = hex[s * 8 + corner_pos(corner[0], corner[1], corner[2])];
              int64_t vr = gid_of(T, s, corner[0] * N, corner[1] * N, corner[2] * N);
              if (T.vinc_off[vr + 1] - T.vinc_off[vr] != 8) continue;
              bool ok = true;
              for (int d = 0; d < 3; ++d) {
                int c1[3] = {corner[0], corner[1], corner[2]};
                c1[d] = 1 - c1[d];
                if (edge_valence(v, hex[s * 8 + corner_pos(c1[0], c1[1], c1[2])], s) != 4) ok = false;
              }
              if (!ok) continue;
            }
            int64_t e = s;
            bool valid = true;
            int entry = -1;  // face of the landing element through which the last step entered
            int64_t ev0 = -1, ev1 = -1;  // mesh edge (nout = 2) or vertex (nout = 3) shared with the patch
            if (nout == 2) {
              int dfree = (x[0] >= 0 && x[0] <= N) ? 0 : ((x[1] >= 0 && x[1] <= N) ? 1 : 2);
              int c0[3] = {corner[0], corner[1], corner[2]}, c1[3] = {corner[0], corner[1], corner[2]};
              c0[dfree] = 0;
              c1[dfree] = 1;
              ev0 = hex[s * 8 + corner_pos(c0[0], c0[1], c0[2])];
              ev1 = hex[s * 8 + corner_pos(c1[0], c1[1], c1[2])];
            } else if (nout == 3) {
              ev0 = hex[s * 8 + corner_pos(corner[0], corner[1], corner[2])];
            }
            for (int step = 0; step < 4; ++step) {
              int d = -1;
              for (int q = 0; q < 3; ++q)
                if (x[q] < 0 || x[q] > N) {
                  d = q;
                  break;
                }
              if (d < 0) break;
              int lf = 2 * d + (x[d] < 0 ? 0 : 1);
              int64_t e2 = T.face_nbr[(e * 6 + lf) * 2];
              if (e2 < 0) {
                valid = false;
                break;
              }
              const FaceMap& fm = fmap[e * 6 + lf];
              int y[3];
              for (int q = 0; q < 3; ++q) y[fm.perm[q]] = fm.sign[q] * x[q] + fm.off[q];
              x[0] = y[0];
              x[1] = y[1];
              x[2] = y[2];
              entry = T.face_nbr[(e * 6 + lf) * 2 + 1];
              e = e2;
            }
            if (!valid) continue;
            const int slot = a + np * (b + np * c);
            T.ip[(size_t)s * pp + slot] = (int32_t)gid_of(T, e, x[0], x[1], x[2]);
            if (nout == 0) continue;
            int64_t cs = -1;
            if (nout == 1) {
              const int d = kFaceAxis[entry], side = kFaceSide[entry];
              int lo, hi;
              other_axes(d, lo, hi);
              if (layer1(x[d], side)) cs = entry * fplane + x[lo] + (int64_t)n1 * x[hi];
            } else if (nout == 2) {
              const int pa = local_corner(e, ev0), pb = local_corner(e, ev1);
              if (pa >= 0 && pb >= 0 && __builtin_popcount(pa ^ pb) == 1) {
                const int ax = __builtin_ctz(pa ^ pb);
                int lo, hi;
                other_axes(ax, lo, hi);
                const int slo = (pa >> lo) & 1, shi = (pa >> hi) & 1;
                if (layer1(x[lo], slo) && layer1(x[hi], shi))
                  cs = 6 * fplane + (int64_t)(ax * 4 + slo + 2 * shi) * n1 + x[ax];
              }
            } else {
              const int pc = local_corner(e, ev0);
              if (pc >= 0 && layer1(x[0], pc & 1) && layer1(x[1], (pc >> 1) & 1) && layer1(x[2], (pc >> 2) & 1))
                cs = 6 * fplane + 12 * (int64_t)n1 + pc;
            }
            if (cs < 0) {
              off_layer = true;
              continue;
            }
            T.xdest[(size_t)s * nx + T.xord[slot]] = (int32_t)(e * nx + cs);
          }
    }
  });
  if (off_layer) throw Error{SEM_EMESH, "patch slot lands off the expected layer"};
  if ((int64_t)E * nx >= (int64_t)INT32_MAX) throw Error{SEM_EUNSUPPORTED, "patch table too large"};
  // every consumer slot is filled by at most one patch
  std::vector<uint8_t> hit((size_t)E * nx, 0);
  for (int32_t d : T.xdest)
    if (d >= 0) {
      if (hit[d]) throw Error{SEM_EMESH, "two patches write one consumer slot"};
      hit[d] = 1;
    }
}

// ---------------------------------------------------------------------------
// coarse space: order-1 operator on the free vertices, BFS levels
// ---------------------------------------------------------------------------
void build_coarse_matrices(HostTables& T, const double* vtx, const int64_t* hex) {
  const int64_t E = T.E;
  // element matrices of the order-1 operator: quadrature at the 8 corners (weights 1)
  T.corner_K.assign((size_t)E * 64, 0.0);
  T.corner_M.assign((size_t)E * 8, 0.0);
  parallel_for(E, [&](int64_t b0, int64_t b1) {
    for (int64_t e = b0; e < b1; ++e) {
      double X[8][3];
      for (int p = 0; p < 8; ++p)
        for (int r = 0; r < 3; ++r) X[p][r] = vtx[hex[e * 8 + p] * 3 + r];
      double* K = &T.corner_K[e * 64];
      for (int q = 0; q < 8; ++q) {
        int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
        double J[3][3];
        for (int r = 0; r < 3; ++r) {
          J[r][0] = 0.5 * (X[corner_pos(1, qb, qc)][r] - X[corner_pos(0, qb, qc)][r]);
          J[r][1] = 0.5 * (X[corner_pos(qa, 1, qc)][r] - X[corner_pos(qa, 0, qc)][r]);
          J[r][2] = 0.5 * (X[corner_pos(qa, qb, 1)][r] - X[corner_pos(qa, qb, 0)][r]);
        }
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        // the mass term with the same corner rule: diagonal, |J| at the corner
        T.corner_M[e * 8 + q] = det;
        // inverse Jacobian by cofactors: Jinv[a][r]
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        // physical gradient of each corner basis function at corner q
        double gphys[8][3];
        for (int p = 0; p < 8; ++p) {
          int pa = p & 1, pb = (p >> 1) & 1, pc = p >> 2;
          double gr[3];
          gr[0] = (pb == qb && pc == qc) ? (pa ? 0.5 : -0.5) : 0.0;
          gr[1] = (pa == qa && pc == qc) ? (pb ? 0.5 : -0.5) : 0.0;
          gr[2] = (pa == qa && pb == qb) ? (pc ? 0.5 : -0.5) : 0.0;
          for (int r = 0; r < 3; ++r) gphys[p][r] = Ji[0][r] * gr[0] + Ji[1][r] * gr[1] + Ji[2][r] * gr[2];
        }
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b)
            K[a * 8 + b] += det * (gphys[a][0] * gphys[b][0] + gphys[a][1] * gphys[b][1] +
                                   gphys[a][2] * gphys[b][2]);
      }
    }
  });
}

void build_coarse_tree(HostTables& T, int leaf_max) {
  const int N = T.N;
  const int64_t E = T.E, V = T.V;
  if (leaf_max <= 0) leaf_max = 128;
  // free vertices and their adjacency
  std::vector<int64_t> vid(E * 8);
  for (int64_t e = 0; e < E; ++e)
    for (int p = 0; p < 8; ++p) vid[e * 8 + p] = gid_of(T, e, (p & 1) * N, ((p >> 1) & 1) * N, (p >> 2) * N);
  std::vector<std::vector<int64_t>> adj(V);
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        if (a != b) adj[vid[e * 8 + a]].push_back(vid[e * 8 + b]);
  std::vector<char> freev(V);
  for (int64_t v = 0; v < V; ++v) freev[v] = T.dir[v] == 0;
  for (int64_t v = 0; v < V; ++v) {
    auto& l = adj[v];
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
    l.erase(std::remove_if(l.begin(), l.end(), [&](int64_t w) { return !freev[w]; }), l.end());
  }
  // element size along each physical axis (mean extent of the elements'
  // vertex boxes): extents are measured in element layers, so stretched
  // meshes are cut across their longest side
  double hax[3] = {0.0, 0.0, 0.0};
  for (int64_t e = 0; e < E; ++e) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int p = 0; p < 8; ++p)
      for (int r = 0; r < 3; ++r) {
        lo[r] = std::min(lo[r], T.xN[vid[e * 8 + p] * 3 + r]);
        hi[r] = std::max(hi[r], T.xN[vid[e * 8 + p] * 3 + r]);
      }
    for (int r = 0; r < 3; ++r) hax[r] += (hi[r] - lo[r]) / (double)E;
  }
  for (int r = 0; r < 3; ++r) hax[r] = std::max(hax[r], 1e-300);
  auto coord = [&](int64_t v, int r) { return T.xN[v * 3 + r]; };

  // --- recursive dissection (explicit task stack; nodes created in pre-order)
  struct TNode {
    std::vector<int64_t> own;
    int32_t parent;
    std::vector<int32_t> children;
  };
  std::vector<TNode> nodes;
  struct Task {
    std::vector<int64_t> verts;
    int32_t parent;
  };
  std::vector<Task> tasks;
  // connected components of the free-vertex graph are independent trees
  {
    std::vector<char> seen(V, 0);
    std::vector<Task> comps;
    for (int64_t v0 = 0; v0 < V; ++v0) {
      if (!freev[v0] || seen[v0]) continue;
      Task t{{v0}, -1};
      seen[v0] = 1;
      for (size_t q = 0; q < t.verts.size(); ++q)
        for (int64_t w : adj[t.verts[q]])
          if (!seen[w]) {
            seen[w] = 1;
            t.verts.push_back(w);
          }
      comps.push_back(std::move(t));
    }
    // processed in ascending order of their smallest vertex
    for (auto it = comps.rbegin(); it != comps.rend(); ++it) tasks.push_back(std::move(*it));
  }
  std::vector<int64_t> stamp(V, -1), level(V, -1);
  int64_t tick = 0;
  auto add_node = [&](std::vector<int64_t> own, int32_t parent) {
    std::sort(own.begin(), own.end());
    nodes.push_back(TNode{std::move(own), parent, {}});
    const int32_t id = (int32_t)nodes.size() - 1;
    if (parent >= 0) nodes[parent].children.push_back(id);
    return id;
  };
  // BFS levels of `verts` (stamped with `tick`) from `start`; returns the
  // level sizes, unreached vertices keep level -1
  auto bfs = [&](const std::vector<int64_t>& start) {
    std::vector<int64_t> sizes;
    std::vector<int64_t> front = start;
    for (int64_t v : front) level[v] = 0;
    int64_t cur = 0;
    while (!front.empty()) {
      sizes.push_back((int64_t)front.size());
      std::vector<int64_t> next;
      for (int64_t v : front)
        for (int64_t w : adj[v])
          if (stamp[w] == tick && level[w] < 0) {
            level[w] = cur + 1;
            next.push_back(w);
          }
      ++cur;
      front.swap(next);
    }
    return sizes;
  };
  while (!tasks.empty()) {
    Task t = std::move(tasks.back());
    tasks.pop_back();
    if ((int64_t)t.verts.size() <= leaf_max) {
      add_node(std::move(t.verts), t.parent);
      continue;
    }
    ++tick;
    for (int64_t v : t.verts) {
      stamp[v] = tick;
      level[v] = -1;
    }
    // longest extent, in element layers
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v : t.verts)
      for (int r = 0; r < 3; ++r) {
        lo[r] = std::min(lo[r], coord(v, r));
        hi[r] = std::max(hi[r], coord(v, r));
      }
    int ax = 0;
    for (int r = 1; r < 3; ++r)
      if ((hi[r] - lo[r]) / hax[r] > (hi[ax] - lo[ax]) / hax[ax]) ax = r;
    // BFS from the layer of vertices at the low end of that extent
    std::vector<int64_t> start;
    for (int64_t v : t.verts)
      if (coord(v, ax) <= lo[ax] + 0.5 * hax[ax]) start.push_back(v);
    std::vector<int64_t> sizes = bfs(start);
    if (sizes.size() < 3) {
      // too flat for a level cut: restart from the single lowest vertex
      for (int64_t v : t.verts) level[v] = -1;
      int64_t v0 = t.verts[0];
      for (int64_t v : t.verts)
        if (coord(v, ax) < coord(v0, ax) || (coord(v, ax) == coord(v0, ax) && v < v0)) v0 = v;
      sizes = bfs({v0});
    }
    // vertices the BFS did not reach are not connected to the rest: own task
    Task rest{{}, t.parent};
    for (int64_t v : t.verts)
      if (level[v] < 0) rest.verts.push_back(v);
    if (sizes.size() < 3) {
      // no level has vertices on both sides: keep the reached part whole
      std::vector<int64_t> reached;
      for (int64_t v : t.verts)
        if (level[v] >= 0) reached.push_back(v);
      add_node(std::move(reached), t.parent);
      if (!rest.verts.empty()) tasks.push_back(std::move(rest));
      continue;
    }
    int64_t reached = 0;
    for (int64_t c : sizes) reached += c;
    // separator: the level where the cumulative count passes half (never the
    // first or the last, so both sides are non-empty)
    int64_t cut = 1, acc = sizes[0];
    while (cut + 1 < (int64_t)sizes.size() - 1 && acc + sizes[cut] < (reached + 1) / 2) acc += sizes[cut++];
    std::vector<int64_t> sep;
    Task left{{}, -1}, right{{}, -1};
    for (int64_t v : t.verts) {
      if (level[v] < 0) continue;
      if (level[v] == cut)
        sep.push_back(v);
      else if (level[v] < cut)
        left.verts.push_back(v);
      else
        right.verts.push_back(v);
    }
    const int32_t id = add_node(std::move(sep), t.parent);
    left.parent = right.parent = id;
    if (!rest.verts.empty()) tasks.push_back(std::move(rest));
    tasks.push_back(std::move(right));
    tasks.push_back(std::move(left));
  }

  // --- post-order numbering
  const int32_t nn = (int32_t)nodes.size();
  std::vector<int32_t> post;
  post.reserve(nn);
  {
    std::vector<std::pair<int32_t, size_t>> st;
    for (int32_t r = 0; r < nn; ++r) {
      if (nodes[r].parent >= 0) continue;
      st.push_back({r, 0});
      while (!st.empty()) {
        auto& top = st.back();
        if (top.second < nodes[top.first].children.size()) {
          const int32_t c = nodes[top.first].children[top.second++];
          st.push_back({c, 0});
        } else {
          post.push_back(top.first);
          st.pop_back();
        }
      }
    }
  }
  std::vector<int32_t> rank(nn);
  for (int32_t q = 0; q < nn; ++q) rank[post[q]] = q;
  T.cidx.assign(V, -1);
  T.fnodes.assign(nn, FrontNode{});
  T.fchildren.assign(nn, {});
  int64_t nc = 0;
  for (int32_t q = 0; q < nn; ++q) {
    const TNode& tn = nodes[post[q]];
    FrontNode& F = T.fnodes[q];
    F.off = nc;
    F.s = (int32_t)tn.own.size();
    F.parent = tn.parent >= 0 ? rank[tn.parent] : -1;
    for (int64_t v : tn.own) T.cidx[v] = (int32_t)nc++;
    for (int32_t c : tn.children) T.fchildren[q].push_back(rank[c]);
    std::sort(T.fchildren[q].begin(), T.fchildren[q].end());
  }
  T.nc = nc;

  // --- boundary of each node: ancestors coupled to its subtree after elimination
  std::vector<std::vector<int32_t>> bnd(nn);
  int32_t maxh = -1;
  for (int32_t q = 0; q < nn; ++q) {
    FrontNode& F = T.fnodes[q];
    const int64_t end = F.off + F.s;
    std::vector<int32_t> u;
    for (int64_t v : nodes[post[q]].own)
      for (int64_t w : adj[v])
        if (T.cidx[w] >= end) u.push_back(T.cidx[w]);
    int32_t h = 0;
    for (int32_t c : T.fchildren[q]) {
      for (int32_t g : bnd[c])
        if (g >= end) u.push_back(g);
      h = std::max(h, T.fnodes[c].height + 1);
    }
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    F.b = (int32_t)u.size();
    F.height = h;
    maxh = std::max(maxh, h);
    bnd[q] = std::move(u);
  }
  // every boundary vertex belongs to an ancestor (the separator property)
  for (int32_t q = 0; q < nn; ++q) {
    for (int32_t g : bnd[q]) {
      int32_t a = T.fnodes[q].parent;
      while (a >= 0 && !(g >= T.fnodes[a].off && g < T.fnodes[a].off + T.fnodes[a].s)) a = T.fnodes[a].parent;
      if (a < 0) throw Error{SEM_EMESH, "coarse dissection: boundary vertex outside the ancestors"};
    }
  }
  // --- offsets, contribution lists, per-height work lists, set-up sizes
  T.fb_idx.clear();
  int64_t fwd = 0, bwd = 0, coff = 0;
  int32_t mf = 0;
  for (int32_t q = 0; q < nn; ++q) {
    FrontNode& F = T.fnodes[q];
    F.bidx = (int64_t)T.fb_idx.size();
    T.fb_idx.insert(T.fb_idx.end(), bnd[q].begin(), bnd[q].end());
    F.fwd = fwd;
    F.bwd = bwd;
    F.coff = coff;
    F.small = F.s <= kSmallFront ? 1 : 0;
    fwd += (int64_t)(F.s + F.b) * F.s;
    bwd += (int64_t)F.s * F.b;
    coff += F.b;
    mf = std::max(mf, F.s + F.b);
  }
  T.fwd_size = fwd;
  T.bwd_size = bwd;
  T.c_size = coff;
  T.max_front = mf;
  T.ct_off.assign(nc + 1, 0);
  for (int32_t q = 0; q < nn; ++q)
    for (int32_t g : bnd[q]) T.ct_off[g + 1]++;
  for (int64_t r = 0; r < nc; ++r) T.ct_off[r + 1] += T.ct_off[r];
  T.ct_pos.assign(T.ct_off[nc], 0);
  {
    std::vector<int32_t> fill(T.ct_off.begin(), T.ct_off.end() - 1);
    for (int32_t q = 0; q < nn; ++q)  // ascending node: fixed subtraction order
      for (int32_t k = 0; k < T.fnodes[q].b; ++k)
        T.ct_pos[fill[bnd[q][k]]++] = (int32_t)(T.fnodes[q].coff + k);
  }
  T.n_heights = maxh + 1;
  T.fy_off.assign(T.n_heights + 1, 0);
  T.fr_off.assign(T.n_heights + 1, 0);
  T.br_off.assign(T.n_heights + 1, 0);
  T.fs_off.assign(T.n_heights + 1, 0);
  T.fy_items.clear();
  T.fr_items.clear();
  T.br_items.clear();
  T.fs_items.clear();
  T.fr_shape.assign(T.n_heights, CoarseTileShape{4, 0});
  T.br_shape.assign(T.n_heights, CoarseTileShape{4, 0});
  for (int32_t h = 0; h < T.n_heights; ++h) {
    // tile shapes from the longest row at this height: s for the forward
    // rows of large nodes, b for the backward rows
    int64_t lf = 0, lb = 0;
    for (int32_t q = 0; q < nn; ++q) {
      const FrontNode& F = T.fnodes[q];
      if (F.height != h) continue;
      if (!F.small) lf = std::max<int64_t>(lf, F.s);
      lb = std::max<int64_t>(lb, F.b);
    }
    T.fr_shape[h] = coarse_tile_shape(lf);
    T.br_shape[h] = coarse_tile_shape(lb);
    const int32_t tf = coarse_tile_rows(T.fr_shape[h]), tb = coarse_tile_rows(T.br_shape[h]);
    for (int32_t q = 0; q < nn; ++q) {
      const FrontNode& F = T.fnodes[q];
      if (F.height != h) continue;
      if (!F.small)  // small nodes assemble their y in the forward kernel
        for (int32_t r = 0; r < F.s; ++r) T.fy_items.push_back((int32_t)(F.off + r));
      if (F.small)
        for (int32_t r = 0; r < (F.s + F.b + 63) / 64; ++r) T.fs_items.push_back(RowItem{q, r});
      else
        for (int32_t r = 0; r < F.s + F.b; r += tf) T.fr_items.push_back(RowItem{q, r});
      for (int32_t r = 0; r < F.s; r += tb) T.br_items.push_back(RowItem{q, r});
    }
    T.fy_off[h + 1] = (int32_t)T.fy_items.size();
    T.fr_off[h + 1] = (int64_t)T.fr_items.size();
    T.br_off[h + 1] = (int64_t)T.br_items.size();
    T.fs_off[h + 1] = (int64_t)T.fs_items.size();
  }
  // largest sum of update matrices waiting for their parent (post-order stack)
  {
    int64_t cur = 0, mx = 0;
    for (int32_t q = 0; q < nn; ++q) {
      for (int32_t c : T.fchildren[q]) cur -= (int64_t)T.fnodes[c].b * T.fnodes[c].b;
      cur += (int64_t)T.fnodes[q].b * T.fnodes[q].b;
      mx = std::max(mx, cur);
    }
    T.ustack_size = mx;
  }
  T.coarse_vid = std::move(vid);
  assemble_coarse_matrix(T);
}

// Lumped surface mass of boundary faces (the Neumann term of eq. (pdeweak)
// with the GLL rule on each face): ws_N = sum over the listed faces holding
// node N of rho_p rho_q |dx/da x dx/db|, a and b the face's two reference axes
// in increasing order, p and q the node's indices along them.  Faces are
// (element, local face 2 axis + side) pairs and must lie on the boundary.
void boundary_face_mass(const HostTables& T, const int64_t* faces, int64_t nf, double* ws) {
  const int N = T.N, n1 = N + 1;
  for (int64_t f = 0; f < nf; ++f) {
    const int64_t e = faces[2 * f];
    const int64_t lf = faces[2 * f + 1];
    if (e < 0 || e >= T.E || lf < 0 || lf > 5) throw Error{SEM_EINVAL, "face out of range"};
    if (T.face_nbr[(e * 6 + lf) * 2] >= 0) throw Error{SEM_EINVAL, "Neumann face is not on the boundary"};
  }
  std::fill(ws, ws + T.n_global, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    const int64_t e = faces[2 * f];
    const int d = (int)(faces[2 * f + 1] / 2), side = (int)(faces[2 * f + 1] % 2);
    const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
    const double* X = &T.X8[e * 24];
    for (int q = 0; q < n1; ++q)
      for (int p = 0; p < n1; ++p) {
        int idx[3];
        idx[d] = side ? N : 0;
        idx[a] = p;
        idx[b] = q;
        const double x[3] = {T.t[idx[0]], T.t[idx[1]], T.t[idx[2]]};
        // dx/dxi_r at the node from the trilinear map of the 8 vertices
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int c = 0; c < 8; ++c) {
          const int bit[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
          double f[3], df[3];
          for (int r = 0; r < 3; ++r) {
            f[r] = bit[r] ? 0.5 * (1.0 + x[r]) : 0.5 * (1.0 - x[r]);
            df[r] = bit[r] ? 0.5 : -0.5;
          }
          const double w[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
          for (int r = 0; r < 3; ++r)
            for (int comp = 0; comp < 3; ++comp) J[comp][r] += X[c * 3 + comp] * w[r];
        }
        const double t1[3] = {J[0][a], J[1][a], J[2][a]}, t2[3] = {J[0][b], J[1][b], J[2][b]};
        const double nx = t1[1] * t2[2] - t1[2] * t2[1], ny = t1[2] * t2[0] - t1[0] * t2[2],
                     nz = t1[0] * t2[1] - t1[1] * t2[0];
        ws[gid_of(T, e, idx[0], idx[1], idx[2])] += T.rho[p] * T.rho[q] * std::sqrt(nx * nx + ny * ny + nz * nz);
      }
  }
}

// CSR of A_c = kappa K_c + c M_c in coarse order, assembled from the corner
// matrices in element order with each element's kappa and c (the sparsity
// follows the free vertices)
void assemble_coarse_matrix(HostTables& T) {
  const int64_t E = T.E, nc = T.nc;
  const std::vector<int64_t>& vid = T.coarse_vid;
  std::vector<std::vector<std::pair<int32_t, double>>> rows(nc);
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < 8; ++a) {
      int32_t ra = T.cidx[vid[e * 8 + a]];
      if (ra < 0) continue;
      for (int b = 0; b < 8; ++b) {
        int32_t cb = T.cidx[vid[e * 8 + b]];
        if (cb < 0) continue;
        const double ke = T.kap_e.empty() ? T.kappa : T.kap_e[e];
        const double ce = T.c_e.empty() ? T.cmass : T.c_e[e];
        double v = ke * T.corner_K[e * 64 + a * 8 + b];
        if (a == b && ce != 0.0) v += ce * T.corner_M[e * 8 + a];
        rows[ra].push_back({cb, v});
      }
    }
  T.ac_off.assign(nc + 1, 0);
  T.ac_col.clear();
  T.ac_val.clear();
  for (int64_t r = 0; r < nc; ++r) {
    auto& l = rows[r];
    std::stable_sort(l.begin(), l.end(), [](auto& x, auto& y) { return x.first < y.first; });
    for (size_t q = 0; q < l.size(); ++q) {
      if (q > 0 && l[q].first == l[q - 1].first)
        T.ac_val.back() += l[q].second;
      else {
        T.ac_col.push_back(l[q].first);
        T.ac_val.push_back(l[q].second);
      }
    }
    T.ac_off[r + 1] = (int32_t)T.ac_col.size();
  }
}

}  // namespace sem
