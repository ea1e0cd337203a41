// Device kernels of the truncated HOSVD (Sec. II.B.1), all FP64.
//
// For a tensor A (n1 x n2 x n3, complex) the mode-d factor U_d holds the
// leading left singular vectors of the unfolding A_(d), i.e. the leading
// eigenvectors of the Gram matrix S_d = A_(d) A_(d)^*; the singular values are
// the square roots of its eigenvalues.  The core is A x1 U1^* x2 U2^* x3 U3^*
// (eq. 6/7).  Kernels:
//   gram_kernel     S_d for every tensor and mode, 64 x 64 output tiles
//   jacobi_kernel   cyclic parallel Jacobi eigensolver of one Hermitian
//                   matrix (n <= 64) per workgroup, held in LDS
//   proj1/2/3       the three n-mode products with U_d^* that form the core
#include <algorithm>

#include "tv_internal.h"

namespace tv {

__device__ __forceinline__ double2 zfma_conj_b(double2 a, double2 b, double2 c) {
  // c + a * conj(b)
  c.x = fma(a.x, b.x, c.x);
  c.x = fma(a.y, b.y, c.x);
  c.y = fma(a.y, b.x, c.y);
  c.y = fma(-a.x, b.y, c.y);
  return c;
}
__device__ __forceinline__ double2 zfma_conj_a(double2 a, double2 b, double2 c) {
  // c + conj(a) * b
  c.x = fma(a.x, b.x, c.x);
  c.x = fma(a.y, b.y, c.x);
  c.y = fma(a.x, b.y, c.y);
  c.y = fma(-a.y, b.x, c.y);
  return c;
}

// Element (i, o) of the mode-d unfolding: o enumerates the other two indices
// with the lower one fastest.
__device__ __forceinline__ int64_t unfold_index(int d, int64_t i, int64_t o, int n1, int n2) {
  if (d == 0) return i + (int64_t)n1 * o;
  if (d == 1) return (o % n1) + (int64_t)n1 * i + (int64_t)n1 * n2 * (o / n1);
  return o + (int64_t)n1 * n2 * i;
}

// Tile pair index -> (ti, tj) with ti <= tj over `tiles` row tiles.
__device__ __forceinline__ void gram_pair(int pr, int tiles, int& ti, int& tj) {
  ti = 0;
  while (pr >= tiles - ti) {
    pr -= tiles - ti;
    ++ti;
  }
  tj = ti + pr;
}

typedef double v4d __attribute__((ext_vector_type(4)));

// S_d = A_(d) A_(d)^*, one 64 x 64 tile (ti <= tj: S is Hermitian, the tile
// below the diagonal is written as the conjugate transpose) of one (tensor,
// mode) per workgroup.  The unfolding streams through LDS 16 columns at a
// time, the next 16 loaded into registers during the current ones' products.
// The products run on FP64 MFMA (v_mfma_f64_16x16x4f64: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16], and accumulator r of lane l is
// D[l / 16 + 4 r][l % 16]): wave w owns the 32 x 32 sub-tile at rows
// 32 (w / 2), columns 32 (w % 2), as 2 x 2 blocks of 16 x 16, each with a
// real and an imaginary accumulator; per 4 columns of the unfolding,
// Re += Xr_re Xc_re^T + Xr_im Xc_im^T and Im += Xr_im Xc_re^T - Xr_re Xc_im^T
// (S = Xr Xc^*).
// With nsplit > 1 the unfolding's columns are cut into nsplit ranges (a
// multiple of 16 each) and every workgroup writes the whole 64 x 64 partial
// tile of its range to P, [split][tensor][mode][pair] tiles row-major;
// gram_reduce_kernel sums them.  grid.x = nsplit * tensors * 3 * tiles
// (tiles + 1) / 2 with tiles = ceil(nmax / 64).
__global__ __launch_bounds__(256) void gram_kernel(const double2* __restrict__ A, int ntens,
                                                   int n1, int n2, int n3, int nmax, int nsplit,
                                                   double2* __restrict__ S,
                                                   double2* __restrict__ P) {
  constexpr int OC = 16;
  __shared__ double2 Xr[64][OC + 1];
  __shared__ double2 Xc[64][OC + 1];
  const int tiles = (nmax + 63) / 64;
  const int pairs = tiles * (tiles + 1) / 2;
  int64_t b = blockIdx.x;
  const int sp = (int)(b % nsplit);
  b /= nsplit;
  const int pr = (int)(b % pairs);
  const int64_t tile_id = b;  // (tensor, mode, pair)
  b /= pairs;
  const int d = (int)(b % 3);
  const int t = (int)(b / 3);
  if (t >= ntens) return;
  int ti, tj;
  gram_pair(pr, tiles, ti, tj);
  const int dims[3] = {n1, n2, n3};
  const int n = dims[d];
  if (tj * 64 >= n) return;
  const int64_t nv = (int64_t)n1 * n2 * n3;
  const int64_t no_all = nv / n;
  const int64_t chunk = ((no_all + nsplit - 1) / nsplit + OC - 1) / OC * OC;
  const int64_t obase = (int64_t)sp * chunk;
  // this workgroup's columns [obase, obase + no) of the unfolding
  const int64_t no = std::max<int64_t>(0, std::min(no_all, obase + chunk) - obase);
  const double2* At = A + (int64_t)t * nv;
  const int tid = threadIdx.x, lane = tid & 63, wr = (tid >> 6) >> 1, wc = (tid >> 6) & 1;
  v4d re[2][2], im[2][2];
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      re[u][v] = v4d{0.0, 0.0, 0.0, 0.0};
      im[u][v] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  // element e of a stage: (row i, column oc), coalesced along the unfolding's
  // contiguous index
  auto coords = [&](int e, int& i, int& oc) {
    if (d == 0) {
      i = e % 64;
      oc = e / 64;
    } else {
      oc = e % OC;
      i = e / OC;
    }
  };
  constexpr int PER = 64 * OC / 256;  // elements per thread per stage
  double2 pr_r[PER], pr_c[PER];
  auto gload = [&](int64_t o0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, oc;
      coords(tid + 256 * q, i, oc);
      const int64_t o = o0 + oc;
      const int ir = ti * 64 + i, ic = tj * 64 + i;
      pr_r[q] = (ir < n && o < no) ? At[unfold_index(d, ir, obase + o, n1, n2)]
                                   : make_double2(0, 0);
      pr_c[q] = (ic < n && o < no) ? At[unfold_index(d, ic, obase + o, n1, n2)]
                                   : make_double2(0, 0);
    }
  };
  gload(0);
  for (int64_t o0 = 0; o0 < no; o0 += OC) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int i, oc;
      coords(tid + 256 * q, i, oc);
      Xr[i][oc] = pr_r[q];
      Xc[i][oc] = pr_c[q];
    }
    __syncthreads();
    if (o0 + OC < no) gload(o0 + OC);
#pragma unroll
    for (int ks = 0; ks < OC; ks += 4) {
      const int kk = ks + (lane >> 4), rr = lane & 15;
      double2 a[2], c[2];
      for (int u = 0; u < 2; ++u) a[u] = Xr[32 * wr + 16 * u + rr][kk];
      for (int v = 0; v < 2; ++v) c[v] = Xc[32 * wc + 16 * v + rr][kk];
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
          re[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, c[v].x, re[u][v], 0, 0, 0);
          re[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, c[v].y, re[u][v], 0, 0, 0);
          im[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, c[v].x, im[u][v], 0, 0, 0);
          im[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].x, c[v].y, im[u][v], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // accumulator r of block (u, v): tile element (32 wr + 16 u + lane / 16 + 4 r,
  // 32 wc + 16 v + lane % 16)
  if (nsplit > 1) {
    double2* Pt = P + ((int64_t)sp * ntens * 3 * pairs + tile_id) * 4096;
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v)
        for (int r = 0; r < 4; ++r)
          Pt[(32 * wr + 16 * u + (lane >> 4) + 4 * r) * 64 + 32 * wc + 16 * v + (lane & 15)] =
              make_double2(re[u][v][r], im[u][v][r]);
    return;
  }
  double2* St = S + ((int64_t)d * ntens + t) * nmax * nmax;
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v)
      for (int r = 0; r < 4; ++r) {
        const int i = ti * 64 + 32 * wr + 16 * u + (lane >> 4) + 4 * r;
        const int j = tj * 64 + 32 * wc + 16 * v + (lane & 15);
        if (i < n && j < n) {
          St[(int64_t)i * n + j] = make_double2(re[u][v][r], im[u][v][r]);
          if (ti != tj) St[(int64_t)j * n + i] = make_double2(re[u][v][r], -im[u][v][r]);
        }
      }
}

// Sum of the nsplit partial tiles of gram_kernel, in split order, into S.
// One thread per tile element; grid.x = tensors * 3 * pairs * 16.
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double2* __restrict__ P,
                                                          int ntens, int n1, int n2, int n3,
                                                          int nmax, int nsplit,
                                                          double2* __restrict__ S) {
  const int tiles = (nmax + 63) / 64;
  const int pairs = tiles * (tiles + 1) / 2;
  const int64_t tile_id = blockIdx.x / 16;
  const int e = (int)(blockIdx.x % 16) * 256 + threadIdx.x;
  const int pr = (int)(tile_id % pairs);
  const int d = (int)((tile_id / pairs) % 3);
  const int t = (int)(tile_id / pairs / 3);
  if (t >= ntens) return;
  int ti, tj;
  gram_pair(pr, tiles, ti, tj);
  const int dims[3] = {n1, n2, n3};
  const int n = dims[d];
  const int i = ti * 64 + e / 64, j = tj * 64 + e % 64;
  if (tj * 64 >= n || i >= n || j >= n) return;
  const int64_t per_split = (int64_t)ntens * 3 * pairs * 4096;
  const double2* Pe = P + tile_id * 4096 + e;
  double2 s = make_double2(0.0, 0.0);
  for (int sp = 0; sp < nsplit; ++sp) {
    const double2 v = Pe[sp * per_split];
    s.x += v.x;
    s.y += v.y;
  }
  double2* St = S + ((int64_t)d * ntens + t) * nmax * nmax;
  St[(int64_t)i * n + j] = s;
  if (ti != tj) St[(int64_t)j * n + i] = make_double2(s.x, -s.y);
}

// Cyclic Jacobi for a Hermitian n x n matrix (n <= 64) in LDS.  Rounds use
// the round-robin pairing, so the n/2 rotations of a round touch disjoint
// rows/columns and are applied together as A <- J^* A J, V <- V J, where J
// is block diagonal over the round's pairs.  Entry (a, b) of A J depends only
// on row a and the pair holding column b, and J^* then mixes only the two
// rows of a pair, so each 2 x 2 block (row pair p, column pair q) of the new
// A is J_p^* A_pq J_q: one pass over the blocks per round.  For a pair (i, j)
// with A_ij = d e^{i phi} the rotation is J = [[c, s], [-s e^{-i phi},
// c e^{-i phi}]] where (c, s) diagonalise the real matrix [[A_ii, d],
// [d, A_jj]] (Golub and Van Loan's symmetric 2x2 Schur step).  Output:
// eigenvalues W (unsorted) and eigenvectors as the columns of V, per matrix.
constexpr int JT = 1024;  // threads of the Jacobi workgroup

__device__ __forceinline__ double2 jrot(double a, double2 x, double2 m, double2 y) {
  // a x + m y (a real, m complex)
  return make_double2(a * x.x + m.x * y.x - m.y * y.y, a * x.y + m.x * y.y + m.y * y.x);
}

__global__ __launch_bounds__(JT) void jacobi_kernel(JacobiBatch B) {
  extern __shared__ double2 jsm[];
  // workgroup -> (group, matrix)
  int64_t mat = blockIdx.x;
  int gi = 0;
  while (gi + 1 < B.ng && mat >= B.g[gi].nmat) {
    mat -= B.g[gi].nmat;
    ++gi;
  }
  const JacobiGroup& G = B.g[gi];
  const int n = G.n;
  const int64_t stride = G.stride, wstride = G.wstride, vstride = G.vstride;
  const double2* __restrict__ S = G.S;
  double* __restrict__ W = G.W;
  double2* __restrict__ Vout = G.V;
  const int max_sweeps = B.max_sweeps;
  const int np = n + (n & 1);
  const int half = np / 2;
  double2* A = jsm;              // n x n, row-major
  double2* V = A + n * n;        // n x n
  double2* prm = V + n * n;      // per pair: (c, s), (cos phi, sin phi)
  int2* pij = reinterpret_cast<int2*>(prm + 64);     // per pair: (i, j or -1)
  double* red = reinterpret_cast<double*>(pij + 32);  // [2][JT / 64]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double2* Sm = S + mat * stride;
  for (int e = tid; e < n * n; e += JT) {
    A[e] = Sm[e];
    V[e] = make_double2((e / n) == (e % n) ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += JT) {
      const double2 v = A[e];
      const double a2 = v.x * v.x + v.y * v.y;
      if (e / n == e % n) dia += a2;
      else off += a2;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o);
      dia += __shfl_down(dia, o);
    }
    if (lane == 0) {
      red[wv] = off;
      red[JT / 64 + wv] = dia;
    }
    __syncthreads();
    double offs = 0.0, dias = 0.0;
    for (int w = 0; w < JT / 64; ++w) {
      offs += red[w];
      dias += red[JT / 64 + w];
    }
    // rotations below 1e-15 of the matrix norm only churn rounding noise
    // (Gram matrices of low multilinear rank have many near-zero diagonal
    // entries, where a threshold relative to sqrt(a_ii a_jj) never settles);
    // the sweeps end once every off-diagonal entry is below that
    const double skip2 = 1e-30 * (offs + dias);
    const bool done = !(offs > (double)n * n * skip2);
    __syncthreads();
    if (done) break;
    for (int round = 0; round < np - 1; ++round) {
      if (tid < half) {
        int i, j;
        if (tid == 0) {
          i = np - 1;
          j = round;
        } else {
          i = (round + tid) % (np - 1);
          j = (round - tid + (np - 1)) % (np - 1);
        }
        if (i > j) {
          const int tmp = i;
          i = j;
          j = tmp;
        }
        double c = 1.0, s = 0.0, cp = 1.0, sp = 0.0;
        if (j < n) {
          const double2 aij = A[i * n + j];
          const double d2 = aij.x * aij.x + aij.y * aij.y;
          const double aii = A[i * n + i].x, ajj = A[j * n + j].x;
          const double dd = sqrt(d2);
          if (dd > 1e-300 && d2 > 1e-34 * fabs(aii * ajj) && d2 > skip2) {
            const double inv = 1.0 / dd;
            cp = aij.x * inv;
            sp = aij.y * inv;
            const double tau = (ajj - aii) * (0.5 * inv);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        prm[2 * tid] = make_double2(c, s);
        prm[2 * tid + 1] = make_double2(cp, sp);
        pij[tid] = make_int2(i, j < n ? j : -1);
      }
      __syncthreads();
      // 2 x 2 blocks: A_pq <- J_p^* A_pq J_q; a pair with no partner (odd n)
      // holds one index and no rotation
      for (int e = tid; e < half * half; e += JT) {
        const int p = e / half, q = e % half;
        const int2 Pp = pij[p], Pq = pij[q];
        const int ip = Pp.x, jp = Pp.y, iq = Pq.x, jq = Pq.y;
        const double2 csq = prm[2 * q], eq = prm[2 * q + 1];
        const double2 csp = prm[2 * p], ep = prm[2 * p + 1];
        const double cq = csq.x, sq = csq.y, cpq = eq.x, spq = eq.y;
        // columns: (x, y) -> (c x - s e^{-i phi} y, s x + c e^{-i phi} y)
        const double2 m1 = make_double2(-sq * cpq, sq * spq);
        const double2 m2 = make_double2(cq * cpq, -cq * spq);
        const double2 z = make_double2(0.0, 0.0);
        double2 x0 = A[ip * n + iq], y0 = jq >= 0 ? A[ip * n + jq] : z;
        double2 x1 = jp >= 0 ? A[jp * n + iq] : z;
        double2 y1 = (jp >= 0 && jq >= 0) ? A[jp * n + jq] : z;
        const double2 X0 = jrot(cq, x0, m1, y0), Y0 = jrot(sq, x0, m2, y0);
        const double2 X1 = jrot(cq, x1, m1, y1), Y1 = jrot(sq, x1, m2, y1);
        // rows: (x, y) -> (c x - s e^{i phi} y, s x + c e^{i phi} y)
        const double cpp = csp.x, spp = csp.y, cpr = ep.x, cpi = ep.y;
        const double2 n1 = make_double2(-spp * cpr, -spp * cpi);
        const double2 n2 = make_double2(cpp * cpr, cpp * cpi);
        A[ip * n + iq] = jrot(cpp, X0, n1, X1);
        if (jq >= 0) A[ip * n + jq] = jrot(cpp, Y0, n1, Y1);
        if (jp >= 0) {
          A[jp * n + iq] = jrot(spp, X0, n2, X1);
          if (jq >= 0) A[jp * n + jq] = jrot(spp, Y0, n2, Y1);
        }
      }
      // V <- V J
      for (int e = tid; e < half * n; e += JT) {
        const int q = e / n, r = e % n;
        const int2 Pq = pij[q];
        if (Pq.y < 0) continue;
        const double2 cs = prm[2 * q], ph = prm[2 * q + 1];
        const double2 m1 = make_double2(-cs.y * ph.x, cs.y * ph.y);
        const double2 m2 = make_double2(cs.x * ph.x, -cs.x * ph.y);
        const double2 x = V[r * n + Pq.x], y = V[r * n + Pq.y];
        V[r * n + Pq.x] = jrot(cs.x, x, m1, y);
        V[r * n + Pq.y] = jrot(cs.y, x, m2, y);
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += JT) W[mat * wstride + i] = A[i * n + i].x;
  double2* Vm = Vout + mat * vstride;
  for (int e = tid; e < n * n; e += JT) Vm[e] = V[e];
}

size_t jacobi_lds_bytes(int n) {
  return 16 * (size_t)2 * n * n + 16 * 64 + 8 * 32 + 8 * 2 * (JT / 64);
}

// T1[t][a][o] = sum_i1 conj(U1[i1, a]) A[i1 + n1 o]; workgroup = 32 values of
// o and all a; U1 given column-major n1 x r1 at u1 + u1off[t].
__global__ __launch_bounds__(256) void proj1_kernel(const double2* __restrict__ A, int n1,
                                                    int64_t no, const double2* __restrict__ u1,
                                                    const int64_t* __restrict__ u1off,
                                                    const int* __restrict__ rk, int r1max,
                                                    double2* __restrict__ T1) {
  __shared__ double2 Us[32][65];
  __shared__ double2 As[32][33];
  const int64_t chunks = (no + 31) / 32;
  const int t = (int)(blockIdx.x / chunks);
  const int64_t o0 = (blockIdx.x % chunks) * 32;
  const int r1 = rk[3 * t];
  const int64_t nv = (int64_t)n1 * no;
  const double2* At = A + (int64_t)t * nv;
  const double2* U = u1 + u1off[t];
  const int tid = threadIdx.x;
  const int ol = tid % 32, ag = tid / 32;  // a = ag + 8 q
  double2 acc[8];
  for (int q = 0; q < 8; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int i0 = 0; i0 < n1; i0 += 32) {
    for (int e = tid; e < 32 * 64; e += 256) {
      const int i = e % 32, a = e / 32;
      Us[i][a] = (i0 + i < n1 && a < r1) ? U[(i0 + i) + (int64_t)n1 * a] : make_double2(0, 0);
    }
    for (int e = tid; e < 32 * 32; e += 256) {
      const int i = e % 32, o = e / 32;
      As[i][o] = (i0 + i < n1 && o0 + o < no) ? At[(i0 + i) + (int64_t)n1 * (o0 + o)]
                                              : make_double2(0, 0);
    }
    __syncthreads();
    for (int i = 0; i < 32; ++i) {
      const double2 av = As[i][ol];
      for (int q = 0; q < 8; ++q) acc[q] = zfma_conj_a(Us[i][ag + 8 * q], av, acc[q]);
    }
    __syncthreads();
  }
  if (o0 + ol < no)
    for (int q = 0; q < 8; ++q) {
      const int a = ag + 8 * q;
      if (a < r1) T1[((int64_t)t * r1max + a) * no + o0 + ol] = acc[q];
    }
}

// T2[t][(a, b)][i3] = sum_i2 conj(U2[i2, b]) T1[t][a][i2 + n2 i3]
__global__ void proj2_kernel(const double2* __restrict__ T1, int n2, int n3, int r1max,
                             int r2max, const double2* __restrict__ u2,
                             const int64_t* __restrict__ u2off, const int* __restrict__ rk,
                             double2* __restrict__ T2) {
  const int t = blockIdx.y;
  const int r1 = rk[3 * t], r2 = rk[3 * t + 1];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)r1 * r2 * n3;
  if (idx >= total) return;
  const int i3 = (int)(idx % n3);
  const int ab = (int)(idx / n3);
  const int a = ab % r1, b = ab / r1;
  const int64_t no = (int64_t)n2 * n3;
  const double2* src = T1 + ((int64_t)t * r1max + a) * no + (int64_t)n2 * i3;
  const double2* U = u2 + u2off[t] + (int64_t)n2 * b;
  double2 acc = make_double2(0.0, 0.0);
  for (int i2 = 0; i2 < n2; ++i2) acc = zfma_conj_a(U[i2], src[i2], acc);
  T2[((int64_t)t * r1max * r2max + a + (int64_t)r1 * b) * n3 + i3] = acc;
}

// G[t][a + r1 (b + r2 c)] = sum_i3 conj(U3[i3, c]) T2[t][(a, b)][i3]
__global__ void proj3_kernel(const double2* __restrict__ T2, int n3, int r1max, int r2max,
                             const double2* __restrict__ u3, const int64_t* __restrict__ u3off,
                             const int* __restrict__ rk, const int64_t* __restrict__ goff,
                             double2* __restrict__ G) {
  const int t = blockIdx.y;
  const int r1 = rk[3 * t], r2 = rk[3 * t + 1], r3 = rk[3 * t + 2];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= r1 * r2 * r3) return;
  const int ab = idx % (r1 * r2), c = idx / (r1 * r2);
  const double2* src = T2 + ((int64_t)t * r1max * r2max + ab) * n3;
  const double2* U = u3 + u3off[t] + (int64_t)n3 * c;
  double2 acc = make_double2(0.0, 0.0);
  for (int i3 = 0; i3 < n3; ++i3) acc = zfma_conj_a(U[i3], src[i3], acc);
  G[goff[t] + idx] = acc;
}

static tv_status last(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, what);
}

// Column ranges of the Gram products: calls with few tensors (a handful of
// workgroups) cut the unfolding's columns so that about 1024 workgroups run.
int gram_splits(int ntens, int nmax) {
  const int tiles = (nmax + 63) / 64;
  const int64_t base = (int64_t)ntens * 3 * (tiles * (tiles + 1) / 2);
  if (base >= 512) return 1;
  return (int)std::min<int64_t>(64, (1024 + base - 1) / base);
}

size_t gram_partial_count(int ntens, int nmax) {
  const int s = gram_splits(ntens, nmax);
  const int tiles = (nmax + 63) / 64;
  return s > 1 ? (size_t)s * ntens * 3 * (tiles * (tiles + 1) / 2) * 4096 : 0;
}

tv_status launch_gram(const double2* A, int ntens, int n1, int n2, int n3, int nmax, double2* S,
                      double2* P, hipStream_t st) {
  const int tiles = (nmax + 63) / 64;
  const int64_t base = (int64_t)ntens * 3 * (tiles * (tiles + 1) / 2);
  const int ns = gram_splits(ntens, nmax);
  if (ns > 1 && !P) return set_error(TV_ERR_INVALID_ARG, "gram: partial buffer missing");
  hipLaunchKernelGGL(gram_kernel, dim3((unsigned)(base * ns)), dim3(256), 0, st, A, ntens, n1,
                     n2, n3, nmax, ns, S, P);
  tv_status s = last("gram_kernel");
  if (s != TV_OK || ns == 1) return s;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)(base * 16)), dim3(256), 0, st, P, ntens,
                     n1, n2, n3, nmax, ns, S);
  return last("gram_reduce_kernel");
}

// Groups of Hermitian matrices (n <= 64 each) diagonalized in one launch,
// one workgroup per matrix: S, nmat input matrices n x n at `stride`; W, n
// eigenvalues per matrix at `wstride`; V, n x n eigenvectors per matrix at
// `vstride` (both output strides leave room for a whole matrix).
tv_status launch_jacobi_batch(const JacobiGroup* groups, int ng, hipStream_t st) {
  if (ng < 1 || ng > 3) return set_error(TV_ERR_INVALID_ARG, "jacobi: 1 to 3 groups");
  JacobiBatch B{};
  B.ng = ng;
  B.max_sweeps = 40;
  size_t lds = 0;
  int64_t blocks = 0;
  for (int g = 0; g < ng; ++g) {
    const JacobiGroup& G = groups[g];
    if (G.n < 1 || G.n > 64 || G.stride < (int64_t)G.n * G.n || G.vstride < (int64_t)G.n * G.n ||
        G.wstride < G.n || G.nmat < 1)
      return set_error(TV_ERR_INVALID_ARG, "jacobi: matrix larger than 64 or strides too small");
    B.g[g] = G;
    lds = std::max(lds, jacobi_lds_bytes(G.n));
    blocks += G.nmat;
  }
  hipError_t e = hipFuncSetAttribute((const void*)jacobi_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute(jacobi)");
  hipLaunchKernelGGL(jacobi_kernel, dim3((unsigned)blocks), dim3(JT), lds, st, B);
  return last("jacobi_kernel");
}

tv_status launch_jacobi(const double2* S, int nmat, int n, int64_t stride, double* W,
                        int64_t wstride, double2* V, int64_t vstride, hipStream_t st) {
  JacobiGroup G{S, W, V, stride, wstride, vstride, n, nmat};
  return launch_jacobi_batch(&G, 1, st);
}

tv_status launch_proj(const double2* A, int ntens, int n1, int n2, int n3, const double2* u1,
                      const double2* u2, const double2* u3, const int64_t* offs,
                      const int* ranks, int r1max, int r2max, double2* T1, double2* T2,
                      double2* G, hipStream_t st) {
  const int64_t no = (int64_t)n2 * n3;
  const int64_t chunks = (no + 31) / 32;
  hipLaunchKernelGGL(proj1_kernel, dim3((unsigned)(chunks * ntens)), dim3(256), 0, st, A, n1,
                     no, u1, offs, ranks, r1max, T1);
  tv_status s = last("proj1_kernel");
  if (s != TV_OK) return s;
  const int64_t tot2 = (int64_t)r1max * r2max * n3;
  hipLaunchKernelGGL(proj2_kernel, dim3((unsigned)((tot2 + 255) / 256), (unsigned)ntens),
                     dim3(256), 0, st, T1, n2, n3, r1max, r2max, u2, offs + ntens, ranks, T2);
  if ((s = last("proj2_kernel")) != TV_OK) return s;
  const int tot3 = r1max * r2max * TV_MAX_RANK;
  hipLaunchKernelGGL(proj3_kernel, dim3((unsigned)((tot3 + 255) / 256), (unsigned)ntens),
                     dim3(256), 0, st, T2, n3, r1max, r2max, u3, offs + 2 * ntens, ranks,
                     offs + 3 * ntens, G);
  return last("proj3_kernel");
}

}  // namespace tv

// ---------------------------------------------------------------------------
// Leading eigenpairs of the Gram matrices of modes longer than 64 (at most 64
// are ever kept): randomized range finder with one power iteration
// (Q = orth(S S Omega)), then Rayleigh-Ritz on Q^* S Q (64 x 64, Jacobi).
// All matrices are row-major, element (i, j) at [i * ld + j].
namespace tv {

// C[b] = op(A[b]) B[b]; op(A)(i, k) = A[i][k] (trans == 0) or conj(A[k][i]).
// One 32 x 32 tile of C per workgroup, K staged through LDS in chunks of 16.
__global__ __launch_bounds__(256) void zgemm_batched_kernel(
    int trans, int M, int N, int K, const double2* __restrict__ A, int lda, int64_t sA,
    const double2* __restrict__ B, int ldb, int64_t sB, double2* __restrict__ C, int ldc,
    int64_t sC, int tilesM, int tilesN) {
  __shared__ double2 As[32][17];
  __shared__ double2 Bs[16][33];
  int64_t blk = blockIdx.x;
  const int tn = (int)(blk % tilesN);
  blk /= tilesN;
  const int tm = (int)(blk % tilesM);
  const int64_t b = blk / tilesM;
  const double2* Ab = A + b * sA;
  const double2* Bb = B + b * sB;
  const int tid = threadIdx.x;
  const int ty = tid / 16, tx = tid % 16;  // outputs (2ty..2ty+1, 2tx..2tx+1)
  double2 acc[2][2];
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) acc[u][v] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 32 * 16; e += 256) {
      const int i = e / 16, kk = e % 16;
      const int gi = tm * 32 + i, gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (gi < M && gk < K) {
        if (trans == 0) {
          v = Ab[(int64_t)gi * lda + gk];
        } else {
          v = Ab[(int64_t)gk * lda + gi];
          v.y = -v.y;
        }
      }
      As[i][kk] = v;
    }
    for (int e = tid; e < 16 * 32; e += 256) {
      const int kk = e / 32, j = e % 32;
      const int gk = k0 + kk, gj = tn * 32 + j;
      Bs[kk][j] = (gk < K && gj < N) ? Bb[(int64_t)gk * ldb + gj] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int kk = 0; kk < 16; ++kk) {
      const double2 a0 = As[2 * ty][kk], a1 = As[2 * ty + 1][kk];
      const double2 b0 = Bs[kk][2 * tx], b1 = Bs[kk][2 * tx + 1];
      const double2 av[2] = {a0, a1}, bv[2] = {b0, b1};
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
          acc[u][v].x = fma(av[u].x, bv[v].x, acc[u][v].x);
          acc[u][v].x = fma(-av[u].y, bv[v].y, acc[u][v].x);
          acc[u][v].y = fma(av[u].x, bv[v].y, acc[u][v].y);
          acc[u][v].y = fma(av[u].y, bv[v].x, acc[u][v].y);
        }
    }
    __syncthreads();
  }
  double2* Cb = C + b * sC;
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int i = tm * 32 + 2 * ty + u, j = tn * 32 + 2 * tx + v;
      if (i < M && j < N) Cb[(int64_t)i * ldc + j] = acc[u][v];
    }
}

// Classical Gram-Schmidt with one reorthogonalisation pass (CGS2), column by
// column, in place on Z (n x l, row-major).  A column whose norm falls below
// 1e-13 of its norm before projection lies in the span of the previous
// ones and is set to zero.  One workgroup per matrix.
template <bool INLDS>
__global__ __launch_bounds__(256) void cgs2_kernel(Cgs2Batch B) {
  // with INLDS the matrix is staged in LDS (rows padded by one value, so a
  // thread per row reading along its row meets no bank conflict)
  extern __shared__ double2 zs[];
  __shared__ double2 c[64];
  __shared__ double2 cpart[4][64];
  __shared__ double red[2][4];
  int64_t mat = blockIdx.x;
  int gi = 0;
  while (gi + 1 < B.ng && mat >= B.g[gi].nmat) {
    mat -= B.g[gi].nmat;
    ++gi;
  }
  const int n = B.g[gi].n, l = B.l;
  double2* Zg = B.g[gi].Z + mat * B.g[gi].stride;
  const int ls = INLDS ? l + 1 : l;
  double2* Zb = INLDS ? zs : Zg;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (INLDS) {
    for (int e = tid; e < n * l; e += 256) zs[(e / l) * ls + e % l] = Zg[e];
    __syncthreads();
  }
  // workgroup sum of one value per thread (every thread calls it); the two
  // slots alternate, so one barrier per sum suffices
  int slot = 0;
  auto block_sum = [&](double v) -> double {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[slot][wv] = v;
    __syncthreads();
    const double s = (red[slot][0] + red[slot][1]) + (red[slot][2] + red[slot][3]);
    slot ^= 1;
    return s;
  };
  // Each thread owns rows i = tid, tid + 256, ... of the column being
  // orthogonalized: it updates, measures and scales only those, so the
  // barriers order just the cross-row reads (the projections' dot products).
  for (int j = 0; j < l; ++j) {
    double s = 0.0;
    for (int i = tid; i < n; i += 256) {
      const double2 v = Zb[(int64_t)i * ls + j];
      s += v.x * v.x + v.y * v.y;
    }
    const double nrm0 = sqrt(block_sum(s));
    s = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      // c[k] = sum_i conj(Q[i,k]) z[i] for k < j: thread (part, kk) sums the
      // rows i = part mod 4, then the four parts are added in order
      {
        const int kk = tid & 63, part = tid >> 6;
        double2 a = make_double2(0.0, 0.0);
        // unrolled so that the loads of several rows are in flight at once
        // (the sums keep their order)
        if (kk < j)
#pragma unroll 8
          for (int i = part; i < n; i += 4) {
            const double2 q = Zb[(int64_t)i * ls + kk], z = Zb[(int64_t)i * ls + j];
            a.x += q.x * z.x + q.y * z.y;  // conj(q) z
            a.y += q.x * z.y - q.y * z.x;
          }
        cpart[part][kk] = a;
      }
      __syncthreads();
      if (tid < j)
        c[tid] = make_double2(cpart[0][tid].x + cpart[1][tid].x + cpart[2][tid].x + cpart[3][tid].x,
                              cpart[0][tid].y + cpart[1][tid].y + cpart[2][tid].y + cpart[3][tid].y);
      __syncthreads();
      for (int i = tid; i < n; i += 256) {
        double2 z = Zb[(int64_t)i * ls + j];
#pragma unroll 8
        for (int k = 0; k < j; ++k) {
          const double2 q = Zb[(int64_t)i * ls + k], ck = c[k];
          z.x -= q.x * ck.x - q.y * ck.y;
          z.y -= q.x * ck.y + q.y * ck.x;
        }
        Zb[(int64_t)i * ls + j] = z;
        if (pass == 1) s += z.x * z.x + z.y * z.y;
      }
      if (pass == 0) __syncthreads();
    }
    const double nrm = sqrt(block_sum(s));
    const double scale = (nrm > 1e-13 * nrm0 && nrm > 1e-300) ? 1.0 / nrm : 0.0;
    for (int i = tid; i < n; i += 256) {
      const double2 v = Zb[(int64_t)i * ls + j];
      Zb[(int64_t)i * ls + j] = make_double2(v.x * scale, v.y * scale);
    }
  }
  if (INLDS) {
    __syncthreads();
    for (int e = tid; e < n * l; e += 256) Zg[e] = zs[(e / l) * ls + e % l];
  }
}

// Deterministic start block Omega (n x l, row-major, complex entries in
// [-1, 1) + i[-1, 1)) from a 32-bit integer hash of the entry index.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}
__global__ void omega_kernel(double2* __restrict__ Om, int n, int l, int64_t stride, int nmat) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * l * nmat) return;
  const int64_t b = e / ((int64_t)n * l), r = e % ((int64_t)n * l);
  const uint32_t h1 = mix32((uint32_t)(2 * r + 1)), h2 = mix32((uint32_t)(2 * r + 2) ^ 0x9e3779b9U);
  Om[b * stride + r] = make_double2(h1 * (2.0 / 4294967296.0) - 1.0, h2 * (2.0 / 4294967296.0) - 1.0);
}

__global__ void trace_kernel(const double2* __restrict__ S, int n, int64_t stride, int nmat,
                             double* __restrict__ tr) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nmat) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += S[b * stride + (int64_t)i * n + i].x;
  tr[b] = s;
}

tv_status launch_zgemm(int trans, int M, int N, int K, const double2* A, int lda, int64_t sA,
                       const double2* B, int ldb, int64_t sB, double2* C, int ldc, int64_t sC,
                       int batch, hipStream_t st) {
  const int tm = (M + 31) / 32, tn = (N + 31) / 32;
  hipLaunchKernelGGL(zgemm_batched_kernel, dim3((unsigned)((int64_t)batch * tm * tn)), dim3(256),
                     0, st, trans, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, tm, tn);
  return last("zgemm_batched_kernel");
}

// Leading l = 64 eigenpairs of nmat Hermitian n x n matrices S (n > 64).
// Outputs: W[b*l + i] eigenvalues (unsorted), U[b*n*l] eigenvectors as the
// columns of an n x l row-major matrix, tr[b] traces.  ws: 3 * nmat * n * l
// + nmat * l * l complex.
// Subspace iteration for the leading 64 eigenpairs of nmat Hermitian n x n
// matrices (n > 64), in two parts around the Rayleigh-Ritz diagonalization
// (so that the caller can batch it with other Jacobi problems): prep builds
// Q = orth(S orth(S Omega)) and T = Q^* S Q (64 x 64) in ws and the traces;
// finish forms U = Q V from T's eigenvectors V.  ws layout: Q, Z, V (n x 64
// each per matrix), T (64 x 64 per matrix).
// CGS2 over groups of n x l matrices (row-major), one workgroup per matrix;
// staged in LDS when every matrix of the batch fits
double2* subspace_T(double2* ws, int nmat, int n);
double2* subspace_V(double2* ws, int nmat, int n);

tv_status launch_cgs2(const Cgs2Group* groups, int ng, int l, hipStream_t st) {
  Cgs2Batch B{};
  B.ng = ng;
  B.l = l;
  int nmax = 0;
  int64_t blocks = 0;
  for (int g = 0; g < ng; ++g) {
    B.g[g] = groups[g];
    nmax = std::max(nmax, groups[g].n);
    blocks += groups[g].nmat;
  }
  const size_t lds = (size_t)nmax * (l + 1) * sizeof(double2);
  if (lds <= 128 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)cgs2_kernel<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute(cgs2)");
    hipLaunchKernelGGL(cgs2_kernel<true>, dim3((unsigned)blocks), dim3(256), lds, st, B);
  } else {
    hipLaunchKernelGGL(cgs2_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, B);
  }
  return last("cgs2_kernel");
}

tv_status launch_subspace_prep_batch(const SubspaceJob* jobs, int nj, int nmat, hipStream_t st) {
  const int l = 64;
  tv_status s;
  double2 *Q[3], *Z[3];
  for (int j = 0; j < nj; ++j) {
    const int n = jobs[j].n;
    const int64_t nl = (int64_t)n * l, tot = (int64_t)nmat * nl;
    Q[j] = jobs[j].ws;
    Z[j] = Q[j] + nmat * nl;
    hipLaunchKernelGGL(omega_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Q[j],
                       n, l, nl, nmat);
    if ((s = last("omega_kernel")) != TV_OK) return s;
    hipLaunchKernelGGL(trace_kernel, dim3((unsigned)((nmat + 255) / 256)), dim3(256), 0, st,
                       jobs[j].S, n, jobs[j].sS, nmat, jobs[j].tr);
    if ((s = last("trace_kernel")) != TV_OK) return s;
  }
  // Z = S Omega, Q = orth(Z); Z = S Q, Q = orth(Z) (two swaps: Q ends in ws),
  // the orthogonalizations of all jobs in one launch
  for (int it = 0; it < 2; ++it) {
    Cgs2Group cg[3];
    for (int j = 0; j < nj; ++j) {
      const int n = jobs[j].n;
      const int64_t nl = (int64_t)n * l;
      if ((s = launch_zgemm(0, n, l, n, jobs[j].S, n, jobs[j].sS, Q[j], l, nl, Z[j], l, nl, nmat,
                            st)) != TV_OK)
        return s;
      cg[j] = Cgs2Group{Z[j], nl, n, nmat};
    }
    if ((s = launch_cgs2(cg, nj, l, st)) != TV_OK) return s;
    for (int j = 0; j < nj; ++j) std::swap(Q[j], Z[j]);
  }
  // Rayleigh-Ritz matrices T = Q^* (S Q)
  for (int j = 0; j < nj; ++j) {
    const int n = jobs[j].n;
    const int64_t nl = (int64_t)n * l;
    if ((s = launch_zgemm(0, n, l, n, jobs[j].S, n, jobs[j].sS, Q[j], l, nl, Z[j], l, nl, nmat,
                          st)) != TV_OK)
      return s;
    if ((s = launch_zgemm(1, l, l, n, Q[j], l, nl, Z[j], l, nl, subspace_T(jobs[j].ws, nmat, n), l,
                          (int64_t)l * l, nmat, st)) != TV_OK)
      return s;
  }
  return TV_OK;
}

tv_status launch_subspace_prep(const double2* S, int nmat, int n, int64_t sS, double* tr,
                               double2* ws, hipStream_t st) {
  SubspaceJob j{S, sS, tr, ws, n};
  return launch_subspace_prep_batch(&j, 1, nmat, st);
}

// the 64 x 64 Rayleigh-Ritz matrices of launch_subspace_prep's workspace
double2* subspace_T(double2* ws, int nmat, int n) { return ws + (int64_t)3 * nmat * n * 64; }
double2* subspace_V(double2* ws, int nmat, int n) { return ws + (int64_t)2 * nmat * n * 64; }

tv_status launch_subspace_finish(int nmat, int n, const double2* ws, const double2* V,
                                 double2* U, hipStream_t st) {
  const int l = 64;
  const int64_t nl = (int64_t)n * l, ll = (int64_t)l * l;
  return launch_zgemm(0, n, l, l, ws, l, nl, V, l, ll, U, l, nl, nmat, st);
}

tv_status launch_subspace_eig(const double2* S, int nmat, int n, int64_t sS, double* W,
                              double2* U, double* tr, double2* ws, hipStream_t st) {
  tv_status s = launch_subspace_prep(S, nmat, n, sS, tr, ws, st);
  if (s != TV_OK) return s;
  double2* T = subspace_T(ws, nmat, n);
  double2* V = subspace_V(ws, nmat, n);
  if ((s = launch_jacobi(T, nmat, 64, 64 * 64, W, 64, V, 64 * 64, st)) != TV_OK) return s;
  return launch_subspace_finish(nmat, n, ws, V, U, st);
}

}  // namespace tv
