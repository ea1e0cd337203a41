// Synthetic coupling-matrix columns on the device, FP64.
//
// Stand-in for the MoM assembly (Sec. II.A.1): the coil element of column j
// is a unit point current p_j at r_j, and the E-field operator of eq. (2)
// with the Green's function of eq. (3), g = exp(-i k0 R) / (4 pi R), gives
//   E(r) = (grad grad + k0^2) g p
//        = k0^2 g [ (1 - i/(k0R) - 1/(k0R)^2) p + (-1 + 3i/(k0R) + 3/(k0R)^2) (Rh.p) Rh ]
// with R = r - r_j, Rh = R / |R|.  PWC voxels take the value at the centre;
// PWL voxels project on {1, (x - xc)/h, (y - yc)/h, (z - zc)/h} with the
// 2x2x2 Gauss-Legendre rule, divided by the voxel volume.
// The magnetic coupling matrix (K operator of eq. 5) takes instead
//   H(r) = curl(g p) = grad g x p = g (-i k0 - 1/R) Rh x p
// on the same voxel bases.  `basis` bit 0 selects PWL, bit 1 the K operator.
#include <algorithm>

#include "tv_internal.h"

namespace tv {

struct ColParams {
  int n1, n2, n3;
  double h, k0;
  int basis;      // 0 PWC, 1 PWL
  int op;         // 0 E-field (eq. 2), 1 H-field (eq. 5)
  int64_t ncols;
  const double* src;  // device [ncols][6]: position then orientation
  double2* out;
  int64_t ldo;        // rows kernel: output stride between rows
};

__device__ inline void point_field(double x, double y, double z, const double* s, double k0,
                                   double2 E[3]) {
  const double dx = x - s[0], dy = y - s[1], dz = z - s[2];
  const double R = sqrt(dx * dx + dy * dy + dz * dz);
  const double inv = 1.0 / R;
  const double hx = dx * inv, hy = dy * inv, hz = dz * inv;
  const double kr = k0 * R, ikr = 1.0 / kr, ikr2 = ikr * ikr;
  double sn, cs;
  sincos(kr, &sn, &cs);
  // k0^2 g = k0^2 (cos kR - i sin kR) / (4 pi R)
  const double amp = k0 * k0 * inv * 0.07957747154594767;  // 1/(4 pi)
  const double gr = amp * cs, gi = -amp * sn;
  // a = (1 - ikr2) - i ikr ; b = (-1 + 3 ikr2) + 3 i ikr
  const double ar = 1.0 - ikr2, ai = -ikr;
  const double br = -1.0 + 3.0 * ikr2, bi = 3.0 * ikr;
  const double rp = hx * s[3] + hy * s[4] + hz * s[5];
  const double hv[3] = {hx, hy, hz};
  for (int c = 0; c < 3; ++c) {
    const double tr = ar * s[3 + c] + br * rp * hv[c];
    const double ti = ai * s[3 + c] + bi * rp * hv[c];
    E[c] = make_double2(gr * tr - gi * ti, gr * ti + gi * tr);
  }
}

__device__ inline void point_hfield(double x, double y, double z, const double* s, double k0,
                                    double2 H[3]) {
  const double dx = x - s[0], dy = y - s[1], dz = z - s[2];
  const double R = sqrt(dx * dx + dy * dy + dz * dz);
  const double inv = 1.0 / R;
  const double hx = dx * inv, hy = dy * inv, hz = dz * inv;
  double sn, cs;
  sincos(k0 * R, &sn, &cs);
  const double amp = inv * 0.07957747154594767;  // 1/(4 pi R)
  const double gr = amp * cs, gi = -amp * sn;
  // dg/dR = g (-1/R - i k0)
  const double dr = -gr * inv + gi * k0, di = -gi * inv - gr * k0;
  const double w[3] = {hy * s[5] - hz * s[4], hz * s[3] - hx * s[5], hx * s[4] - hy * s[3]};
  for (int c = 0; c < 3; ++c) H[c] = make_double2(dr * w[c], di * w[c]);
}

__device__ inline void field(int op, double x, double y, double z, const double* s, double k0,
                             double2 F[3]) {
  if (op == 0)
    point_field(x, y, z, s, k0, F);
  else
    point_hfield(x, y, z, s, k0, F);
}

// Up to kChunk sources (and rows) passed by value in the kernel arguments,
// so that the public entry points need no device staging buffer.
constexpr int kChunk = 32;
struct SrcChunk {
  double src[kChunk * 6];
  int64_t rows[kChunk];
};

template <bool ARGS>
__global__ void columns_kernel(ColParams P, SrcChunk C) {
  const int64_t nv = (int64_t)P.n1 * P.n2 * P.n3;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (v >= nv || j >= P.ncols) return;
  const int i1 = (int)(v % P.n1);
  const int i2 = (int)((v / P.n1) % P.n2);
  const int i3 = (int)(v / ((int64_t)P.n1 * P.n2));
  const double cx = (i1 - 0.5 * (P.n1 - 1)) * P.h;
  const double cy = (i2 - 0.5 * (P.n2 - 1)) * P.h;
  const double cz = (i3 - 0.5 * (P.n3 - 1)) * P.h;
  __shared__ double s[6];
  if (threadIdx.x < 6) s[threadIdx.x] = ARGS ? C.src[j * 6 + threadIdx.x] : P.src[j * 6 + threadIdx.x];
  __syncthreads();
  if (P.basis == 0) {
    double2 E[3];
    field(P.op, cx, cy, cz, s, P.k0, E);
    for (int c = 0; c < 3; ++c) P.out[(j * 3 + c) * nv + v] = E[c];
    return;
  }
  // PWL: tensor 4c + l, nodes at centre +- h/(2 sqrt 3) per axis, weight 1/8
  const double off = 0.28867513459481287;  // 1 / (2 sqrt 3)
  double2 acc[12];
  for (int i = 0; i < 12; ++i) acc[i] = make_double2(0.0, 0.0);
  for (int q = 0; q < 8; ++q) {
    const double ux = (q & 1) ? off : -off;
    const double uy = (q & 2) ? off : -off;
    const double uz = (q & 4) ? off : -off;
    double2 E[3];
    field(P.op, cx + ux * P.h, cy + uy * P.h, cz + uz * P.h, s, P.k0, E);
    const double phi[4] = {0.125, 0.125 * ux, 0.125 * uy, 0.125 * uz};
    for (int c = 0; c < 3; ++c)
      for (int l = 0; l < 4; ++l) {
        acc[4 * c + l].x += E[c].x * phi[l];
        acc[4 * c + l].y += E[c].y * phi[l];
      }
  }
  for (int t = 0; t < 12; ++t) P.out[(j * 12 + t) * nv + v] = acc[t];
}

// Row `row` of the coupling matrix, one source j per lane: the field of
// every coil element at one voxel v and tensor index k (row = k nv + v, the
// row order of Algorithm 1).  Same closed form and quadrature as the columns.
template <bool ARGS>
__global__ void rows_kernel(ColParams P, const int64_t* rows, SrcChunk C) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P.ncols) return;
  const int64_t nv = (int64_t)P.n1 * P.n2 * P.n3;
  const int64_t row = ARGS ? C.rows[blockIdx.y] : rows[blockIdx.y];
  const int k = (int)(row / nv);
  const int64_t v = row - (int64_t)k * nv;
  const int i1 = (int)(v % P.n1);
  const int i2 = (int)((v / P.n1) % P.n2);
  const int i3 = (int)(v / ((int64_t)P.n1 * P.n2));
  const double cx = (i1 - 0.5 * (P.n1 - 1)) * P.h;
  const double cy = (i2 - 0.5 * (P.n2 - 1)) * P.h;
  const double cz = (i3 - 0.5 * (P.n3 - 1)) * P.h;
  double s[6];
  for (int c = 0; c < 6; ++c) s[c] = ARGS ? C.src[j * 6 + c] : P.src[j * 6 + c];
  double2* out = P.out + (int64_t)blockIdx.y * P.ldo + j;
  if (P.basis == 0) {
    double2 E[3];
    field(P.op, cx, cy, cz, s, P.k0, E);
    *out = E[k];
    return;
  }
  const int c = k / 4, l = k % 4;
  const double off = 0.28867513459481287;  // 1 / (2 sqrt 3)
  double2 acc = make_double2(0.0, 0.0);
  for (int q = 0; q < 8; ++q) {
    const double u[3] = {(q & 1) ? off : -off, (q & 2) ? off : -off, (q & 4) ? off : -off};
    double2 E[3];
    field(P.op, cx + u[0] * P.h, cy + u[1] * P.h, cz + u[2] * P.h, s, P.k0, E);
    const double phi = l == 0 ? 0.125 : 0.125 * u[l - 1];
    acc.x += E[c].x * phi;
    acc.y += E[c].y * phi;
  }
  *out = acc;
}

// Sources as [n][6] (position, orientation), checked to lie outside the
// voxel domain and to have unit orientations.
tv_status stage_sources(int n1, int n2, int n3, double h, int64_t n, const double* pos,
                        const double* ori, std::vector<double>& src) {
  const double half[3] = {0.5 * (n1 - 1) * h, 0.5 * (n2 - 1) * h, 0.5 * (n3 - 1) * h};
  src.assign((size_t)n * 6, 0.0);
  for (int64_t j = 0; j < n; ++j) {
    double d2 = 0.0, on = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double p = pos[3 * j + c];
      const double nearest = p < -half[c] ? -half[c] : (p > half[c] ? half[c] : p);
      d2 += (p - nearest) * (p - nearest);
      on += ori[3 * j + c] * ori[3 * j + c];
      src[6 * j + c] = p;
      src[6 * j + 3 + c] = ori[3 * j + c];
    }
    if (!(d2 > (0.25 * h) * (0.25 * h)))
      return set_error(TV_ERR_INVALID_ARG, "a source lies inside the voxel domain");
    if (!(fabs(on - 1.0) < 1e-9)) return set_error(TV_ERR_INVALID_ARG, "orientation not unit");
  }
  return TV_OK;
}

tv_status launch_dipole_columns(int n1, int n2, int n3, double h, double k0, int basis,
                                int64_t ncols, const double* d_src, double2* out,
                                hipStream_t st) {
  const int64_t nv = (int64_t)n1 * n2 * n3;
  ColParams P{n1, n2, n3, h, k0, basis & 1, basis >> 1, ncols, d_src, out, 0};
  SrcChunk C{};
  hipLaunchKernelGGL(columns_kernel<false>, dim3((unsigned)((nv + 255) / 256), (unsigned)ncols),
                     dim3(256), 0, st, P, C);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "columns kernel launch");
}

tv_status launch_dipole_rows(int n1, int n2, int n3, double h, double k0, int basis,
                             int64_t nsrc, const double* d_src, int64_t nrows,
                             const int64_t* d_rows, double2* out, hipStream_t st) {
  ColParams P{n1, n2, n3, h, k0, basis & 1, basis >> 1, nsrc, d_src, out, nsrc};
  SrcChunk C{};
  hipLaunchKernelGGL(rows_kernel<false>, dim3((unsigned)((nsrc + 255) / 256), (unsigned)nrows),
                     dim3(256), 0, st, P, d_rows, C);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TV_OK : hip_error(e, "rows kernel launch");
}

}  // namespace tv

using namespace tv;

extern "C" tv_status tv_dipole_rows(int32_t n1, int32_t n2, int32_t n3, double h, double k0,
                                    int32_t basis, int64_t nsrc, const double* pos,
                                    const double* ori, int64_t nrows, const int64_t* rows,
                                    void* out, void* stream) {
  clear_error();
  if (n1 < 1 || n2 < 1 || n3 < 1 || nsrc < 1 || nrows < 0)
    return set_error(TV_ERR_SHAPE, "grid sizes and nsrc must be >= 1, nrows >= 0");
  if (!(h > 0.0) || !(k0 > 0.0)) return set_error(TV_ERR_INVALID_ARG, "h and k0 must be > 0");
  if (basis < 0 || basis > 3) return set_error(TV_ERR_INVALID_ARG, "basis must be in 0..3");
  if (nrows == 0) return TV_OK;
  if (!pos || !ori || !rows || !out) return set_error(TV_ERR_INVALID_ARG, "NULL pointer");
  if (nrows > 65535) return set_error(TV_ERR_NOT_SUPPORTED, "at most 65535 rows per call");
  const int64_t total = (int64_t)((basis & 1) ? 12 : 3) * n1 * n2 * n3;
  for (int64_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= total) return set_error(TV_ERR_SHAPE, "row index out of range");
  std::vector<double> src;
  tv_status s = stage_sources(n1, n2, n3, h, nsrc, pos, ori, src);
  if (s != TV_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  // sources and rows in chunks of kChunk through the kernel arguments
  for (int64_t r0 = 0; r0 < nrows; r0 += kChunk) {
    const int nr = (int)std::min<int64_t>(kChunk, nrows - r0);
    for (int64_t j0 = 0; j0 < nsrc; j0 += kChunk) {
      const int nj = (int)std::min<int64_t>(kChunk, nsrc - j0);
      SrcChunk C{};
      std::copy(src.begin() + 6 * j0, src.begin() + 6 * (j0 + nj), C.src);
      std::copy(rows + r0, rows + r0 + nr, C.rows);
      ColParams P{n1, n2, n3, h, k0, basis & 1, basis >> 1, nj, nullptr,
                  (double2*)out + r0 * nsrc + j0, nsrc};
      hipLaunchKernelGGL(rows_kernel<true>, dim3(1, (unsigned)nr), dim3(kChunk), 0, st, P,
                         (const int64_t*)nullptr, C);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_error(e, "rows kernel launch");
    }
  }
  hipError_t e = hipStreamSynchronize(st);
  return e == hipSuccess ? TV_OK : hip_error(e, "tv_dipole_rows");
}

extern "C" tv_status tv_dipole_columns(int32_t n1, int32_t n2, int32_t n3, double h, double k0,
                                       int32_t basis, int64_t ncols, const double* pos,
                                       const double* ori, void* out, void* stream) {
  clear_error();
  if (n1 < 1 || n2 < 1 || n3 < 1 || ncols < 0)
    return set_error(TV_ERR_SHAPE, "grid sizes must be >= 1 and ncols >= 0");
  if (!(h > 0.0) || !(k0 > 0.0)) return set_error(TV_ERR_INVALID_ARG, "h and k0 must be > 0");
  if (basis < 0 || basis > 3) return set_error(TV_ERR_INVALID_ARG, "basis must be in 0..3");
  if (ncols == 0) return TV_OK;
  if (!pos || !ori || !out) return set_error(TV_ERR_INVALID_ARG, "NULL pointer");
  if (ncols > 65535) return set_error(TV_ERR_NOT_SUPPORTED, "at most 65535 columns per call");
  const int64_t nv = (int64_t)n1 * n2 * n3;
  // every voxel centre must be away from every source
  std::vector<double> src;
  tv_status s0 = stage_sources(n1, n2, n3, h, ncols, pos, ori, src);
  if (s0 != TV_OK) return s0;
  hipStream_t st = (hipStream_t)stream;
  // sources in chunks of kChunk through the kernel arguments
  for (int64_t j0 = 0; j0 < ncols; j0 += kChunk) {
    const int nj = (int)std::min<int64_t>(kChunk, ncols - j0);
    SrcChunk C{};
    std::copy(src.begin() + 6 * j0, src.begin() + 6 * (j0 + nj), C.src);
    ColParams P{n1, n2, n3, h, k0, basis & 1, basis >> 1, nj, nullptr,
                (double2*)out + j0 * ((basis & 1) ? 12 : 3) * nv, 0};
    hipLaunchKernelGGL(columns_kernel<true>, dim3((unsigned)((nv + 255) / 256), (unsigned)nj),
                       dim3(256), 0, st, P, C);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "columns kernel launch");
  }
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  return TV_OK;
}
