// Shared host/device definitions of the separable Helmholtz solver:
// complex arithmetic on HIP vector types and the per-block stage descriptors
// that the host plan builds once and the batched kernels read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hs {

template <typename R> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename R> using cplx = typename cplx_t<R>::type;

template <typename R>
__host__ __device__ __forceinline__ cplx<R> mk(R re, R im) {
  cplx<R> z;
  z.x = re;
  z.y = im;
  return z;
}
template <typename C>
__host__ __device__ __forceinline__ C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C>
__host__ __device__ __forceinline__ C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename C>
__host__ __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// acc + a * b
template <typename C>
__host__ __device__ __forceinline__ C cfma(C a, C b, C acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc - a * b
template <typename C>
__host__ __device__ __forceinline__ C cfms(C a, C b, C acc) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <typename C>
__host__ __device__ __forceinline__ C cconj(C a) { a.y = -a.y; return a; }
template <typename C, typename R>
__host__ __device__ __forceinline__ C cscale(C a, R s) { a.x *= s; a.y *= s; return a; }
// 1/z as conj(z)/|z|^2.  Used for z pivots, whose modulus the plan checks to lie
// in [1e-12, 1e12] times the operator scale, far from over- and underflow.
template <typename C>
__host__ __device__ __forceinline__ C crcp(C z) {
  auto n = z.x * z.x + z.y * z.y;
  auto inv = decltype(n)(1) / n;
  C r;
  r.x = z.x * inv;
  r.y = -z.y * inv;
  return r;
}

// ---------------------------------------------------------------------------
// Stage descriptors.  Offsets are in complex elements relative to base pointers
// passed to each launch, so one descriptor table serves every call of a plan.
// ---------------------------------------------------------------------------

// Dense transform along a contiguous axis: for lines (p, q) of one RHS r,
//   dst[r*dst_r + p*dst_p + q*dst_q + o] = scale * sum_k T[o*n_in + k] * src[r*src_r + p*src_p + q*src_q + k]
struct XformDesc {
  int64_t tab;      // offset of the n_out x n_in table (row-major) in the table buffer
  int32_t n_in, n_out;
  int32_t P, Q;     // line index ranges
  int64_t src, src_r, src_p, src_q;
  int64_t dst, dst_r, dst_p, dst_q;
  int32_t sine;     // 1: table is the real orthonormal sine matrix (imaginary part zero)
  int32_t real_tab; // 1: ftab holds the real table itself, 0: its real embedding
  int64_t ftab;     // offset of the same table as MFMA fragments (see xform_mfma.hip)
  int64_t htab = -1;   // complex64 path: offset (16-byte units) of its split-fp16 fragments, -1 if none
  float hsinv = 1.f;   // 1 / the power-of-two scale of those fragments (see xform_h3.hip)
  int32_t pad_ = 0;
};

// Dense transform along a strided axis, in place: for plane p of RHS r and
// column c (contiguous), data[o][c] = sum_k T[o][k] data[k][c] (n_in == n_out).
struct XformYDesc {
  int64_t tab;
  int32_t n, ncols;
  int32_t P, real_tab;   // real_tab: as in XformDesc
  int64_t data, s_r, s_p, s_k;
  int64_t ftab;     // offset of the same table as MFMA fragments
  int64_t htab = -1;   // as in XformDesc
  float hsinv = 1.f;
  int32_t pad_ = 0;
};

// Orthonormal sine transform (DST-I, n = N - 1 points, N a power of two) of
// lines (p, q) of one RHS r; element i of a line sits at
//   base + r*_r + p*_p + q*_q + i*_i      (for src and dst separately).
// Used on uniform axes in place of the dense table (same matrix).
struct DstDesc {
  int32_t n, P, Q, pad_;
  int64_t src, src_r, src_p, src_q, src_i;
  int64_t dst, dst_r, dst_p, dst_q, dst_i;
};

// One batched z sweep over the (a, b) modes of a block.
//  rhs(a,b,z,r) = [dense_in ? data(r,z,b,a) : 0]
//               + sum_i colx_i[a] * gx_i(r,z,b) + sum_j coly_j[b] * gy_j(r,z,a)
//  (Dz - diag k^2 + (lam_x[a] + lam_y[b]) diag sigma) x = rhs,   out(r,z,b,a) = x
// element (r,z,b,a) of data / out sits at base + r*_r + z*plane + b*rs + a
// (rows and z planes may be padded, rs >= na and plane >= nb*rs, so that
// tiles of modes start on whole cache lines).
constexpr int kMaxTerms = 4;
// separators of each axis per interface-contraction descriptor (one read of
// the global spectral array serves this many)
constexpr int kMaxContractTerms = 8;
constexpr int kMaxRefine = 16;   // refinement steps of the complex64 path
struct SweepDesc {
  int32_t na, nb, nz, dense_in;
  int32_t nxt, nyt, rs, pad1_;    // rs: row stride of data and out
  double fp64_below;              // complex64 path: modes with Re(lam_x + lam_y) <= this solve in FP64
  int64_t lam_x, lam_y;           // table offsets (complex, length na / nb)
  int64_t zlo, zdiag, zup;        // table offsets (complex, length nz)
  int64_t zsig;                   // table offset of sigma at the z nodes (real parts), scaling the shift
  int64_t data, data_r;           // workspace offsets
  int64_t out, out_r;
  int64_t colx[kMaxTerms]; int32_t colx_stride[kMaxTerms];   // table offsets
  int64_t gx[kMaxTerms];          // workspace offsets
  int64_t coly[kMaxTerms]; int32_t coly_stride[kMaxTerms];
  int64_t gy[kMaxTerms];
  int64_t gx_r, gy_r, gx_z, gy_z;   // gx(r,z,b) = gx + r*gx_r + z*gx_z + b
  int64_t plane;                    // z-plane stride of data and out
};

// Contraction of a spectral array X(r,z,b,a) = src + r*src_r + z*plane + b*rs + a
// along both axes in one read, with up to kMaxTerms coefficient vectors each:
//   out_x,t(r,z,b) = sum_a cx_t[a] X(r,z,b,a)   at dx + t*dx_t + r*dx_r + z*dx_z + b
//   out_y,t(r,z,a) = sum_b cy_t[b] X(r,z,b,a)   at dy + t*dy_t + r*dy_r + z*dy_z + a
// A z plane is split into nslab slabs of `rows` rows b and ncs slabs of
// `cols` columns a.  With nslab > 1 the y sums of each row slab go to
//   part + r*part_r + s*part_s + t*part_t + z*part_z + a,
// with ncs > 1 the x sums of each column slab go to
//   xpart + r*xpart_r + c*xpart_s + t*xpart_t + z*xpart_z + b,
// and a second pass adds the slabs in order.
struct ContractDesc {
  int32_t na, nb, nz, nxt, nyt, nslab, rows, ncs;
  int32_t cols, rs;               // rs: row stride of X (>= na)
  int64_t src, src_r;
  int64_t cx[kMaxContractTerms], cy[kMaxContractTerms];   // table offsets
  int32_t cx_stride[kMaxContractTerms], cy_stride[kMaxContractTerms];
  int64_t dx, dx_t, dx_r, dx_z;
  int64_t dy, dy_t, dy_r, dy_z;
  int64_t part, part_s, part_t, part_r, part_z;
  int64_t xpart, xpart_s, xpart_t, xpart_r, xpart_z;
  int64_t plane;                  // z-plane stride of X (>= na*nb)
};

// Dense spectral right-hand side of the global interface solve, for
// separator counts above kMaxTerms (too many to add inside the z solve):
//   out(r,z,b,a) = sum_i cx[i*na + a] gx_i(r,z,b) + sum_j cy[j*nb + b] gy_j(r,z,a)
// with gx_i(r,z,b) at gx + r*gx_r + i*gx_t + z*gx_z + b (gy_j likewise with a),
// out(r,z,b,a) at out + r*out_r + z*plane + b*rs + a; cx, cy are table offsets.
struct ExpandDesc {
  int32_t na, nb, nz, nxt, nyt, rs;
  int64_t cx, cy;
  int64_t gx, gx_t, gx_r, gx_z;
  int64_t gy, gy_t, gy_r, gy_z;
  int64_t out, out_r, plane;
};

}  // namespace hs
