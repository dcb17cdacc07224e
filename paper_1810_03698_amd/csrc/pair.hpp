// Far-field pair terms of the four boundary-integral kernels, shared by the
// forward and transposed source-target products and by the near/self
// correction.  The correction subtracts exactly the value the product added
// (same inputs, same operation sequence, no contraction), so that for tiny
// panels the rounding of the pair terms cancels instead of being amplified
// by 1/r^3.
#pragma once

#include <hip/hip_runtime.h>

namespace pbmp {

// FP32 cut-off on r^2 (r < 1e-4 A): such a pair adds nothing.  Pairs that
// close only occur between a panel and itself (the one-node rule puts the
// node on the centroid) or a near neighbour, and the near correction removes
// exactly the value the product added, so skipping them is exact; it keeps
// coincident FP32 points finite without 1/r-sized terms in FP32 sums.
constexpr float kMinR2f = 1e-8f;
// The FP64 products skip pairs closer than 1e-10 A: only a one-node rule's
// node on its own panel's centroid comes that close (the node and the
// centroid are computed with different roundings, so they need not
// coincide exactly), since a node is at least a sixth of an altitude from
// every other panel's centroid.
constexpr double kMinR2d = 1e-20;

// Reciprocal distance and screened reciprocal distance of one far-field
// node for the difference R = p - y = (dx,dy,dz): ri = 1/r, er = e^{-k r}/r.
// nk = -k log2(e).  FLOOR: ri = er = 0 below the cut-off.
template <bool FLOOR = true>
__device__ __forceinline__ void node_core(float dx, float dy, float dz, float nk,
                                          float &ri, float &er) {
#pragma clang fp contract(off)
  const float rr = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  ri = __builtin_amdgcn_rsqf(rr);
  if (FLOOR) ri = rr < kMinR2f ? 0.0f : ri;
  const float ek = __builtin_amdgcn_exp2f(nk * (rr * ri));
  er = ek * ri;
}

// Adds one node's terms: vl += 1/r, vy += e^{-kr}/r, kl += 1/r^3,
// ky += (1 + k r) e^{-k r}/r^3 (as e/r^3 + k e/r^2).
__device__ __forceinline__ void node_terms(float dx, float dy, float dz,
                                           float kappa, float nk, float &vl,
                                           float &vy, float &kl, float &ky) {
#pragma clang fp contract(off)
  float ri, er;
  node_core<true>(dx, dy, dz, nk, ri, er);
  const float ri2 = ri * ri;
  vl = vl + ri;
  vy = vy + er;
  kl = fmaf(ri2, ri, kl);
  ky = fmaf(er, ri2, fmaf(kappa * er, ri, ky));
}

// 1/sqrt(rr) in FP64: the hardware estimate (v_rsq_f64) refined by two
// Newton steps y <- y + y (1 - rr y^2) / 2, each of which squares the
// relative error, so the result is within an ulp or two of the exact
// value; a square root and a division would take three times the
// instructions.  rr must be positive and normal.
__device__ __forceinline__ double rsqrt_fp64(double rr) {
  double y = __builtin_amdgcn_rsq(rr);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-rr, y * y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// e^x in FP64 for x <= 0 (the screening factor e^{-kappa r}; no overflow
// or NaN handling).  Cody-Waite reduction x = n ln2 + f, |f| <= ln2/2, with
// ln2 split into a 32-bit head (n * head is exact for |n| < 2^21) and the
// rounded tail; e^f by its Taylor series to degree 13 (remainder below
// 0.35^14/14! < 5e-18) in Horner form; then scaled by 2^n (e^x below the
// smallest subnormal comes out as zero).
__device__ __forceinline__ double exp_fp64(double x) {
  constexpr double kLog2e = 1.4426950408889634;
  constexpr double kLn2Hi = 0x1.62e42ffp-1;
  constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
  const double n = rint(x * kLog2e);
  double f = fma(-n, kLn2Hi, x);
  f = fma(-n, kLn2Lo, f);
  constexpr double kFact[14] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0,
                                362880.0, 3628800.0, 39916800.0, 479001600.0,
                                6227020800.0};
  double p = 1.0 / kFact[13];
#pragma unroll
  for (int k = 12; k >= 0; --k) p = fma(p, f, 1.0 / kFact[k]);
  return ldexp(p, (int)n);
}

__device__ __forceinline__ void node_terms(double dx, double dy, double dz,
                                           double kappa, double, double &vl,
                                           double &vy, double &kl, double &ky) {
#pragma clang fp contract(off)
  const double rr = dx * dx + dy * dy + dz * dz;
  // a node on the target (the one-node rule on a panel's own centroid)
  // adds nothing, here and in the correction that removes it again
  const bool on = rr < kMinR2d;
  const double y = rsqrt_fp64(on ? 1.0 : rr);
  const double ri = on ? 0.0 : y;
  const double rad = rr * y;
  const double ek = exp_fp64(-kappa * rad);
  const double ri3 = ri * ri * ri;
  vl = vl + ri;
  vy = vy + ek * ri;
  kl = kl + ri3;
  ky = ky + (1.0 + kappa * rad) * ek * ri3;
}

// n.(p - y0): the nodes of a flat panel share its plane, so this is n.R
// for every node; taken from the difference vector (error eps |p - y0|).
__device__ __forceinline__ float normal_dist(float nx, float ny, float nz,
                                             float dx, float dy, float dz) {
#pragma clang fp contract(off)
  return fmaf(nx, dx, fmaf(ny, dy, nz * dz));
}

__device__ __forceinline__ double normal_dist(double nx, double ny, double nz,
                                              double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return nx * dx + ny * dy + nz * dz;
}

// Sums of one panel (nf nodes from a 16-word record) at target p, as the
// products weight them: out = (vl, n.R kl, vy, n.R ky) before the strengths.
template <class T>
__device__ __forceinline__ void panel_terms(const T *rec, int nf, T px, T py,
                                            T pz, T kappa, T nk, T out[4]) {
  T vl = T(0), vy = T(0), kl = T(0), ky = T(0);
  T d0[3] = {T(0), T(0), T(0)};
  for (int q = 0; q < nf; ++q) {
    const T dx = px - rec[3 * q], dy = py - rec[3 * q + 1], dz = pz - rec[3 * q + 2];
    if (q == 0) {
      d0[0] = dx;
      d0[1] = dy;
      d0[2] = dz;
    }
    node_terms(dx, dy, dz, kappa, nk, vl, vy, kl, ky);
  }
  const T nR = normal_dist(rec[9], rec[10], rec[11], d0[0], d0[1], d0[2]);
  out[0] = vl;
  out[1] = nR * kl;
  out[2] = vy;
  out[3] = nR * ky;
}

// Far-rule pair function of the operator for R = c_i - y (one node):
//   f = a1 n.R/r^3 - a2/r - a3 n.R (1 + k r) e/r^3 + a4 e/r,  e = e^{-k r}
// with a1 = l1_i phi_j, a2 = l1_i dphi_j, a3 = l2_i phi_j, a4 = eps l2_i dphi_j
// (the pair's share of lambda_x . A x; with the panel's packed strengths
// s_K, s_V in place of phi_j, dphi_j the weight and area are included).
// Returns f, df/dR, df/dn.
__device__ inline double op_pair(const double R[3], const double n[3], double kappa,
                                 double a1, double a2, double a3, double a4, double gR[3],
                                 double gn[3]) {
  const double rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  if (rr < kMinR2d) {  // a node on the target (one-node rule, self panel): no term
    for (int d = 0; d < 3; ++d) gR[d] = gn[d] = 0.0;
    return 0.0;
  }
  const double ri = rsqrt_fp64(rr);
  const double r = rr * ri, ri3 = ri * ri * ri, ri5 = ri3 * ri * ri;
  const double e = exp_fp64(-kappa * r);
  const double nR = n[0] * R[0] + n[1] * R[1] + n[2] * R[2];
  const double ky = (1.0 + kappa * r) * e;
  const double f = a1 * nR * ri3 - a2 * ri - a3 * nR * ky * ri3 + a4 * e * ri;
  const double c3 = e * (3.0 + 3.0 * kappa * r + kappa * kappa * rr);
  for (int d = 0; d < 3; ++d) {
    gR[d] = a1 * (n[d] * ri3 - 3.0 * nR * R[d] * ri5) + a2 * R[d] * ri3 -
            a3 * (ky * n[d] * ri3 - nR * c3 * R[d] * ri5) - a4 * ky * R[d] * ri3;
    gn[d] = a1 * R[d] * ri3 - a3 * ky * R[d] * ri3;
  }
  return f;
}

}  // namespace pbmp
