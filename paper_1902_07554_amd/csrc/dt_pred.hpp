// Device geometric predicates for gfx950.
//
// Two predicates decide everything combinatorial in the method (paper,
// Section "Geometric Primitives" and "Implementation Notes": the partial
// and border triangulations rely on orientation and in-sphere tests
// evaluated with adaptive precision):
//   Orient1(p_0..p_D) = det [ p_i 1 ]                      ((D+1)x(D+1))
//   In(p_0..p_D, q)   = det [ p_i |p_i|^2 1 ; q |q|^2 1 ]   ((D+2)x(D+2))
// For a cell with Orient1 > 0, q lies strictly inside its circumsphere iff
// In > 0.
//
// Evaluation order, cheapest first:
//   1. (optional) FP32 filter on translated coordinates, scaled by a power
//      of two and rounded to FP32, with an a-priori error bound covering the
//      FP64 subtraction, the rounding to FP32 and every FP32 operation;
//   2. FP64 filter on translated coordinates with an a-priori bound;
//   3. exact evaluation with floating-point expansions (sums of
//      non-overlapping doubles built from the error-free two-sum and
//      two-product transformations; Shewchuk 1997) on the original
//      coordinates.
// Error bounds: for the longest term of an expression, K counts the
// roundings it passes through: one per input factor (the rounded
// coordinate differences; in FP32 two, the FP64 difference and the
// conversion) plus the rounded products and sums on its path to the
// result.  The computed value then satisfies |err| <= gamma_K * P, where P
// is the same polynomial over absolute values and gamma_K = K u / (1 - K u);
// P itself is computed with relative error <= gamma_K.  So |value| >
// K u P_hat certifies the sign up to terms of order (K u)^2; the bound used
// is 2 K u P_hat, the factor 2 being slack (u = 2^-53 for FP64, 2^-24 for
// FP32).
//
// Ties (In = 0 exactly) are broken by a symbolic perturbation of the
// lifting: the height of point i becomes |p_i|^2 + eps_i with
// eps_i >> eps_j when key_i < key_j.  Expanding along the height column,
// In_pert = In + sum_i eps_i Cof_i with Cof_i = (-1)^(i+D) Orient1(others);
// the first nonzero cofactor in key order decides.  The exact stage
// computes In from that same expansion, so the cofactors come for free.
//
// Compile without floating-point contraction (-ffp-contract=off): the
// bounds assume separately rounded products and sums, and the error-free
// transformations rely on it.
#pragma once
#include "dt_common.hpp"

namespace dtk {

// Up to D+2 points of a predicate (x, y, z; z unused in 2D) and their
// perturbation keys.  Held in registers on the filtered path; copied to
// private memory only when the exact stage runs.
struct PtsX {
  double p[5][3];
  unsigned long long key[5];
};

// Per-thread predicate counts: [0] orient, [1] insphere.
struct PredStats {
  uint32_t calls[2];
  uint32_t f32ok[2];
  uint32_t exact[2];
};

// ------------------------------------------------------------ expansions
__device__ __forceinline__ void two_sum(double a, double b, double& x, double& y) {
  x = a + b;
  double bv = x - a;
  double av = x - bv;
  double br = b - bv;
  double ar = a - av;
  y = ar + br;
}
// requires |a| >= |b| or a == 0
__device__ __forceinline__ void fast_two_sum(double a, double b, double& x, double& y) {
  x = a + b;
  double bv = x - a;
  y = b - bv;
}
__device__ __forceinline__ void two_prod(double a, double b, double& x, double& y) {
  x = a * b;
  y = __builtin_fma(a, b, -x);
}

// Expansion = components of increasing magnitude, non-overlapping, zero
// components removed.  Buffers have fixed capacities; exceeding one raises
// FAIL_EXACT_CAP and the predicate's answer is discarded by the host.
struct ExpCtx {
  uint32_t* flags;
  bool bad;
};

__device__ __noinline__ void exp_fail(ExpCtx& c) {
  if (!c.bad) atomicOr(c.flags, FAIL_EXACT_CAP);
  c.bad = true;
}

// h = e + b
__device__ inline int exp_grow(ExpCtx& c, const double* e, int n, double b, double* h, int cap) {
  double q = b;
  int m = 0;
  for (int i = 0; i < n; i++) {
    double x, y;
    two_sum(q, e[i], x, y);
    q = x;
    if (y != 0.0) {
      if (m >= cap) { exp_fail(c); return 1; }
      h[m++] = y;
    }
  }
  if (q != 0.0 || m == 0) {
    if (m >= cap) { exp_fail(c); return 1; }
    h[m++] = q;
  }
  return m;
}

// h = e + f, adding f one component at a time; tmp has capacity cap.
__device__ inline int exp_add(ExpCtx& c, const double* e, int ne, const double* f, int nf,
                              double* h, double* tmp, int cap) {
  if (ne < nf) {
    const double* t = e; e = f; f = t;
    int tn = ne; ne = nf; nf = tn;
  }
  if (ne > cap) { exp_fail(c); h[0] = 0.0; return 1; }
  for (int i = 0; i < ne; i++) h[i] = e[i];
  int n = ne;
  for (int j = 0; j < nf; j++) {
    if (f[j] == 0.0) continue;
    n = exp_grow(c, h, n, f[j], tmp, cap);
    if (c.bad) { h[0] = 0.0; return 1; }
    for (int i = 0; i < n; i++) h[i] = tmp[i];
  }
  return n;
}

// h = e * b
__device__ inline int exp_scale(ExpCtx& c, const double* e, int n, double b, double* h, int cap) {
  if (b == 0.0) { h[0] = 0.0; return 1; }
  double q, hh;
  two_prod(e[0], b, q, hh);
  int m = 0;
  if (hh != 0.0) h[m++] = hh;
  for (int i = 1; i < n; i++) {
    double t1, t0, s, x;
    two_prod(e[i], b, t1, t0);
    two_sum(q, t0, s, x);
    if (x != 0.0) {
      if (m >= cap) { exp_fail(c); return 1; }
      h[m++] = x;
    }
    fast_two_sum(t1, s, q, x);
    if (x != 0.0) {
      if (m >= cap) { exp_fail(c); return 1; }
      h[m++] = x;
    }
  }
  if (q != 0.0 || m == 0) {
    if (m >= cap) { exp_fail(c); return 1; }
    h[m++] = q;
  }
  return m;
}

// Compression: renormalise from the largest component down, then from the
// smallest up; the result is non-adjacent and about (bit span)/53 long.
__device__ inline int exp_compress(double* e, int n) {
  if (n <= 1) return n;
  int bottom = n - 1;
  double q = e[bottom];
  for (int i = n - 2; i >= 0; i--) {
    double x, y;
    fast_two_sum(q, e[i], x, y);
    if (y != 0.0) {
      e[bottom--] = x;
      q = y;
    } else {
      q = x;
    }
  }
  e[bottom] = q;
  int top = 0;
  for (int i = bottom + 1; i < n; i++) {
    double x, y;
    fast_two_sum(e[i], q, x, y);
    if (y != 0.0) e[top++] = y;
    q = x;
  }
  e[top++] = q;
  return top;
}

__device__ __forceinline__ int exp_sign(const double* e, int n) {
  double t = e[n - 1];
  return (t > 0.0) - (t < 0.0);
}

// u0 v1 - u1 v0 exactly (at most 4 components)
__device__ inline int det2_exact(ExpCtx& c, double u0, double u1, double v0, double v1, double* h) {
  double a1, a0, b1, b0;
  two_prod(u0, v1, a1, a0);
  two_prod(-u1, v0, b1, b0);
  double e[2] = {a0, a1}, f[2] = {b0, b1};
  double tmp[4];
  return exp_add(c, e, 2, f, 2, h, tmp, 4);
}

constexpr int XC = 48;   // accumulator capacity
constexpr int XT = 96;   // temporary capacity

// Exact Orient1 of points P[0..D] as a compressed expansion in out (XC).
__device__ inline int orient1_expansion(ExpCtx& c, int D, const double* const* P, double* acc) {
  double t1[XT], t2[XT];
  int na = 1;
  acc[0] = 0.0;
  if (D == 2) {
    // det [p 1] = det2(p1,p2) - det2(p0,p2) + det2(p0,p1)
    for (int i = 0; i < 3; i++) {
      int a = (i == 0) ? 1 : 0, b = (i == 2) ? 1 : 2;
      double m[4];
      int nm = det2_exact(c, P[a][0], P[a][1], P[b][0], P[b][1], m);
      if (i == 1)
        for (int j = 0; j < nm; j++) m[j] = -m[j];
      na = exp_add(c, acc, na, m, nm, t1, t2, XC);
      if (c.bad) return 1;
      for (int j = 0; j < na; j++) acc[j] = t1[j];
    }
  } else {
    // det [p 1] (4x4) = sum_i (-1)^(i+3) det3(rows != i),
    // det3(u,v,w) = u.z det2(v,w) - v.z det2(u,w) + w.z det2(u,v)
    for (int i = 0; i < 4; i++) {
      int r[3], t = 0;
      for (int j = 0; j < 4; j++)
        if (j != i) r[t++] = j;
      double d3[XC];
      int n3 = 1;
      d3[0] = 0.0;
      for (int s = 0; s < 3; s++) {
        int u = r[s], v = r[(s == 0) ? 1 : 0], w = r[(s == 2) ? 1 : 2];
        double m[4], sc[8];
        int nm = det2_exact(c, P[v][0], P[v][1], P[w][0], P[w][1], m);
        double z = (s == 1) ? -P[u][2] : P[u][2];
        int ns = exp_scale(c, m, nm, z, sc, 8);
        n3 = exp_add(c, d3, n3, sc, ns, t1, t2, XC);
        if (c.bad) return 1;
        for (int j = 0; j < n3; j++) d3[j] = t1[j];
      }
      if (((i + 3) & 1) != 0)
        for (int j = 0; j < n3; j++) d3[j] = -d3[j];
      na = exp_add(c, acc, na, d3, n3, t1, t2, XC);
      if (c.bad) return 1;
      for (int j = 0; j < na; j++) acc[j] = t1[j];
      na = exp_compress(acc, na);
    }
  }
  return exp_compress(acc, na);
}

// Exact sign of Orient1 of X.p[0..D] (slow path, own stack frame).
__device__ __noinline__ int orient1_exact(uint32_t* flags, int D, PtsX X) {
  ExpCtx c{flags, false};
  const double* P[4] = {X.p[0], X.p[1], X.p[2], X.p[3]};
  double acc[XC];
  int n = orient1_expansion(c, D, P, acc);
  return c.bad ? 0 : exp_sign(acc, n);
}

// Exact sign of In_pert of X.p[0..D+1] (slow path).
// In = sum_i (-1)^(i+D) h_i Orient1(others), h_i = |p_i|^2.
__device__ __noinline__ int in_exact_pert(uint32_t* flags, int D, PtsX X) {
  ExpCtx c{flags, false};
  double acc[XC], o[XC], lift[8], prod[XT], t1[XT], t2[XT];
  int na = 1;
  acc[0] = 0.0;
  int csign[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < D + 2; i++) {
    const double* Q[4];
    int t = 0;
    for (int j = 0; j < D + 2; j++)
      if (j != i) Q[t++] = X.p[j];
    int no = orient1_expansion(c, D, Q, o);
    if (c.bad) return 0;
    if (((i + D) & 1) != 0)
      for (int j = 0; j < no; j++) o[j] = -o[j];
    csign[i] = exp_sign(o, no);
    if (csign[i] == 0) continue;
    lift[0] = 0.0;
    int nl = 1;
    for (int k = 0; k < D; k++) {
      double x1, x0;
      two_prod(X.p[i][k], X.p[i][k], x1, x0);
      double sq[2] = {x0, x1};
      double tt[8];
      nl = exp_add(c, lift, nl, sq, 2, t1, tt, 8);
      for (int j = 0; j < nl; j++) lift[j] = t1[j];
    }
    nl = exp_compress(lift, nl);
    for (int j = 0; j < nl; j++) {
      int np = exp_scale(c, o, no, lift[j], prod, XT);
      if (c.bad) return 0;
      na = exp_add(c, acc, na, prod, np, t1, t2, XC);
      if (c.bad) return 0;
      for (int l = 0; l < na; l++) acc[l] = t1[l];
      na = exp_compress(acc, na);
    }
  }
  int s = exp_sign(acc, na);
  if (s != 0) return s;
  int ord[5] = {0, 1, 2, 3, 4};
  for (int i = 1; i < D + 2; i++)
    for (int j = i; j > 0 && X.key[ord[j]] < X.key[ord[j - 1]]; j--) {
      int t = ord[j]; ord[j] = ord[j - 1]; ord[j - 1] = t;
    }
  for (int t = 0; t < D + 2; t++)
    if (csign[ord[t]] != 0) return csign[ord[t]];
  return 0;
}

// ------------------------------------------------------------ FP64 filters
constexpr double U64 = 1.1102230246251565e-16;   // 2^-53

__device__ __forceinline__ int cert64(double v, double p, double K) {
  if (!(p < 1e300) || p < 1e-280) return 0;
  double b = 2.0 * K * U64 * p;
  return (v > b) ? 1 : ((v < -b) ? -1 : 0);
}

// sign det[p_i - p_0] (D x D).  2D: degree 2, path mul, sub -> K = 4.
// 3D: degree 3, path mul, sub (minor), mul, sub, add -> K = 3 + 5 = 8.
template <int D>
__device__ __forceinline__ int orient_f64(const PtsX& X) {
  if (D == 2) {
    double ax = X.p[1][0] - X.p[0][0], ay = X.p[1][1] - X.p[0][1];
    double bx = X.p[2][0] - X.p[0][0], by = X.p[2][1] - X.p[0][1];
    double l = ax * by, r = ay * bx;
    return cert64(l - r, fabs(l) + fabs(r), 4.0);
  } else {
    double a0 = X.p[1][0] - X.p[0][0], a1 = X.p[1][1] - X.p[0][1], a2 = X.p[1][2] - X.p[0][2];
    double b0 = X.p[2][0] - X.p[0][0], b1 = X.p[2][1] - X.p[0][1], b2 = X.p[2][2] - X.p[0][2];
    double c0 = X.p[3][0] - X.p[0][0], c1 = X.p[3][1] - X.p[0][1], c2 = X.p[3][2] - X.p[0][2];
    double x12 = b1 * c2, x21 = b2 * c1, x02 = b0 * c2, x20 = b2 * c0, x01 = b0 * c1, x10 = b1 * c0;
    double v = a0 * (x12 - x21) - a1 * (x02 - x20) + a2 * (x01 - x10);
    double p = fabs(a0) * (fabs(x12) + fabs(x21)) + fabs(a1) * (fabs(x02) + fabs(x20)) +
               fabs(a2) * (fabs(x01) + fabs(x10));
    return cert64(v, p, 8.0);
  }
}

// sign det[p_i - q, |p_i - q|^2] ((D+1)x(D+1)).
// 2D: degree 4; path mul, add (height), mul, sub (minor), mul, sub, add
//     -> K = 4 + 7 = 11.
// 3D: degree 5; path mul, add, add (height), mul, sub (2x2 minor), mul,
//     sub, add (3x3 minor), mul, three accumulations (the first, from 0,
//     is exact) -> K = 5 + 12 = 17.
template <int D>
__device__ __forceinline__ int in_f64(const PtsX& X) {
  if (D == 2) {
    const double* q = X.p[3];
    double x0 = X.p[0][0] - q[0], y0 = X.p[0][1] - q[1];
    double x1 = X.p[1][0] - q[0], y1 = X.p[1][1] - q[1];
    double x2 = X.p[2][0] - q[0], y2 = X.p[2][1] - q[1];
    double l0 = x0 * x0 + y0 * y0, l1 = x1 * x1 + y1 * y1, l2 = x2 * x2 + y2 * y2;
    double a = x1 * y2, b = y1 * x2, cc = x0 * y2, d = y0 * x2, e = x0 * y1, f = y0 * x1;
    double v = l0 * (a - b) - l1 * (cc - d) + l2 * (e - f);
    double p = l0 * (fabs(a) + fabs(b)) + l1 * (fabs(cc) + fabs(d)) + l2 * (fabs(e) + fabs(f));
    return cert64(v, p, 11.0);
  } else {
    const double* q = X.p[4];
    double d[4][3], l[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      d[i][0] = X.p[i][0] - q[0];
      d[i][1] = X.p[i][1] - q[1];
      d[i][2] = X.p[i][2] - q[2];
      l[i] = d[i][0] * d[i][0] + d[i][1] * d[i][1] + d[i][2] * d[i][2];
    }
    double v = 0.0, p = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r0 = (i == 0) ? 1 : 0, r1 = (i <= 1) ? 2 : 1, r2 = (i <= 2) ? 3 : 2;
      const double *a = d[r0], *b = d[r1], *cc = d[r2];
      double x12 = b[1] * cc[2], x21 = b[2] * cc[1], x02 = b[0] * cc[2], x20 = b[2] * cc[0];
      double x01 = b[0] * cc[1], x10 = b[1] * cc[0];
      double m3 = a[0] * (x12 - x21) - a[1] * (x02 - x20) + a[2] * (x01 - x10);
      double q3 = fabs(a[0]) * (fabs(x12) + fabs(x21)) + fabs(a[1]) * (fabs(x02) + fabs(x20)) +
                  fabs(a[2]) * (fabs(x01) + fabs(x10));
      double t = l[i] * m3;
      v = ((i & 1) == 0) ? v - t : v + t;   // cofactor sign (-1)^(i+3)
      p += l[i] * q3;
    }
    return cert64(v, p, 17.0);
  }
}

// ------------------------------------------------------------ FP32 filters
// Differences are formed in FP64, scaled by 2^s (exact) so the largest lies
// in [1, 2), then rounded to FP32.  Per input factor that is two roundings
// (FP64 subtraction, folded into an FP32 unit, and the conversion); a term
// of degree g with a chain of c FP32 operations thus carries K = 2g + c
// units of 2^-24 (the paths are those of the FP64 filters).  Underflow of
// FP32 intermediates (each at most 2^-150 absolute, a few hundred of them)
// is absorbed by an absolute allowance of 1e-36, far above their sum.
constexpr float U32 = 5.9604645e-08f;   // 2^-24

__device__ __forceinline__ int cert32(float v, float p, float K) {
  if (!(p < 1e30f) || p < 1e-30f) return 0;
  float b = 2.0f * K * U32 * p + 1e-36f;
  return (v > b) ? 1 : ((v < -b) ? -1 : 0);
}

__device__ __forceinline__ double pow2_scale(double m) {
  int e;
  frexp(m, &e);            // m in [2^(e-1), 2^e)
  return ldexp(1.0, 1 - e);
}

template <int D>
__device__ __forceinline__ int orient_f32(const PtsX& X) {
  if (D == 2) {
    double ax = X.p[1][0] - X.p[0][0], ay = X.p[1][1] - X.p[0][1];
    double bx = X.p[2][0] - X.p[0][0], by = X.p[2][1] - X.p[0][1];
    double m = fmax(fmax(fabs(ax), fabs(ay)), fmax(fabs(bx), fabs(by)));
    if (!(m > 1e-150 && m < 1e150)) return 0;
    double s = pow2_scale(m);
    float fax = (float)(ax * s), fay = (float)(ay * s), fbx = (float)(bx * s), fby = (float)(by * s);
    float l = fax * fby, r = fay * fbx;
    return cert32(l - r, fabsf(l) + fabsf(r), 6.0f);            // g=2, c=2
  } else {
    double a[3], b[3], c[3];
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      a[k] = X.p[1][k] - X.p[0][k];
      b[k] = X.p[2][k] - X.p[0][k];
      c[k] = X.p[3][k] - X.p[0][k];
      m = fmax(m, fmax(fabs(a[k]), fmax(fabs(b[k]), fabs(c[k]))));
    }
    if (!(m > 1e-100 && m < 1e100)) return 0;
    double s = pow2_scale(m);
    float A0 = (float)(a[0] * s), A1 = (float)(a[1] * s), A2 = (float)(a[2] * s);
    float B0 = (float)(b[0] * s), B1 = (float)(b[1] * s), B2 = (float)(b[2] * s);
    float C0 = (float)(c[0] * s), C1 = (float)(c[1] * s), C2 = (float)(c[2] * s);
    float x12 = B1 * C2, x21 = B2 * C1, x02 = B0 * C2, x20 = B2 * C0, x01 = B0 * C1, x10 = B1 * C0;
    float v = A0 * (x12 - x21) - A1 * (x02 - x20) + A2 * (x01 - x10);
    float p = fabsf(A0) * (fabsf(x12) + fabsf(x21)) + fabsf(A1) * (fabsf(x02) + fabsf(x20)) +
              fabsf(A2) * (fabsf(x01) + fabsf(x10));
    return cert32(v, p, 11.0f);                                  // g=3, c=5
  }
}

template <int D>
__device__ __forceinline__ int in_f32(const PtsX& X) {
  if (D == 2) {
    const double* q = X.p[3];
    double x[3], y[3];
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      x[i] = X.p[i][0] - q[0];
      y[i] = X.p[i][1] - q[1];
      m = fmax(m, fmax(fabs(x[i]), fabs(y[i])));
    }
    if (!(m > 1e-60 && m < 1e60)) return 0;
    double s = pow2_scale(m);
    float Xf[3], Yf[3], L[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      Xf[i] = (float)(x[i] * s);
      Yf[i] = (float)(y[i] * s);
      L[i] = Xf[i] * Xf[i] + Yf[i] * Yf[i];
    }
    float a = Xf[1] * Yf[2], b = Yf[1] * Xf[2], cc = Xf[0] * Yf[2], d = Yf[0] * Xf[2];
    float e = Xf[0] * Yf[1], f = Yf[0] * Xf[1];
    float v = L[0] * (a - b) - L[1] * (cc - d) + L[2] * (e - f);
    float p = L[0] * (fabsf(a) + fabsf(b)) + L[1] * (fabsf(cc) + fabsf(d)) +
              L[2] * (fabsf(e) + fabsf(f));
    return cert32(v, p, 15.0f);                                  // g=4, c=7
  } else {
    const double* q = X.p[4];
    double d[4][3];
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
#pragma unroll
      for (int k = 0; k < 3; k++) {
        d[i][k] = X.p[i][k] - q[k];
        m = fmax(m, fabs(d[i][k]));
      }
    }
    if (!(m > 1e-40 && m < 1e40)) return 0;
    double s = pow2_scale(m);
    float F[4][3], L[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      F[i][0] = (float)(d[i][0] * s);
      F[i][1] = (float)(d[i][1] * s);
      F[i][2] = (float)(d[i][2] * s);
      L[i] = F[i][0] * F[i][0] + F[i][1] * F[i][1] + F[i][2] * F[i][2];
    }
    float v = 0.0f, p = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r0 = (i == 0) ? 1 : 0, r1 = (i <= 1) ? 2 : 1, r2 = (i <= 2) ? 3 : 2;
      const float *a = F[r0], *b = F[r1], *cc = F[r2];
      float x12 = b[1] * cc[2], x21 = b[2] * cc[1], x02 = b[0] * cc[2], x20 = b[2] * cc[0];
      float x01 = b[0] * cc[1], x10 = b[1] * cc[0];
      float m3 = a[0] * (x12 - x21) - a[1] * (x02 - x20) + a[2] * (x01 - x10);
      float q3 = fabsf(a[0]) * (fabsf(x12) + fabsf(x21)) + fabsf(a[1]) * (fabsf(x02) + fabsf(x20)) +
                 fabsf(a[2]) * (fabsf(x01) + fabsf(x10));
      float t = L[i] * m3;
      v = ((i & 1) == 0) ? v - t : v + t;
      p += L[i] * q3;
    }
    return cert32(v, p, 22.0f);                                  // g=5, c=12
  }
}

// ------------------------------------------------------------ front ends
// Out-of-line FP64 filter followed by the exact stage, for the FP32 mode:
// keeping it out of the callers' inline code keeps their register use (and
// so the number of resident wavefronts) at the level of the FP32 path.
// Result: 2*sign + (1 if the exact stage ran).
template <int D>
__device__ __noinline__ int orient_slow64(uint32_t* flags, PtsX X) {
  int s = orient_f64<D>(X);
  if (s) return 2 * ((D & 1) ? -s : s);
  return 2 * orient1_exact(flags, D, X) + 1;
}
template <int D>
__device__ __noinline__ int insphere_slow64(uint32_t* flags, PtsX X) {
  int s = in_f64<D>(X);
  if (s) return 2 * s;
  return 2 * in_exact_pert(flags, D, X) + 1;
}
__device__ __forceinline__ int slow_sign(int r) { return (r - (r & 1)) / 2; }

// F32: FP32 filter first (then FP64, then exact); otherwise FP64 first.
template <bool F32>
struct PredT {
  uint32_t* flags;
  PredStats st;

  __device__ void init(uint32_t* f) {
    flags = f;
    st.calls[0] = st.calls[1] = st.f32ok[0] = st.f32ok[1] = st.exact[0] = st.exact[1] = 0;
  }

  // sign of Orient1(X.p[0..D]) = (-1)^D sign det[p_i - p_0]
  template <int D>
  __device__ int orient(const PtsX& X) {
    st.calls[0]++;
    if (F32) {
      int s = orient_f32<D>(X);
      if (s) { st.f32ok[0]++; return (D & 1) ? -s : s; }
      int r = orient_slow64<D>(flags, X);
      st.exact[0] += (uint32_t)(r & 1);
      return slow_sign(r);
    } else {
      int s = orient_f64<D>(X);
      if (s) return (D & 1) ? -s : s;
      st.exact[0]++;
      return orient1_exact(flags, D, X);
    }
  }

  // sign of In_pert(X.p[0..D], X.p[D+1])
  template <int D>
  __device__ int insphere(const PtsX& X) {
    st.calls[1]++;
    if (F32) {
      int s = in_f32<D>(X);
      if (s) { st.f32ok[1]++; return s; }
      int r = insphere_slow64<D>(flags, X);
      st.exact[1] += (uint32_t)(r & 1);
      return slow_sign(r);
    } else {
      int s = in_f64<D>(X);
      if (s) return s;
      st.exact[1]++;
      return in_exact_pert(flags, D, X);
    }
  }
};

}  // namespace dtk
