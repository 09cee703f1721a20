// Device-side building blocks shared by the forward and adjoint kernels of
// libtenoaa: the paper's constants, the scalar TENO-AA reconstruction
// (Sec. 3-4) and the local frame of a sweep direction.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "tenoaa_sos.h"

namespace tenoaa {
namespace {

// ---------------------------------------------------------------- constants
// Sec. 3.2: eps of the scale-separation formula, q = 7.
constexpr double EPS = 1e-40;
// Sec. 3.4: C_r, alpha_1, alpha_2; C_T = 10^{-K}, K = 7..14.
constexpr double C_R = 0.265;
constexpr double ALPHA1 = 14.0;
constexpr double ALPHA2 = 6.4;
constexpr double CT_TABLE[8] = {1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12, 1e-13, 1e-14};
// 1/C_T - 1 = 10^K - 1 (exact doubles), the bound of the large-stencil test
// in the form S b^7 <= 1/C_T - 1 (teno_aa)
constexpr double INV_CT_M1[8] = {9999999.0,      99999999.0,      999999999.0,      9999999999.0,
                                 99999999999.0, 999999999999.0, 9999999999999.0, 99999999999999.0};
// Sec. 4.1 / 4.2: linear schemes on S3, S4, S5, leftmost coefficient first.
constexpr double LIN6[6] = {0.02852274270130377, -0.1714015614372447, 0.650378818735941,
                            0.6253788187359414, -0.1589015614372448, 0.02602274270130375};
constexpr double LIN8[8] = {-0.006866688980568011, 0.05128582585522106, -0.1968478198727312,
                            0.6552858258552222,    0.6452858258552218,  -0.1908478198727314,
                            0.04928582585522098,   -0.006580974694853729};
constexpr double LIN10[10] = {0.001911786299492748, -0.0170332977472532, 0.07339445614860979,
                              -0.221228429084247,   0.6657332621611695,  0.6557332621611695,
                              -0.2145617624175796,  0.07053731329146805, -0.01631901203296621,
                              0.001832421220128962};
// Sec. 4.1: optimal weights of the small stencils, and the fallback weights
// w_k = d_k delta_k / sum_l d_l delta_l (Sec. 3.3) for the 8 delta masks,
// evaluated at compile time with the IEEE operations a run-time evaluation
// would use.
constexpr double DK[3] = {0.5065006634, 0.3699651429, 0.1235341937};
constexpr double fallback_weight(int mask, int k) {
  const double d0 = DK[0] * ((mask & 1) ? 1.0 : 0.0);
  const double d1 = DK[1] * ((mask & 2) ? 1.0 : 0.0);
  const double d2 = DK[2] * ((mask & 4) ? 1.0 : 0.0);
  const double dsum = (d0 + d1) + d2;
  const double num = k == 0 ? d0 : (k == 1 ? d1 : d2);
  return mask == 0 ? 0.0 : num / dsum;
}
struct WTable {
  double w[8][3];
};
constexpr WTable make_wtable() {
  WTable t{};
  for (int m = 0; m < 8; ++m)
    for (int k = 0; k < 3; ++k) t.w[m][k] = fallback_weight(m, k);
  return t;
}
constexpr WTable WFALL = make_wtable();

// -------------------------------------------------------------- small math
// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1, so
// every index into a register array or constant table is a constant.
template <int N, class F>
__device__ __forceinline__ void unroll(F&& f) {
  if constexpr (N > 0) {
    unroll<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }

// Reciprocal for decision-only quantities: the hardware estimate refined by
// one Newton step (relative error below 3e-15 for finite non-zero x).
__device__ __forceinline__ double rcp_dec(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Correctly rounded division and square root.  The compiler's FP64 sequences
// are within an ulp but, in rare operands extremely close to a rounding
// midpoint, not correctly rounded; one exact fma remainder of the result and
// of its neighbour on the remainder's side decides between the two, so every
// value the kernels compute matches an IEEE evaluation bit for bit.
__device__ __forceinline__ double next_toward(double q, bool up) {
  const long long bits = __double_as_longlong(q);
  return __longlong_as_double(bits + (((q > 0.0) == up) ? 1 : -1));
}

__device__ __forceinline__ double div_rn(double a, double b) {
  const double q = a / b;
  const double r = fma(-q, b, a);  // exact: q is within an ulp of a / b
  if (!(r != 0.0) || q == 0.0 || !(fabs(q) <= 1.7976931348623157e308)) return q;
  const double qn = next_toward(q, (r > 0.0) == (b > 0.0));
  const double rn = fma(-qn, b, a);
  const double ar = fabs(r), arn = fabs(rn);
  if (arn < ar || (arn == ar && (__double_as_longlong(q) & 1))) return qn;  // nearer; a tie goes to even
  return q;
}

__device__ __forceinline__ double sqrt_rn(double x) {
  const double s = sqrt(x);
  if (!(x > 0.0) || !(s <= 1.7976931348623157e308)) return s;
  const double r = fma(-s, s, x);  // exact
  // with lo <= sqrt(x) < lo + u (u the gap above lo, lo*u exact), sqrt(x) is
  // above the midpoint iff x - lo^2 - lo*u > 0; that quantity is a multiple of
  // u^2, so the one rounding of the fma cannot change its sign
  if (r >= 0.0) {
    const double hi = next_toward(s, true);
    return fma(-s, hi - s, r) > 0.0 ? hi : s;
  }
  const double lo = next_toward(s, false);
  const double rl = fma(-lo, lo, x);
  return fma(-lo, s - lo, rl) > 0.0 ? s : lo;
}

// x / 6 correctly rounded: one product by RN(1/6) and one fma correction of
// the exact remainder (Markstein's theorem: the reciprocal within 1/2 ulp and
// the first quotient within 1 ulp make the corrected quotient the correctly
// rounded one, in round-to-nearest, away from underflow and overflow).  Equal
// to the IEEE division x / 6.0 bit for bit in that range.
__device__ __forceinline__ double div6(double x) {
  constexpr double y = 1.0 / 6.0;
  const double q = x * y;
  const double r = fma(-6.0, q, x);
  return fma(r, y, q);
}

// gamma = 1/(beta + eps)^7 (Sec. 3.2, q = 7), decision-only.
__device__ __forceinline__ double gamma7(double beta) {
  const double r = rcp_dec(beta + EPS);
  const double r2 = r * r;
  const double r4 = r2 * r2;
  return (r4 * r2) * r;
}

// Smoothness indicator of a large stencil of width R whose leftmost value is
// v[P]: the exact sum of squares beta = sum_k D[k] y_k^2 over the stencil's
// first differences d_m = f_{P+m+1} - f_{P+m}, y_k = sum_{m >= k} L[m][k] d_m.
// The differences are the ones the cut-off's eta and the other indicators
// use (the compiler computes each once).
template <int R, int P, int W>
__device__ __forceinline__ double sos_beta(const double (&v)[W]) {
  static_assert(R == 6 || R == 8 || R == 10 || R == 12, "large stencils only");
  double dif[R - 1];
  unroll<R - 1>([&](auto m) { dif[m] = v[P + m + 1] - v[P + m]; });
  double beta = 0.0;
  unroll<R - 1>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    // L has a unit diagonal, so the sum starts from d_k itself (no product by 1)
    constexpr double lkk = (R == 12)   ? SOS_S6_L[k][k]
                           : (R == 10) ? SOS_S5_L[k][k]
                           : (R == 8)  ? SOS_S4_L[k][k]
                                       : SOS_S3_L[k][k];
    static_assert(lkk == 1.0, "the factor must have a unit diagonal");
    double y = dif[k];
    unroll<R - 1>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if constexpr (m > k) {
        constexpr double l = (R == 12)   ? SOS_S6_L[m][k]
                             : (R == 10) ? SOS_S5_L[m][k]
                             : (R == 8)  ? SOS_S4_L[m][k]
                                         : SOS_S3_L[m][k];
        if constexpr (l != 0.0) y = fma(l, dif[m], y);
      }
    });
    constexpr double dk = (R == 12) ? SOS_S6_D[k] : (R == 10) ? SOS_S5_D[k] : (R == 8) ? SOS_S4_D[k] : SOS_S3_D[k];
    beta = fma(dk, y * y, beta);
  });
  return beta;
}

template <int R>
__device__ __host__ constexpr double lin_coef(int q) {
  return (R == 12) ? LIN12[q] : (R == 10) ? LIN10[q] : (R == 8) ? LIN8[q] : LIN6[q];
}

// Linear scheme of width R on the values starting at v[P] (Sec. 4.1).
template <int R, int P, int W>
__device__ __forceinline__ double linear_flux(const double (&v)[W]) {
  constexpr double c0 = lin_coef<R>(0);
  double acc = c0 * v[P];
  unroll<R - 1>([&](auto qq) {
    constexpr int q = decltype(qq)::value;
    constexpr double c = lin_coef<R>(q + 1);
    acc = fma(c, v[P + q + 1], acc);
  });
  return acc;
}

// ------------------------------------------------- scalar TENO-AA (Sec. 3-4)
// v[0..W-1] = f_{i-G+1..i+G}, ORDER = W = 8, 10 or 12 (TENO12-AA: the
// framework with the twelve-point stencil S6 above S5).  Returns
// fhat_{i+1/2}; flag gets the decision byte (bits 0-1 large stencil, with
// bit 2 set for S6; 2-4 deltas of the fallback; 5-7 K-7).  With AUDIT, near
// gets 1 if a test the reconstruction made lies within the relative distance
// tol of its threshold (chi_p / C_T or chi_k / C_T within 1 +- tol, or the
// cut-off exponent B within tol B of an integer while m > 0), else 0.
// The TENO5 fallback's flux once its deltas are decided (Sec. 3.3): the
// renormalised weights of the kept small stencils times their third-order
// candidates.  Shared by teno_aa and replay_recon, outside teno_aa's
// contracted decision arithmetic.
template <int ORDER>
__device__ __forceinline__ double fallback_flux(const double (&v)[ORDER], int dm) {
  constexpr int I = ORDER / 2 - 1;
  const double fm1 = v[I - 1], f0 = v[I], f1 = v[I + 1];
  const double h0 = div6((-fm1 + 5.0 * f0) + 2.0 * f1);
  const double h1 = div6((2.0 * f0 + 5.0 * f1) - v[I + 2]);
  const double h2 = div6((2.0 * v[I - 2] - 7.0 * fm1) + 11.0 * f0);
  return fma(WFALL.w[dm][2], h2, fma(WFALL.w[dm][1], h1, WFALL.w[dm][0] * h0));
}

template <int ORDER, bool AUDIT = false>
__device__ __forceinline__ double teno_aa(const double (&v)[ORDER], uint8_t& flag, uint8_t* near = nullptr,
                                          double tol = 0.0) {
  // every operation written in this body is decision-only (the fluxes come
  // from linear_flux and fallback_flux), so the compiler may fuse its
  // multiply-adds: a decision then differs from the oracle's only within a
  // few ulps of its threshold, inside the band the parity checks exclude
#pragma clang fp contract(fast)
  constexpr int G = ORDER / 2;
  constexpr int I = G - 1;  // index of f_i

  // Sec. 3.4: eta_j = (|2 a b| + eps) / (a^2 + b^2 + eps), j = -1..2, with
  // a = f_{j+1} - f_j, b = f_j - f_{j-1}; the minimum is located by cross
  // multiplication and divided out once.
  double dd[5];  // f_{k+1} - f_k for k = -2..2
  unroll<5>([&](auto q) { dd[q] = v[I - 2 + q + 1] - v[I - 2 + q]; });
  double nb = 0.0, db = 1.0;
  unroll<4>([&](auto jj) {
    const double a = dd[jj + 1];
    const double b = dd[jj];
    const double num = fabs((2.0 * a) * b) + EPS;
    const double den = (a * a + b * b) + EPS;
    if (jj == 0 || num * db < nb * den) {
      nb = num;
      db = den;
    }
  });
  const double etabar = nb * rcp_dec(db);  // decision-only
  double ratio = etabar * (1.0 / C_R);
  if (ratio > 1.0) ratio = 1.0;
  const double m = 1.0 - ratio;
  const double om = 1.0 - m;
  const double om2 = om * om;
  const double g = (om2 * om2) * (1.0 + 4.0 * m);
  const double B = ALPHA1 - ALPHA2 * (1.0 - g);
  int K = (int)floor(B);
  K = K < 7 ? 7 : (K > 14 ? 14 : K);
  const double CT = CT_TABLE[K - 7];
  const double TK = INV_CT_M1[K - 7];
  const uint8_t kbits = (uint8_t)((K - 7) << 5);
  // chi / C_T - 1 = (g - t) / t for the test g >= t
  [[maybe_unused]] auto close = [&](double g, double t) { return fabs(g - t) <= tol * t; };
  if constexpr (AUDIT) *near = (m > 0.0 && fabs(B - rint(B)) <= tol * B) ? 1 : 0;

  // small stencils (Sec. 4.2, printed WENO-JS indicators) in difference form
  const double b0a = dd[1] + dd[2];                // f_{i+1} - f_{i-1}
  const double b0b = dd[2] - dd[1];                // f_{i-1} - 2 f_i + f_{i+1}
  const double b1a = (dd[3] - dd[2]) - 2.0 * dd[2];  // f_{i+2} - 4 f_{i+1} + 3 f_i
  const double b1b = dd[3] - dd[2];
  const double b2a = (dd[1] - dd[0]) + 2.0 * dd[1];  // f_{i-2} - 4 f_{i-1} + 3 f_i
  const double b2b = dd[1] - dd[0];
  constexpr double C13 = 13.0 / 12.0;
  const double g0 = gamma7(fma(C13, b0b * b0b, 0.25 * (b0a * b0a)));
  const double g1 = gamma7(fma(C13, b1b * b1b, 0.25 * (b1a * b1a)));
  const double g2 = gamma7(fma(C13, b2b * b2b, 0.25 * (b2a * b2a)));
  const double S = (g0 + g1) + g2;
  // Sec. 3.3's test of a large stencil, gamma_p >= C_T (S + gamma_p) with
  // gamma_p = 1/b^7 (b = beta_p + eps), taken as S b^7 <= 1/C_T - 1: the
  // same inequality without the reciprocal of b (decision-only; an overflow
  // of S b^7 fails the test, as the exact ratio does)
  auto passes = [&](double beta) {
    const double b = beta + EPS;
    const double b2 = b * b;
    const double b4 = b2 * b2;
    return S * ((b4 * b2) * b) <= TK;
  };

  // Sec. 3.3: the groups (S0,S1,S2,Sp), largest p first; Sp is taken when
  // chi_p = gamma_p / (S + gamma_p) >= C_T.  Stencil Sp starts at v[G - p].
  if constexpr (ORDER == 12) {
    const double bp = sos_beta<12, 0>(v);
    if constexpr (AUDIT) {
      const double gp = gamma7(bp);
      *near |= close(gp, CT * (S + gp)) ? 1 : 0;
    }
    if (passes(bp)) {
      flag = (uint8_t)(7 | kbits);
      return linear_flux<12, 0>(v);
    }
  }
  if constexpr (ORDER >= 10) {
    constexpr int P = G - 5;
    const double bp = sos_beta<10, P>(v);
    if constexpr (AUDIT) {
      const double gp = gamma7(bp);
      *near |= close(gp, CT * (S + gp)) ? 1 : 0;
    }
    if (passes(bp)) {
      flag = (uint8_t)(3 | kbits);
      return linear_flux<10, P>(v);
    }
  }
  {
    constexpr int P = G - 4;
    const double bp = sos_beta<8, P>(v);
    if constexpr (AUDIT) {
      const double gp = gamma7(bp);
      *near |= close(gp, CT * (S + gp)) ? 1 : 0;
    }
    if (passes(bp)) {
      flag = (uint8_t)(2 | kbits);
      return linear_flux<8, P>(v);
    }
  }
  {
    constexpr int P = G - 3;
    const double bp = sos_beta<6, P>(v);
    if constexpr (AUDIT) {
      const double gp = gamma7(bp);
      *near |= close(gp, CT * (S + gp)) ? 1 : 0;
    }
    if (passes(bp)) {
      flag = (uint8_t)(1 | kbits);
      return linear_flux<6, P>(v);
    }
  }
  // fallback: TENO5 cut-off among the small stencils (Sec. 3.3)
  const double cs = CT * S;
  if constexpr (AUDIT) *near |= (close(g0, cs) || close(g1, cs) || close(g2, cs)) ? 1 : 0;
  const int dm = (g0 >= cs ? 1 : 0) | (g1 >= cs ? 2 : 0) | (g2 >= cs ? 4 : 0);
  flag = (uint8_t)((dm << 2) | kbits);
  return fallback_flux<ORDER>(v, dm);
}

// The reconstruction a recorded decision byte selects, evaluated exactly as
// teno_aa evaluates it once it has decided (replay of recorded decisions).
template <int ORDER>
__device__ __forceinline__ double replay_recon(const double (&v)[ORDER], uint8_t flag) {
  constexpr int G = ORDER / 2;
  const int sel = flag & 3;
  if constexpr (ORDER == 12) {
    if (sel == 3 && (flag & 4)) return linear_flux<12, 0>(v);
  }
  if constexpr (ORDER >= 10) {
    if (sel == 3) return linear_flux<10, G - 5>(v);
  }
  if (sel == 2) return linear_flux<8, G - 4>(v);
  if (sel == 1) return linear_flux<6, G - 3>(v);
  return fallback_flux<ORDER>(v, (flag >> 2) & 7);
}

// Local frame of direction DIR: component 0 = rho, 1 = normal momentum,
// 2.. = tangential momenta in ascending axis order, last = E.
template <int NDIM, int DIR>
struct Frame {
  static constexpr int NV = NDIM + 2;
  // axis index of tangential k (k = 0 .. NDIM-2)
  static __host__ __device__ constexpr int tan_axis(int k) { return (k < DIR) ? k : k + 1; }
  // local velocity slot (0 = normal, 1 + k = tangential k) of axis a
  static __host__ __device__ constexpr int slot_of_axis(int a) {
    return a == DIR ? 0 : (a < DIR ? 1 + a : a);
  }
};

}  // namespace
}  // namespace tenoaa
