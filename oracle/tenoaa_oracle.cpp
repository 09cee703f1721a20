// TENO-AA8 / TENO-AA10 compressible-Euler right-hand side: the ORACLE.
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, serial, slow FP64 CPU
// implementation of L. Fu, "Very-high-order TENO schemes with adaptive
// accuracy order and adaptive dissipation control" (arXiv 2109.14340), written
// so that a reader can check every step against the paper by eye.  Only the
// test suite, the smoke check and the benchmark's CPU-baseline leg load it.
// It shares no code, header or table with the GPU library; the two are
// written independently against the same paper and the same written
// evaluation order (below), and the tests compare them.
//
// What it computes (paper section in brackets):
//   * smoothness indicators beta_{k,r} by their definition: the Jiang-Shu
//     integral of the squared derivatives of the candidate polynomial over
//     the cell [x_{i-1/2}, x_{i+1/2}] (Sec. 3.2, eq. for beta_{k,r}), the
//     polynomial being the one whose cell averages over the stencil equal the
//     data (Sec. 2, primitive-function definition).  The integral is taken
//     exactly with Gauss-Legendre quadrature on the Newton form of the
//     primitive, so constants give exactly zero;
//   * scale separation gamma_k = 1/(beta_k+eps)^q, q = 7, eps = 1e-40 (Sec. 3.2);
//   * the ENO-like selection cascade over the groups (S0,S1,S2,Sp) from the
//     largest large stencil down, the TENO5 fallback with renormalised d_k
//     (Sec. 3.3), and TENO8-AA = TENO10-AA without S5 (Sec. 4.3);
//   * the adaptive cut-off C_T from the first-order undivided-difference
//     measure eta, m, g(m), [beta] (Sec. 3.4);
//   * the optimised linear schemes and candidate fluxes (Sec. 4.1, 4.2);
//   * Roe-averaged characteristic projection, LLF or Rusanov splitting, or
//     the Roe flux with entropy fix (Sec. 5.2's blast waves and
//     Rayleigh-Taylor runs), SSP-RK3, dimension-by-dimension sweeps (Sec. 5
//     opening paragraph);
//   * ghost cells for periodic, outflow, slip and no-slip walls, the
//     second-order Dirichlet form (Appendix A; outflow is the zeroth-order
//     copy reading) and prescribed supersonic-inflow states;
//   * the positivity-preserving flux limiter of Hu, Adams & Shu 2013 that the
//     paper applies in its extreme cases (Sec. 5.3 opening paragraph), in
//     the reading stated at or_limit_face below.
//
// Evaluation order.  The GPU path must reproduce, bit for bit, every value
// that feeds a threshold decision (the split characteristic fluxes), so this
// file fixes one order for each formula: the order written here, with no
// contraction (build with -ffp-contract=off) and std::fma only where it is
// spelled out.  The smoothness indicators, gamma, chi and the C_T bucket are
// decision-only quantities; the GPU may evaluate them differently and the
// tests then allow disagreement only where this file reports a decision
// within a relative 1e-12 of its threshold ("margin").
//
// The numerical core is templated on the scalar type so that a forward-mode
// (dual-number) evaluation with frozen decisions gives exact directional
// derivatives for the adjoint tests.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// Forward-mode derivative pair.  The value part is computed by exactly the
// FP64 operations of the plain evaluation (fma included), so a derivative
// evaluation takes the same decisions as the plain one; the d part carries
// the exact directional derivative (to rounding).
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}  // NOLINT: constants promote implicitly
  Dual(double x, double y) : v(x), d(y) {}
};
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}

inline double re(double x) { return x; }
inline double re(const Dual& x) { return x.v; }
inline double fmaT(double a, double b, double c) { return std::fma(a, b, c); }
inline Dual fmaT(const Dual& a, const Dual& b, const Dual& c) {
  return Dual(std::fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d);
}
inline double absT(double x) { return std::fabs(x); }
inline Dual absT(const Dual& x) { return x.v < 0.0 ? -x : x; }
inline double sqrtT(double x) { return std::sqrt(x); }
inline Dual sqrtT(const Dual& x) {
  const double r = std::sqrt(x.v);
  return Dual(r, x.d / (2.0 * r));
}

// ---------------------------------------------------------------- constants
// Sec. 3.2: eps and q of the scale-separation formula.
const double EPS = 1e-40;
// Sec. 3.4: C_r, alpha_1, alpha_2 and eps of the discontinuity detector.
const double C_R = 0.265;
const double ALPHA1 = 14.0;
const double ALPHA2 = 6.4;
// Sec. 3.4: C_T = 10^{-[beta]}, [beta] in 7..14, kept as decimal literals.
const double CT_OF_K[15] = {0, 0, 0, 0, 0, 0, 0, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12, 1e-13, 1e-14};
// Sec. 4.1: optimal weights of the small stencils.
const double DK[3] = {0.5065006634, 0.3699651429, 0.1235341937};
// Sec. 4.1: optimised linear schemes on S3 (6-point), S4 (8-point), S5 (10-point),
// coefficients from the leftmost stencil cell to the rightmost.
const double LIN6[6] = {0.02852274270130377, -0.1714015614372447, 0.650378818735941,
                        0.6253788187359414, -0.1589015614372448, 0.02602274270130375};
const double LIN8[8] = {-0.006866688980568011, 0.05128582585522106, -0.1968478198727312,
                        0.6552858258552222,    0.6452858258552218,  -0.1908478198727314,
                        0.04928582585522098,   -0.006580974694853729};
const double LIN10[10] = {0.001911786299492748, -0.0170332977472532,  0.07339445614860979,
                          -0.221228429084247,   0.6657332621611695,   0.6557332621611695,
                          -0.2145617624175796,  0.07053731329146805,  -0.01631901203296621,
                          0.001832421220128962};

// TENO12-AA (the framework of Sec. 3.1 with one more symmetric large
// stencil, S6 = cells i-5 .. i+6): the paper prints no optimised scheme for
// it, so S6 takes the maximum-order (12th) reconstruction, written by
// gen_teno12.py in exact arithmetic and rounded once.
const double LIN12[12] = {-0.00018037518037518038, 0.002417027417027417, -0.01544011544011544, 0.06392496392496393,
                          -0.20393217893217894,    0.6532106782106782,   0.6532106782106782,   -0.20393217893217894,
                          0.06392496392496393,     -0.01544011544011544, 0.002417027417027417, -0.00018037518037518038};

// Candidate stencils of Sec. 3.1 / 4.2, as (leftmost cell offset from i, width).
const int ST_LO[7] = {-1, 0, -2, -2, -3, -4, -5};
const int ST_R[7] = {3, 3, 3, 6, 8, 10, 12};

// ---------------------------------------------- smoothness indicator tables
// beta_{k,r} = sum_{j=1}^{r-1} dx^{2j-1} int_{cell i} (d^j p_k/dx^j)^2 dx.
// In units of dx the stencil cell l (0-based) spans [l-1/2, l+1/2]; the
// primitive P of p_k takes the values P(b-1/2) = sum_{l<b} f_l at the r+1 cell
// boundaries, so in Newton form over those nodes
//   P(x) = const + sum_{m=1}^{r-1} Delta^m f_0 / (m+1)! * omega_{m+1}(x) + f_0 x,
//   omega_{m+1}(x) = prod_{b=0}^{m} (x - (b - 1/2)),
// and p_k^{(j)} = P^{(j+1)} involves only the forward differences Delta^m f_0,
// m >= j.  The integral over cell i (local index e = -lo) of the square of a
// polynomial of degree r-1-j is exact with (r-1)-point Gauss-Legendre.
struct BetaTable {
  int r = 0, lo = 0, nq = 0;
  double w[11];
  double M[11][11][11];  // M[j-1][q][m-1] = omega_{m+1}^{(j+1)}(x_q) / (m+1)!
};
BetaTable g_beta[7];
bool g_beta_ready = false;

void gauss_legendre(int n, double* x, double* w) {
  // Newton iteration on the Legendre polynomial P_n from the three-term recurrence.
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 200; ++it) {
      double pn = 1.0, pm = 0.0;
      for (int k = 1; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * pn - (k - 1.0) * pm) / k;
        pm = pn;
        pn = pk;
      }
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double pn = 1.0, pm = 0.0;
    for (int k = 1; k <= n; ++k) {
      double pk = ((2.0 * k - 1.0) * z * pn - (k - 1.0) * pm) / k;
      pm = pn;
      pn = pk;
    }
    dp = n * (z * pn - pm) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void build_beta_tables() {
  if (g_beta_ready) return;
  for (int k = 0; k < 7; ++k) {
    BetaTable& T = g_beta[k];
    T.r = ST_R[k];
    T.lo = ST_LO[k];
    T.nq = T.r - 1;
    double gx[11], gw[11];
    gauss_legendre(T.nq, gx, gw);
    const double e = -T.lo;  // local index of cell i inside the stencil
    for (int q = 0; q < T.nq; ++q) T.w[q] = 0.5 * gw[q];
    std::memset(T.M, 0, sizeof(T.M));
    for (int m = 1; m <= T.r - 1; ++m) {
      // omega_{m+1}(e + t) as a polynomial in t (coefficients are dyadic, exact).
      double c[14] = {0};
      c[0] = 1.0;
      int deg = 0;
      for (int b = 0; b <= m; ++b) {
        const double root = (b - 0.5) - e;  // factor (t - root)
        double nc[14] = {0};
        for (int a = 0; a <= deg; ++a) {
          nc[a + 1] += c[a];
          nc[a] -= root * c[a];
        }
        ++deg;
        std::memcpy(c, nc, sizeof(c));
      }
      double fact = 1.0;
      for (int a = 2; a <= m + 1; ++a) fact *= a;
      for (int j = 1; j <= m; ++j) {
        // (j+1)-th derivative of the t-polynomial
        double dc[14] = {0};
        for (int a = j + 1; a <= deg; ++a) {
          double f = 1.0;
          for (int s = 0; s <= j; ++s) f *= (a - s);
          dc[a - j - 1] = c[a] * f;
        }
        for (int q = 0; q < T.nq; ++q) {
          const double t = 0.5 * gx[q];
          double v = 0.0;
          for (int a = deg - j - 1; a >= 0; --a) v = v * t + dc[a];
          T.M[j - 1][q][m - 1] = v / fact;
        }
      }
    }
  }
  g_beta_ready = true;
}

// f points at the stencil's leftmost value; returns beta for candidate k.
double beta_of(int k, const double* f) {
  const BetaTable& T = g_beta[k];
  double tab[12], dif[11];
  for (int l = 0; l < T.r; ++l) tab[l] = f[l];
  for (int m = 1; m <= T.r - 1; ++m) {
    for (int l = 0; l + m < T.r; ++l) tab[l] = tab[l + 1] - tab[l];
    dif[m - 1] = tab[0];  // Delta^m f_0
  }
  double beta = 0.0;
  for (int j = 1; j <= T.r - 1; ++j) {
    for (int q = 0; q < T.nq; ++q) {
      double d = 0.0;
      for (int m = j; m <= T.r - 1; ++m) d += T.M[j - 1][q][m - 1] * dif[m - 1];
      beta += T.w[q] * d * d;
    }
  }
  return beta;
}

// ------------------------------------------------- scalar TENO-AA reconstruction
// Flag byte: bits 0-1 = chosen large stencil (0 none, 1 S3, 2 S4, 3 S5 or,
// with bit 2 set, S6), bits 2-4 = delta_0..delta_2 of the fallback (free when
// a large stencil is chosen), bits 5-7 = [beta] - 7.
struct Decision {
  uint8_t flag = 0;
  double margin = INFINITY;  // min relative distance of any decision to its threshold
};

// Candidate fluxes of Sec. 4.2 at x_{i+1/2}; fk points at f_{i} inside the window.
template <class T>
T small_flux(int k, const T* fi) {
  if (k == 0) return ((-fi[-1] + 5.0 * fi[0]) + 2.0 * fi[1]) / 6.0;
  if (k == 1) return ((2.0 * fi[0] + 5.0 * fi[1]) - fi[2]) / 6.0;
  return ((2.0 * fi[-2] - 7.0 * fi[-1]) + 11.0 * fi[0]) / 6.0;
}

template <class T>
T large_flux(int k, const T* fi) {
  const double* c = (k == 3) ? LIN6 : (k == 4) ? LIN8 : (k == 5) ? LIN10 : LIN12;
  const int lo = ST_LO[k], r = ST_R[k];
  T acc = c[0] * fi[lo];
  for (int m = 1; m < r; ++m) acc = fmaT(T(c[m]), fi[lo + m], acc);
  return acc;
}

template <class T>
T fallback_flux(uint8_t dmask, const T* fi) {
  const double del[3] = {(dmask & 1) ? 1.0 : 0.0, (dmask & 2) ? 1.0 : 0.0, (dmask & 4) ? 1.0 : 0.0};
  const double dsum = (DK[0] * del[0] + DK[1] * del[1]) + DK[2] * del[2];
  const double w0 = (DK[0] * del[0]) / dsum;
  const double w1 = (DK[1] * del[1]) / dsum;
  const double w2 = (DK[2] * del[2]) / dsum;
  return fmaT(T(w2), small_flux(2, fi), fmaT(T(w1), small_flux(1, fi), w0 * small_flux(0, fi)));
}

double rel_margin(double chi, double ct) { return std::fabs(chi / ct - 1.0); }

// Large stencil p (3..6) as a flag byte's bits 0-2.
int sel_bits(int p) { return p == 6 ? (3 | 4) : p - 2; }

// fv = f_{-G+1..G} (r = 2G values); i sits at index G-1.  order is 8, 10 or
// 12.  If frozen is non-null the decisions are taken from *frozen instead.
template <class T>
T teno_aa(int order, const T* fv, Decision* dec, const uint8_t* frozen) {
  const int G = order / 2;
  const T* fi = fv + (G - 1);
  if (frozen) {
    const uint8_t fl = *frozen;
    const int sel = fl & 3;
    if (sel == 3 && (fl & 4)) return large_flux(6, fi);
    if (sel) return large_flux(sel + 2, fi);
    return fallback_flux<T>((fl >> 2) & 7, fi);
  }
  double f[12];
  for (int l = 0; l < order; ++l) f[l] = re(fv[l]);
  const double* x = f + (G - 1);  // x[k] = f_{i+k}

  // Sec. 3.4: eta_j over j = -1..2, eta_{j+1/2} = min, m, g(m), [beta], C_T.
  double etabar = 0.0;
  for (int j = -1; j <= 2; ++j) {
    const double a = x[j + 1] - x[j];
    const double b = x[j] - x[j - 1];
    const double eta = (std::fabs((2.0 * a) * b) + EPS) / ((a * a + b * b) + EPS);
    if (j == -1 || eta < etabar) etabar = eta;
  }
  double ratio = etabar / C_R;
  if (ratio > 1.0) ratio = 1.0;
  const double m = 1.0 - ratio;
  const double om = 1.0 - m;
  const double om2 = om * om;
  const double g = (om2 * om2) * (1.0 + 4.0 * m);
  const double B = ALPHA1 - ALPHA2 * (1.0 - g);
  int K = (int)std::floor(B);
  if (K < 7) K = 7;
  if (K > 14) K = 14;
  const double CT = CT_OF_K[K];
  Decision d;
  if (m > 0.0) d.margin = std::min(d.margin, std::fabs(B - std::nearbyint(B)) / B);

  // Sec. 3.2: scale separation on the three small stencils.
  double gam[7];
  for (int k = 0; k < 3; ++k) {
    const double xb = beta_of(k, x + ST_LO[k]) + EPS;
    const double x2 = xb * xb, x4 = x2 * x2;
    gam[k] = 1.0 / ((x4 * x2) * xb);
  }
  // Sec. 3.3: groups (S0,S1,S2,Sp), largest p first.
  const int pmax = order / 2;
  for (int p = pmax; p >= 3; --p) {
    const double xb = beta_of(p, x + ST_LO[p]) + EPS;
    const double x2 = xb * xb, x4 = x2 * x2;
    gam[p] = 1.0 / ((x4 * x2) * xb);
    const double chi = gam[p] / (((gam[0] + gam[1]) + gam[2]) + gam[p]);
    d.margin = std::min(d.margin, rel_margin(chi, CT));
    if (chi >= CT) {
      d.flag = (uint8_t)(sel_bits(p) | ((K - 7) << 5));
      if (dec) *dec = d;
      return large_flux(p, fi);
    }
  }
  // Fallback: TENO5 cut-off on the small stencils, normalised among themselves.
  const double sum3 = (gam[0] + gam[1]) + gam[2];
  uint8_t dm = 0;
  for (int k = 0; k < 3; ++k) {
    const double chi = gam[k] / sum3;
    d.margin = std::min(d.margin, rel_margin(chi, CT));
    if (chi >= CT) dm |= (uint8_t)(1 << k);
  }
  d.flag = (uint8_t)((dm << 2) | ((K - 7) << 5));
  if (dec) *dec = d;
  return fallback_flux<T>(dm, fi);
}

// ------------------------------------------------------------- Euler system
struct Grid {
  int ndim;
  int64_t n[3];
  double dx[3];
  int bc_lo[3], bc_hi[3];
  // Boundary values of side (d, 0 = low / 1 = high), bc_sets sets each.
  // Dirichlet: per set nv planes of face primitives (rho, u_x, [u_y], [u_z], p)
  // over the face plane.  Inflow: per set G layers (ghost cell r = 1..G
  // outward from the face) of nv planes of the ghost cells' primitives.
  int bc_sets;
  const double* bc_values[3][2];
};
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_SYMMETRY = 2, BC_NOSLIP = 3, BC_DIRICHLET = 4, BC_INFLOW = 5 };

template <class T>
struct CellQ {
  T W[5];  // conserved, axis order (rho, m_x, [m_y], [m_z], E)
  T F[5];  // physical flux along the sweep direction, axis order
  T u[3];
  T p, c, H, sr;
};

// Sec. 1 (Euler equations, ideal-gas EOS), primitives of one cell.
template <class T>
void cell_state(int ndim, double gam, int d, const T* W, CellQ<T>& q) {
  const int nv = ndim + 2;
  for (int c = 0; c < nv; ++c) q.W[c] = W[c];
  const T rho = W[0];
  const T ir = 1.0 / rho;  // divisions by rho as products with its reciprocal
  T q2 = T(0.0);
  for (int k = 0; k < ndim; ++k) {
    q.u[k] = W[1 + k] * ir;
    q2 = (k == 0) ? q.u[0] * q.u[0] : q2 + q.u[k] * q.u[k];
  }
  const T E = W[nv - 1];
  q.p = (gam - 1.0) * (E - (0.5 * rho) * q2);
  q.c = sqrtT((gam * q.p) * ir);
  q.H = (E + q.p) * ir;
  q.sr = sqrtT(rho);
  const T un = q.u[d];
  q.F[0] = W[1 + d];
  for (int k = 0; k < ndim; ++k) q.F[1 + k] = (k == d) ? W[1 + k] * un + q.p : W[1 + k] * un;
  q.F[nv - 1] = (E + q.p) * un;
}

// Pressure of a conserved state, the same arithmetic as in cell_state.
template <class T>
T pressure_of(int ndim, double gam, const T* W) {
  const int nv = ndim + 2;
  const T rho = W[0];
  const T ir = 1.0 / rho;
  T q2 = T(0.0);
  for (int k = 0; k < ndim; ++k) {
    const T uk = W[1 + k] * ir;
    q2 = (k == 0) ? uk * uk : q2 + uk * uk;
  }
  return (gam - 1.0) * (W[nv - 1] - (0.5 * rho) * q2);
}

// Roe-averaged eigenvectors of the x_d flux Jacobian (Sec. 5, characteristic
// decomposition at the face).  Local frame: (rho, m_n, m_t1, [m_t2], E) with
// tangential axes in ascending order; fields (u-c, u, shear..., u+c).
template <class T>
struct Eigen {
  int nv;
  int perm[5];  // local component -> axis component
  T L[5][5], R[5][5];
};

template <class T>
void roe_eigen(int ndim, double gam, int d, const CellQ<T>& a, const CellQ<T>& b, Eigen<T>& e) {
  const int nv = ndim + 2;
  e.nv = nv;
  e.perm[0] = 0;
  e.perm[1] = 1 + d;
  int t = 2;
  for (int k = 0; k < ndim; ++k)
    if (k != d) e.perm[t++] = 1 + k;
  e.perm[nv - 1] = nv - 1;

  const T den = a.sr + b.sr;
  const T iden = 1.0 / den;  // the Roe weights' denominator, inverted once
  T ur[3];
  T q2 = T(0.0);
  for (int k = 0; k < ndim; ++k) {
    ur[k] = (a.sr * a.u[k] + b.sr * b.u[k]) * iden;
    q2 = (k == 0) ? ur[0] * ur[0] : q2 + ur[k] * ur[k];
  }
  const T H = (a.sr * a.H + b.sr * b.H) * iden;
  const T qq = 0.5 * q2;
  const T c2 = (gam - 1.0) * (H - qq);
  const T c = sqrtT(c2);
  const T b1 = (gam - 1.0) / c2;
  const T b2 = b1 * qq;
  const T un = ur[d];
  T ut[2];
  int nt = 0;
  for (int k = 0; k < ndim; ++k)
    if (k != d) ut[nt++] = ur[k];
  const T ic = 1.0 / c;
  const T unc = un * ic;

  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) e.L[i][j] = e.R[i][j] = T(0.0);
  const int last = nv - 1;
  // Left eigenvectors (rows).
  e.L[0][0] = 0.5 * (b2 + unc);
  e.L[0][1] = 0.5 * (-b1 * un - ic);
  e.L[1][0] = 1.0 - b2;
  e.L[1][1] = b1 * un;
  e.L[last][0] = 0.5 * (b2 - unc);
  e.L[last][1] = 0.5 * (-b1 * un + ic);
  for (int k = 0; k < nt; ++k) {
    e.L[0][2 + k] = 0.5 * (-b1 * ut[k]);
    e.L[1][2 + k] = b1 * ut[k];
    e.L[last][2 + k] = 0.5 * (-b1 * ut[k]);
    e.L[2 + k][0] = -ut[k];
    e.L[2 + k][2 + k] = T(1.0);
  }
  e.L[0][last] = 0.5 * b1;
  e.L[1][last] = -b1;
  e.L[last][last] = 0.5 * b1;
  // Right eigenvectors (columns).
  e.R[0][0] = T(1.0);
  e.R[1][0] = un - c;
  e.R[last][0] = H - un * c;
  e.R[0][1] = T(1.0);
  e.R[1][1] = un;
  e.R[last][1] = qq;
  e.R[0][last] = T(1.0);
  e.R[1][last] = un + c;
  e.R[last][last] = H + un * c;
  for (int k = 0; k < nt; ++k) {
    e.R[2 + k][0] = ut[k];
    e.R[2 + k][1] = ut[k];
    e.R[2 + k][last] = ut[k];
    e.R[2 + k][2 + k] = T(1.0);
    e.R[last][2 + k] = ut[k];
  }
}

// Characteristic speed of field s at a cell.
template <class T>
T char_speed(int nv, int s, const T& un, const T& c) {
  if (s == 0) return un - c;
  if (s == nv - 1) return un + c;
  return un;
}

struct Scheme {
  int order, splitting, positivity;
};


// Positivity limiter: a reading of Hu, Adams & Shu (2013), which the paper
// applies in its extreme cases (Sec. 5.3, opening paragraph) without restating.
// With mu = kappa_d * dt/dx_d the face flux F enters the two half-states
//   X+(F) = U_i - mu F,   X-(F) = U_{i+1} + mu F,
// whose weighted average is the forward-Euler update.  The first-order
// Lax-Friedrichs flux FL (alpha = max(|u_n|+c) over the two cells) keeps both
// half-states admissible when mu * alpha <= 1.  The high-order flux FH is
// pulled towards FL: first so that the density of both half-states stays
// >= min(1e-13, rho(X(FL))), then so that their pressure stays
// >= min(1e-13, p(X(FL))), using that pressure is concave in U.
// `thetas`, if given, receives (theta_rho, theta_p).
template <class T>
void limit_face(int ndim, double gam, int d, double mu, const CellQ<T>& a, const CellQ<T>& b, T* F,
                double* thetas = nullptr) {
  const int nv = ndim + 2;
  const T sa = absT(a.u[d]) + a.c;
  const T sb = absT(b.u[d]) + b.c;
  const T aL = (re(sa) >= re(sb)) ? sa : sb;
  T FL[5];
  for (int c = 0; c < nv; ++c) FL[c] = 0.5 * ((a.F[c] + b.F[c]) - aL * (b.W[c] - a.W[c]));
  T X[5];
  // density step
  double theta_r = 1.0;
  for (int side = 0; side < 2; ++side) {
    const CellQ<T>& cq = side == 0 ? a : b;
    const double sg = side == 0 ? -1.0 : 1.0;
    const double rL = re(cq.W[0] + (sg * mu) * FL[0]);
    const double rH = re(cq.W[0] + (sg * mu) * F[0]);
    const double eps = std::min(1e-13, rL);
    const double th = (rH < eps) ? (rL - eps) / (rL - rH) : 1.0;
    theta_r = std::min(theta_r, th);
  }
  T Fs[5];
  for (int c = 0; c < nv; ++c) Fs[c] = (theta_r < 1.0) ? FL[c] + theta_r * (F[c] - FL[c]) : F[c];
  // pressure step
  double theta_p = 1.0;
  for (int side = 0; side < 2; ++side) {
    const CellQ<T>& cq = side == 0 ? a : b;
    const double sg = side == 0 ? -1.0 : 1.0;
    for (int c = 0; c < nv; ++c) X[c] = cq.W[c] + (sg * mu) * FL[c];
    const double pL = re(pressure_of(ndim, gam, X));
    for (int c = 0; c < nv; ++c) X[c] = cq.W[c] + (sg * mu) * Fs[c];
    const double pS = re(pressure_of(ndim, gam, X));
    const double eps = std::min(1e-13, pL);
    const double th = (pS < eps) ? (pL - eps) / (pL - pS) : 1.0;
    theta_p = std::min(theta_p, th);
  }
  for (int c = 0; c < nv; ++c) F[c] = (theta_p < 1.0) ? FL[c] + theta_p * (Fs[c] - FL[c]) : Fs[c];
  if (thetas) {
    thetas[0] = theta_r;
    thetas[1] = theta_p;
  }
}

// Number of faces along direction d (face f is the left face of cell f).
int64_t faces_along(const Grid& g, int d) {
  return g.bc_lo[d] == BC_PERIODIC ? g.n[d] : g.n[d] + 1;
}
int64_t faces_total(const Grid& g, int d) {
  int64_t t = faces_along(g, d);
  for (int k = 0; k < g.ndim; ++k)
    if (k != d) t *= g.n[k];
  return t;
}
int64_t flag_offset(const Grid& g, int d) {
  int64_t off = 0;
  for (int k = 0; k < d; ++k) off += (int64_t)(g.ndim + 2) * 2 * faces_total(g, k);
  return off;
}

// Dirichlet ghost cell (Appendix A): in primitive variables the ghost is the
// mirror cell reflected through the prescribed face value,
// (rho, u, p)_ghost = 2 (rho, u, p)_face - (rho, u, p)_mirror, which makes the
// face value the second-order average of the two.  fv points at the face's
// density; its velocities and pressure follow at strides of `plane`.
template <class T>
void dirichlet_ghost(int ndim, double gam, const T* m, const double* fv, int64_t plane, T* out) {
  const int nv = ndim + 2;
  const T rho = m[0];
  const T ir = 1.0 / rho;
  T u[3];
  T q2 = T(0.0);
  for (int k = 0; k < ndim; ++k) {
    u[k] = m[1 + k] * ir;
    q2 = (k == 0) ? u[0] * u[0] : q2 + u[k] * u[k];
  }
  const T p = (gam - 1.0) * (m[nv - 1] - (0.5 * rho) * q2);
  const T rg = 2.0 * fv[0] - rho;
  T qg = T(0.0);
  for (int k = 0; k < ndim; ++k) {
    const T ug = 2.0 * fv[(1 + k) * plane] - u[k];
    out[1 + k] = rg * ug;
    qg = (k == 0) ? ug * ug : qg + ug * ug;
  }
  const T pg = 2.0 * fv[(nv - 1) * plane] - p;
  out[0] = rg;
  out[nv - 1] = pg / (gam - 1.0) + (0.5 * rg) * qg;
}

// Prescribed ghost cell (supersonic inflow, where every characteristic
// enters the domain): the conserved state of the given primitives.
template <class T>
void inflow_ghost(int ndim, double gam, const double* pv, int64_t plane, T* out) {
  const int nv = ndim + 2;
  const double rho = pv[0];
  double q2 = 0.0;
  for (int k = 0; k < ndim; ++k) {
    const double u = pv[(1 + k) * plane];
    out[1 + k] = T(rho * u);
    q2 = (k == 0) ? u * u : q2 + u * u;
  }
  out[0] = T(rho);
  out[nv - 1] = T(pv[(nv - 1) * plane] / (gam - 1.0) + (0.5 * rho) * q2);
}

// Ghost cells in conserved variables along one pencil (Appendix A).  fv: the
// boundary values of this pencil's side in its value set (Dirichlet, inflow).
template <class T>
void fill_ghosts(int ndim, double gam, int d, int bc, bool low, int64_t n, int G, const double* fv, int64_t plane,
                 std::vector<T>& line) {
  const int nv = ndim + 2;
  auto at = [&](int64_t l) -> T* { return &line[(size_t)(l + G) * nv]; };
  for (int r = 1; r <= G; ++r) {
    const int64_t dst = low ? -r : n - 1 + r;
    int64_t src;
    if (bc == BC_PERIODIC) src = low ? n - r : r - 1;
    else if (bc == BC_OUTFLOW) src = low ? 0 : n - 1;
    else src = low ? r - 1 : n - r;  // mirror
    if (bc == BC_DIRICHLET) {
      dirichlet_ghost<T>(ndim, gam, at(src), fv, plane, at(dst));
      continue;
    }
    if (bc == BC_INFLOW) {
      inflow_ghost<T>(ndim, gam, fv + (int64_t)(r - 1) * nv * plane, plane, at(dst));
      continue;
    }
    for (int c = 0; c < nv; ++c) at(dst)[c] = at(src)[c];
    if (bc == BC_SYMMETRY) at(dst)[1 + d] = -at(dst)[1 + d];
    if (bc == BC_NOSLIP)
      for (int k = 0; k < ndim; ++k) at(dst)[1 + k] = -at(dst)[1 + k];
  }
}

// Cells of the face plane of direction d (the grid without axis d).
int64_t plane_cells(const Grid& g, int d) {
  int64_t t = 1;
  for (int k = 0; k < 3; ++k)
    if (k != d) t *= g.n[k];
  return t;
}

// Boundary values of side (d, hi) in value set `set` at plane cell pidx
// (remaining axes, the lower one fastest), or null if the side takes none.
// A set holds one layer of nv planes (Dirichlet) or G layers (inflow).
const double* face_values(const Grid& g, int G, int d, int hi, int set, int64_t pidx) {
  const int bc = hi ? g.bc_hi[d] : g.bc_lo[d];
  if (bc != BC_DIRICHLET && bc != BC_INFLOW) return nullptr;
  const int64_t plane = plane_cells(g, d);
  const int64_t layers = bc == BC_INFLOW ? G : 1;
  return g.bc_values[d][hi] + (int64_t)set * layers * (g.ndim + 2) * plane + pidx;
}

// a_d = max of |u_d| + c over the cells and over the ghost cells next to the
// faces of every side with prescribed values (Dirichlet, inflow; value set 0),
// whose states the boundary faces see; the ghosts of the other boundaries
// copy domain cells.  Used for dt and the limiter weights.
void wave_speeds(const Grid& g, double gam, const double* U, double* amax) {
  const int nv = g.ndim + 2;
  const int64_t nc = g.n[0] * g.n[1] * g.n[2];
  for (int d = 0; d < 3; ++d) amax[d] = 0.0;
  double W[5];
  CellQ<double> q;
  auto fold = [&](const double* w) {
    cell_state(g.ndim, gam, 0, w, q);
    for (int d = 0; d < g.ndim; ++d) amax[d] = std::max(amax[d], std::fabs(q.u[d]) + q.c);
  };
  for (int64_t i = 0; i < nc; ++i) {
    for (int c = 0; c < nv; ++c) W[c] = U[c * nc + i];
    fold(W);
  }
  const int64_t stride[3] = {1, g.n[0], g.n[0] * g.n[1]};
  double Gh[5];
  for (int d = 0; d < g.ndim; ++d) {
    int oa[2], no = 0;
    for (int k = 0; k < 3; ++k)
      if (k != d) oa[no++] = k;
    const int64_t plane = plane_cells(g, d);
    for (int hi = 0; hi < 2; ++hi) {
      const int bc = hi ? g.bc_hi[d] : g.bc_lo[d];
      if (bc != BC_DIRICHLET && bc != BC_INFLOW) continue;
      for (int64_t o1 = 0; o1 < g.n[oa[1]]; ++o1)
        for (int64_t o0 = 0; o0 < g.n[oa[0]]; ++o0) {
          const int64_t pidx = o0 + g.n[oa[0]] * o1;
          const int64_t cell = (hi ? g.n[d] - 1 : 0) * stride[d] + o0 * stride[oa[0]] + o1 * stride[oa[1]];
          // the G argument only places inflow layers, and layer 1 is first in either case
          const double* fv = face_values(g, 1, d, hi, 0, pidx);
          if (bc == BC_DIRICHLET) {
            for (int c = 0; c < nv; ++c) W[c] = U[c * nc + cell];
            dirichlet_ghost<double>(g.ndim, gam, W, fv, plane, Gh);
          } else {
            inflow_ghost<double>(g.ndim, gam, fv, plane, Gh);
          }
          fold(Gh);
        }
    }
  }
}

// dt = CFL / sum_d a_d/dx_d, once per step from U^n (Sec. 5, CFL 0.4 typical).
double dt_from(const Grid& g, double cfl, const double* amax) {
  double s = amax[0] / g.dx[0];
  for (int d = 1; d < g.ndim; ++d) s = s + amax[d] / g.dx[d];
  return cfl / s;
}

// Numerical flux of direction d at face f (between cells f-1 and f) of one
// pencil; cl[l] is the cell record of pencil cell l, l = -G .. n+G-1.
// Decisions go to flags/margins at fbase + (2 s + side) * nft when given.
template <class T>
void face_flux(const Grid& g, const Scheme& sc, double gam, int d, const CellQ<T>* cl, int64_t f, double mu,
               bool limit, int64_t fbase, int64_t nft, uint8_t* flags, double* margins, const uint8_t* frozen,
               T* Fo) {
  const int nd = g.ndim, nv = nd + 2, G = sc.order / 2;
  const CellQ<T>* win = cl + (f - G);  // window of cells f-G .. f+G-1
  const CellQ<T>& ca = cl[f - 1];
  const CellQ<T>& cb = cl[f];
  Eigen<T> e;
  roe_eigen(nd, gam, d, ca, cb, e);
  T v[12], gch[12], gp[12], gm[12], fv[12];
  T fhat[5];
  for (int s = 0; s < nv; ++s) {
    // projection onto field s of the conserved state and physical flux
    for (int j = 0; j < 2 * G; ++j) {
      T av = e.L[s][0] * win[j].W[e.perm[0]];
      T ag = e.L[s][0] * win[j].F[e.perm[0]];
      for (int c = 1; c < nv; ++c) {
        av = fmaT(e.L[s][c], win[j].W[e.perm[c]], av);
        ag = fmaT(e.L[s][c], win[j].F[e.perm[c]], ag);
      }
      v[j] = av;
      gch[j] = ag;
    }
    // splitting speed over the window: LLF per field (also the Roe flux's
    // fallback), Rusanov one for all fields
    T alpha = T(-1.0);
    for (int j = 0; j < 2 * G; ++j) {
      const T un = win[j].u[d];
      const T lam = sc.splitting != 1 ? absT(char_speed(nv, s, un, win[j].c)) : absT(un) + win[j].c;
      if (re(lam) > re(alpha)) alpha = lam;
    }
    for (int j = 0; j < 2 * G; ++j) {
      gp[j] = 0.5 * fmaT(alpha, v[j], gch[j]);
      gm[j] = 0.5 * fmaT(-alpha, v[j], gch[j]);
    }
    // Roe flux with entropy fix: where the field's eigenvalue has one strict
    // sign at both cells of the face, the unsplit characteristic flux is
    // reconstructed from the upwind side only; elsewhere (a sonic point, or
    // a zero eigenvalue) the field falls back to the LLF split above.
    // With recorded decisions the side is replayed too: the side whose byte
    // is 0 was not reconstructed.
    int upwind = 0;  // 0: split, 1: + side only, 2: - side only
    if (sc.splitting == 2 && frozen) {
      const uint8_t bp = frozen[fbase + ((int64_t)s * 2) * nft];
      const uint8_t bm = frozen[fbase + ((int64_t)s * 2 + 1) * nft];
      upwind = bm == 0 ? 1 : (bp == 0 ? 2 : 0);
    } else if (sc.splitting == 2) {
      const double la = re(char_speed(nv, s, ca.u[d], ca.c));
      const double lb = re(char_speed(nv, s, cb.u[d], cb.c));
      upwind = (la > 0.0 && lb > 0.0) ? 1 : ((la < 0.0 && lb < 0.0) ? 2 : 0);
    }
    if (upwind) {
      const int side = upwind - 1;
      for (int k = 0; k < 2 * G; ++k) fv[k] = side == 0 ? gch[k] : gch[2 * G - 1 - k];
      const int64_t fi = fbase + ((int64_t)s * 2 + side) * nft;
      const int64_t fo = fbase + ((int64_t)s * 2 + (1 - side)) * nft;
      Decision dec;
      fhat[s] = teno_aa(sc.order, fv, &dec, frozen ? frozen + fi : nullptr);
      if (flags && !frozen) {
        flags[fi] = dec.flag;
        flags[fo] = 0;  // the side not reconstructed (no real decision has this byte)
      }
      if (margins && !frozen) {
        margins[fi] = dec.margin;
        margins[fo] = 1.0;
      }
      continue;
    }
    T sum = T(0.0);
    for (int side = 0; side < 2; ++side) {
      // + side: f_k = g+_{i+k}; - side mirrored: f_k = g-_{i+1-k}
      for (int k = 0; k < 2 * G; ++k) fv[k] = side == 0 ? gp[k] : gm[2 * G - 1 - k];
      const int64_t fi = fbase + ((int64_t)s * 2 + side) * nft;
      Decision dec;
      const T h = teno_aa(sc.order, fv, &dec, frozen ? frozen + fi : nullptr);
      if (flags && !frozen) flags[fi] = dec.flag;
      if (margins && !frozen) margins[fi] = dec.margin;
      sum = side == 0 ? h : sum + h;
    }
    fhat[s] = sum;
  }
  // back to conserved components: F = sum_s R[:,s] fhat_s, then axis order
  for (int c = 0; c < nv; ++c) {
    T acc = e.R[c][0] * fhat[0];
    for (int s = 1; s < nv; ++s) acc = fmaT(e.R[c][s], fhat[s], acc);
    Fo[e.perm[c]] = acc;
  }
  if (limit) limit_face(nd, gam, d, mu, ca, cb, Fo);
}

// Conserved pencil of direction d through (o0, o1) with G ghost cells per
// side, and its cell records (cells[l + G] for l = -G .. n+G-1).
// pidx: the pencil's cell of the face plane; set: the Dirichlet value set.
template <class T>
void load_pencil(const Grid& g, double gam, int d, int G, const T* U, int64_t base, int64_t pidx, int set,
                 std::vector<T>& line, std::vector<CellQ<T>>& cells) {
  const int nd = g.ndim, nv = nd + 2;
  const int64_t n = g.n[d];
  const int64_t nc = g.n[0] * g.n[1] * g.n[2];
  const int64_t stride[3] = {1, g.n[0], g.n[0] * g.n[1]};
  const int64_t plane = plane_cells(g, d);
  for (int64_t l = 0; l < n; ++l)
    for (int c = 0; c < nv; ++c) line[(size_t)(l + G) * nv + c] = U[c * nc + base + l * stride[d]];
  fill_ghosts(nd, gam, d, g.bc_lo[d], true, n, G, face_values(g, G, d, 0, set, pidx), plane, line);
  fill_ghosts(nd, gam, d, g.bc_hi[d], false, n, G, face_values(g, G, d, 1, set, pidx), plane, line);
  for (int64_t l = -G; l < n + G; ++l) cell_state(nd, gam, d, &line[(size_t)(l + G) * nv], cells[(size_t)(l + G)]);
}

// Semi-discrete right-hand side dU/dt = -sum_d (F_{i+1/2} - F_{i-1/2})/dx_d
// (Sec. 2, conservative finite-difference form), directions in order x, y, z.
// face_out[d], if given, receives the face fluxes of direction d, layout
// [nv][faces of d] in the flag arrays' face order.
template <class T>
int rhs_impl(const Grid& g, const Scheme& sc, double gam, const T* U, T* dU, double dt_lim, const double* amax,
             uint8_t* flags, double* margins, const uint8_t* frozen, int set = 0, double* const* face_out = nullptr) {
  const int nd = g.ndim, nv = nd + 2, G = sc.order / 2;
  const int64_t nc = g.n[0] * g.n[1] * g.n[2];
  for (int64_t i = 0; i < nv * nc; ++i) dU[i] = T(0.0);
  const bool limit = sc.positivity && dt_lim > 0.0;
  double mu[3] = {0, 0, 0};
  if (limit) {
    double S = (dt_lim / g.dx[0]) * amax[0];
    for (int d = 1; d < nd; ++d) S = S + (dt_lim / g.dx[d]) * amax[d];
    for (int d = 0; d < nd; ++d) mu[d] = (2.0 * S) / amax[d];
  }
  const int64_t stride[3] = {1, g.n[0], g.n[0] * g.n[1]};
  for (int d = 0; d < nd; ++d) {
    const int64_t n = g.n[d];
    const bool periodic = g.bc_lo[d] == BC_PERIODIC;
    const double rdx = 1.0 / g.dx[d];  // the flux difference divides by dx as a product
    const int64_t nf = faces_along(g, d);
    const int64_t nft = faces_total(g, d);
    const int64_t foff = flag_offset(g, d);
    int oa[2];
    int no = 0;
    for (int k = 0; k < 3; ++k)
      if (k != d) oa[no++] = k;
    std::vector<T> line((size_t)(n + 2 * G) * nv);
    std::vector<CellQ<T>> cells((size_t)(n + 2 * G));
    std::vector<T> Fh((size_t)nf * nv);
    for (int64_t o1 = 0; o1 < g.n[oa[1]]; ++o1) {
      for (int64_t o0 = 0; o0 < g.n[oa[0]]; ++o0) {
        const int64_t base = o0 * stride[oa[0]] + o1 * stride[oa[1]];
        load_pencil(g, gam, d, G, U, base, o0 + g.n[oa[0]] * o1, set, line, cells);
        for (int64_t f = 0; f < nf; ++f) {
          // face linear index inside the flag array of direction d
          int64_t idx[3] = {0, 0, 0};
          idx[d] = f;
          idx[oa[0]] = o0;
          idx[oa[1]] = o1;
          const int64_t m0 = (d == 0) ? nf : g.n[0];
          const int64_t m1 = (d == 1) ? nf : g.n[1];
          const int64_t flin = (idx[2] * m1 + idx[1]) * m0 + idx[0];
          face_flux<T>(g, sc, gam, d, cells.data() + G, f, limit ? mu[d] : 0.0, limit, foff + flin, nft, flags,
                       margins, frozen, &Fh[(size_t)f * nv]);
          if (face_out && face_out[d])
            for (int c = 0; c < nv; ++c) face_out[d][c * nft + flin] = re(Fh[(size_t)f * nv + c]);
        }
        for (int64_t i = 0; i < n; ++i) {
          const int64_t fr = periodic ? (i + 1) % n : i + 1;
          for (int c = 0; c < nv; ++c) {
            const int64_t cell = c * nc + base + i * stride[d];
            dU[cell] = dU[cell] - (Fh[(size_t)fr * nv + c] - Fh[(size_t)i * nv + c]) * rdx;
          }
        }
      }
    }
  }
  return 0;
}

// SSP-RK3 in the Shu-Osher form printed in Sec. 5:
//   u1 = un + dt L(un)
//   u2 = 3/4 un + 1/4 u1 + 1/4 dt L(u1)
//   u^{n+1} = 1/3 un + 2/3 u2 + 2/3 dt L(u2)
// L(stage, in, out) evaluates the right-hand side of stage 0, 1, 2.
template <class RHS>
void ssp_rk3(int64_t N, double dt, double* U, RHS&& L) {
  std::vector<double> Un(U, U + N), U1((size_t)N), U2((size_t)N), dU((size_t)N);
  L(0, Un.data(), dU.data());
  for (int64_t i = 0; i < N; ++i) U1[(size_t)i] = Un[(size_t)i] + dt * dU[(size_t)i];
  L(1, U1.data(), dU.data());
  for (int64_t i = 0; i < N; ++i)
    U2[(size_t)i] = 0.75 * Un[(size_t)i] + 0.25 * U1[(size_t)i] + (0.25 * dt) * dU[(size_t)i];
  L(2, U2.data(), dU.data());
  for (int64_t i = 0; i < N; ++i)
    U[i] = (1.0 / 3.0) * Un[(size_t)i] + (2.0 / 3.0) * U2[(size_t)i] + ((2.0 / 3.0) * dt) * dU[(size_t)i];
}

int check_grid(const Grid& g, const Scheme& s) {
  if (g.ndim < 1 || g.ndim > 3) return -1;
  if (s.order != 8 && s.order != 10 && s.order != 12) return -1;
  for (int d = 0; d < 3; ++d) {
    if (g.n[d] < 1) return -1;
    if (d < g.ndim) {
      if (g.n[d] < s.order / 2 || g.dx[d] <= 0.0) return -1;
      if ((g.bc_lo[d] == BC_PERIODIC) != (g.bc_hi[d] == BC_PERIODIC)) return -1;
      if (g.bc_lo[d] < 0 || g.bc_lo[d] > 5 || g.bc_hi[d] < 0 || g.bc_hi[d] > 5) return -1;
      for (int h = 0; h < 2; ++h)
        if ((h ? g.bc_hi[d] : g.bc_lo[d]) >= BC_DIRICHLET) {
          if (!g.bc_values[d][h] || (g.bc_sets != 1 && g.bc_sets != 3)) return -1;
        }
    } else if (g.n[d] != 1) {
      return -1;
    }
  }
  return 0;
}

}  // namespace

// ------------------------------------------------------------------ C API
extern "C" {

// bc_values[d][0/1]: host arrays of the boundary values of the low/high side
// of direction d, bc_sets (1 or 3) sets, each of nv planes of primitives
// (rho, u_x, [u_y], [u_z], p) over the face plane (Dirichlet: the face
// values; inflow: order/2 such layers, the ghost cells outward from the
// face); or_step uses set s in stage s when bc_sets is 3, every other call
// set 0.
struct or_grid {
  int32_t ndim;
  int32_t bc_sets;
  int64_t n[3];
  double dx[3];
  int32_t bc_lo[3];
  int32_t bc_hi[3];
  const double* bc_values[3][2];
};

static Grid to_grid(const or_grid* g) {
  Grid r;
  r.ndim = g->ndim;
  r.bc_sets = g->bc_sets;
  for (int d = 0; d < 3; ++d) {
    r.n[d] = g->n[d];
    r.dx[d] = g->dx[d];
    r.bc_lo[d] = g->bc_lo[d];
    r.bc_hi[d] = g->bc_hi[d];
    r.bc_values[d][0] = g->bc_values[d][0];
    r.bc_values[d][1] = g->bc_values[d][1];
  }
  return r;
}

// beta of candidate k (0..6) for the values of its stencil, leftmost first.
double or_beta(int k, const double* f) {
  build_beta_tables();
  if (k < 0 || k > 6) return NAN;
  return beta_of(k, f);
}

// Scalar TENO-AA reconstruction of f_{i+1/2} from f_{-G+1..G}.
double or_teno(int order, const double* fv, uint8_t* flag, double* margin) {
  build_beta_tables();
  Decision d;
  const double h = teno_aa(order, fv, &d, nullptr);
  if (flag) *flag = d.flag;
  if (margin) *margin = d.margin;
  return h;
}

// Candidate flux k (0..6) at i+1/2; fi points at f_i inside a long enough array.
double or_candidate_flux(int k, const double* fi) {
  if (k < 3) return small_flux(k, fi);
  return large_flux(k, fi);
}

void or_wave_speeds(const or_grid* g, double gam, const double* U, double* amax) {
  wave_speeds(to_grid(g), gam, U, amax);
}

double or_dt(const or_grid* g, double gam, double cfl, const double* U) {
  double a[3];
  Grid G = to_grid(g);
  wave_speeds(G, gam, U, a);
  return dt_from(G, cfl, a);
}

int64_t or_flags_size(const or_grid* g) {
  Grid G = to_grid(g);
  return flag_offset(G, G.ndim);
}

// One RHS.  The limiter acts only if positivity != 0 and dt_lim > 0; its wave
// speeds a_d are taken from U.  flags/margins may be null.
int or_rhs(const or_grid* g, int order, int splitting, int positivity, double gam, const double* U, double* dU,
           double dt_lim, uint8_t* flags, double* margins) {
  build_beta_tables();
  Grid G = to_grid(g);
  Scheme s{order, splitting, positivity};
  if (check_grid(G, s)) return -1;
  double a[3] = {0, 0, 0};
  if (positivity && dt_lim > 0.0) wave_speeds(G, gam, U, a);
  return rhs_impl<double>(G, s, gam, U, dU, dt_lim, a, flags, margins, nullptr);
}

// dU/dt at the listed cells only (flat cell indices), written to out[k*nv + c].
// amax (wave speeds of the whole state, for the limiter) may be null when the
// limiter is off.  Used to check full-size results at sampled cells.
// Face fluxes of every direction for the right-hand side or_rhs would
// evaluate: F[d] (nv x faces of d, flag-array face order) for d < ndim.
int or_face_fluxes(const or_grid* g, int order, int splitting, int positivity, double gam, const double* U,
                   double dt_lim, double* F0, double* F1, double* F2) {
  build_beta_tables();
  Grid G = to_grid(g);
  Scheme s{order, splitting, positivity};
  if (check_grid(G, s)) return -1;
  double amax[3];
  wave_speeds(G, gam, U, amax);
  const int64_t nc = G.n[0] * G.n[1] * G.n[2];
  std::vector<double> dU((size_t)(G.ndim + 2) * nc);
  double* fo[3] = {F0, F1, F2};
  return rhs_impl<double>(G, s, gam, U, dU.data(), dt_lim, amax, nullptr, nullptr, nullptr, 0, fo);
}

int or_rhs_cells(const or_grid* g, int order, int splitting, int positivity, double gam, const double* U,
                 double dt_lim, const double* amax, int64_t ncells, const int64_t* cells, double* out) {
  build_beta_tables();
  Grid G = to_grid(g);
  Scheme s{order, splitting, positivity};
  if (check_grid(G, s)) return -1;
  const int nd = G.ndim, nv = nd + 2, Gh = order / 2;
  const bool limit = positivity && dt_lim > 0.0;
  double mu[3] = {0, 0, 0};
  if (limit) {
    if (!amax) return -1;
    double S = (dt_lim / G.dx[0]) * amax[0];
    for (int d = 1; d < nd; ++d) S = S + (dt_lim / G.dx[d]) * amax[d];
    for (int d = 0; d < nd; ++d) mu[d] = (2.0 * S) / amax[d];
  }
  const int64_t stride[3] = {1, G.n[0], G.n[0] * G.n[1]};
  for (int64_t k = 0; k < ncells; ++k) {
    const int64_t cell = cells[k];
    const int64_t co[3] = {cell % G.n[0], (cell / G.n[0]) % G.n[1], cell / (G.n[0] * G.n[1])};
    double du[5] = {0, 0, 0, 0, 0};
    for (int d = 0; d < nd; ++d) {
      const int64_t n = G.n[d];
      const bool periodic = G.bc_lo[d] == BC_PERIODIC;
      std::vector<double> line((size_t)(n + 2 * Gh) * nv);
      std::vector<CellQ<double>> cq((size_t)(n + 2 * Gh));
      const int64_t base = cell - co[d] * stride[d];
      int oa[2], no = 0;
      for (int k2 = 0; k2 < 3; ++k2)
        if (k2 != d) oa[no++] = k2;
      load_pencil(G, gam, d, Gh, U, base, co[oa[0]] + G.n[oa[0]] * co[oa[1]], 0, line, cq);
      double Fl[5], Fr[5];
      const int64_t i = co[d];
      const int64_t fr = periodic ? (i + 1) % n : i + 1;
      face_flux<double>(G, s, gam, d, cq.data() + Gh, i, mu[d], limit, 0, 0, nullptr, nullptr, nullptr, Fl);
      face_flux<double>(G, s, gam, d, cq.data() + Gh, fr, mu[d], limit, 0, 0, nullptr, nullptr, nullptr, Fr);
      const double rdx = 1.0 / G.dx[d];
      for (int c = 0; c < nv; ++c) du[c] = du[c] - (Fr[c] - Fl[c]) * rdx;
    }
    for (int c = 0; c < nv; ++c) out[k * nv + c] = du[c];
  }
  return 0;
}

// RHS with every decision frozen to the given flags and its exact directional
// derivative along V (forward mode): rhs_out = RHS(U), jvp = J(U) V.
int or_rhs_jvp(const or_grid* g, int order, int splitting, double gam, const double* U, const double* V,
               const uint8_t* flags, double* rhs_out, double* jvp) {
  build_beta_tables();
  Grid G = to_grid(g);
  Scheme s{order, splitting, 0};
  if (check_grid(G, s) || !flags) return -1;
  const int64_t N = (int64_t)(G.ndim + 2) * G.n[0] * G.n[1] * G.n[2];
  std::vector<Dual> Ud((size_t)N), dUd((size_t)N);
  for (int64_t i = 0; i < N; ++i) Ud[(size_t)i] = Dual(U[i], V[i]);
  double a[3] = {0, 0, 0};
  rhs_impl<Dual>(G, s, gam, Ud.data(), dUd.data(), 0.0, a, nullptr, nullptr, flags);
  for (int64_t i = 0; i < N; ++i) {
    if (rhs_out) rhs_out[i] = dUd[(size_t)i].v;
    jvp[i] = dUd[(size_t)i].d;
  }
  return 0;
}

// Directional derivative of one SSP-RK3 step along V with dt fixed and each
// stage's decisions frozen to flags3 (stage-major, as written by or_step),
// in forward mode through the three stages.  Limiter off.
// With positivity the limiter acts in every stage as in or_step (its wave
// speeds from U, dt the given one); its factors theta are evaluated from the
// values and so enter as constants: F = F_LF + theta (F_H - F_LF) is
// differentiated with theta frozen.
int or_step_jvp(const or_grid* g, int order, int splitting, int positivity, double gam, const double* U,
                const double* V, double dt, const uint8_t* flags3, double* jvp) {
  build_beta_tables();
  Grid G = to_grid(g);
  Scheme s{order, splitting, positivity};
  if (check_grid(G, s) || !flags3 || !(dt > 0.0)) return -1;
  const int64_t N = (int64_t)(G.ndim + 2) * G.n[0] * G.n[1] * G.n[2];
  const int64_t nfl = flag_offset(G, G.ndim);
  std::vector<Dual> Un((size_t)N), U1((size_t)N), U2((size_t)N), L((size_t)N);
  for (int64_t i = 0; i < N; ++i) Un[(size_t)i] = Dual(U[i], V[i]);
  double a[3] = {0, 0, 0};
  if (positivity) wave_speeds(G, gam, U, a);
  const double dl = positivity ? dt : 0.0;
  rhs_impl<Dual>(G, s, gam, Un.data(), L.data(), dl, a, nullptr, nullptr, flags3);
  for (int64_t i = 0; i < N; ++i) U1[(size_t)i] = Un[(size_t)i] + dt * L[(size_t)i];
  rhs_impl<Dual>(G, s, gam, U1.data(), L.data(), dl, a, nullptr, nullptr, flags3 + nfl, G.bc_sets == 3 ? 1 : 0);
  for (int64_t i = 0; i < N; ++i)
    U2[(size_t)i] = 0.75 * Un[(size_t)i] + 0.25 * U1[(size_t)i] + (0.25 * dt) * L[(size_t)i];
  rhs_impl<Dual>(G, s, gam, U2.data(), L.data(), dl, a, nullptr, nullptr, flags3 + 2 * nfl, G.bc_sets == 3 ? 2 : 0);
  for (int64_t i = 0; i < N; ++i) {
    const Dual u3 = (1.0 / 3.0) * Un[(size_t)i] + (2.0 / 3.0) * U2[(size_t)i] + ((2.0 / 3.0) * dt) * L[(size_t)i];
    jvp[i] = u3.d;
  }
  return 0;
}

// One SSP-RK3 step (Sec. 5, Shu-Osher form) in place.  *dt > 0 is used as
// given, otherwise dt = CFL / sum_d a_d/dx_d from U^n and written back.
// flags3/margins3 (optional) receive the decisions of the three stages.
int or_step(const or_grid* g, int order, int splitting, int positivity, double gam, double cfl, double* U,
            double* dt, uint8_t* flags3, double* margins3) {
  build_beta_tables();
  Grid G = to_grid(g);
  Scheme s{order, splitting, positivity};
  if (check_grid(G, s)) return -1;
  const int64_t N = (int64_t)(G.ndim + 2) * G.n[0] * G.n[1] * G.n[2];
  const int64_t nfl = flag_offset(G, G.ndim);
  double a[3];
  wave_speeds(G, gam, U, a);
  if (!(*dt > 0.0)) *dt = dt_from(G, cfl, a);
  const double h = *dt;
  ssp_rk3(N, h, U, [&](int st, const double* in, double* out) {
    rhs_impl<double>(G, s, gam, in, out, h, a, flags3 ? flags3 + st * nfl : nullptr,
                     margins3 ? margins3 + st * nfl : nullptr, nullptr, G.bc_sets == 3 ? st : 0);
  });
  return 0;
}

// Scalar linear advection u_t + u_x = 0 on a periodic grid (Sec. 5.1): the
// flux is f = u with positive speed, so only the upwind-biased reconstruction
// enters.  dudt = -(fhat_{i+1/2} - fhat_{i-1/2})/dx.
int or_advect_rhs(int order, int64_t n, double dx, const double* u, double* dudt, uint8_t* flags) {
  build_beta_tables();
  if ((order != 8 && order != 10 && order != 12) || n < order) return -1;
  const int G = order / 2;
  std::vector<double> fh((size_t)n), fv((size_t)(2 * G));
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 2 * G; ++k) fv[(size_t)k] = u[((i - G + 1 + k) % n + n) % n];
    Decision d;
    fh[(size_t)i] = teno_aa(order, fv.data(), &d, nullptr);  // fhat_{i+1/2}
    if (flags) flags[i] = d.flag;
  }
  for (int64_t i = 0; i < n; ++i) dudt[i] = -(fh[(size_t)i] - fh[(size_t)((i - 1 + n) % n)]) / dx;
  return 0;
}

// One SSP-RK3 step of the periodic scalar advection problem with time step dt.
int or_advect_step(int order, int64_t n, double dx, double dt, double* u, uint8_t* flags3) {
  if ((order != 8 && order != 10 && order != 12) || n < order) return -1;
  ssp_rk3(n, dt, u, [&](int st, const double* in, double* out) {
    or_advect_rhs(order, n, dx, in, out, flags3 ? flags3 + st * n : nullptr);
  });
  return 0;
}

// Roe-averaged eigen-system at a face of direction d between states Wa, Wb
// (axis order).  L and R are nv x nv row-major in the local frame; lam holds
// the characteristic speeds; perm maps local to axis components.
void or_eigen(int ndim, double gam, int d, const double* Wa, const double* Wb, double* L, double* R, double* lam,
              int32_t* perm) {
  CellQ<double> a, b;
  cell_state(ndim, gam, d, Wa, a);
  cell_state(ndim, gam, d, Wb, b);
  Eigen<double> e;
  roe_eigen(ndim, gam, d, a, b, e);
  const int nv = ndim + 2;
  for (int i = 0; i < nv; ++i) {
    perm[i] = e.perm[i];
    for (int j = 0; j < nv; ++j) {
      L[i * nv + j] = e.L[i][j];
      R[i * nv + j] = e.R[i][j];
    }
  }
  // speeds at the Roe state: the normal-momentum row of R holds u_n - c, u_n, u_n + c
  for (int s = 0; s < nv; ++s) lam[s] = (s == 0) ? e.R[1][0] : (s == nv - 1) ? e.R[1][nv - 1] : e.R[1][1];
}

// The positivity limiter of one face of direction d between the cells of
// conserved states Wa (left) and Wb (right), axis order, with factor mu =
// kappa_d dt / dx_d: F (axis order) holds the high-order flux on entry and the
// limited flux on return; thetas receives (theta_rho, theta_p).
void or_limit_face(int ndim, double gam, int d, double mu, const double* Wa, const double* Wb, double* F,
                   double* thetas) {
  CellQ<double> a, b;
  cell_state(ndim, gam, d, Wa, a);
  cell_state(ndim, gam, d, Wb, b);
  limit_face<double>(ndim, gam, d, mu, a, b, F, thetas);
}

}  // extern "C"
