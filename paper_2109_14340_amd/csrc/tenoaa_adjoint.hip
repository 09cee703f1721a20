// Adjoint (vector-Jacobian product) of the TENO-AA Euler right-hand side.
//
// For a state U and a seed R = dL/d(dU/dt), one sweep kernel per direction
// accumulates U_bar += (d(dU/dt)_d / dU)^T R with every threshold decision of
// the method frozen at U: the stencil chosen by the cascade and the cut-off
// deltas (Sec. 3.3 of the paper), hence the linear weights of each
// reconstruction; the cell that attains each LLF/Rusanov splitting speed and
// the sign of that speed.  Everything else - cell primitives, Roe average,
// eigenvectors, projection, split, back-projection - is differentiated
// exactly.  The positivity limiter is not differentiated (its callers reject
// it).
//
// The forward sweep of the same direction runs first and leaves, per face,
// the decision bytes and the per-field fluxes fh_s.  Per block: the tile of
// cells is staged exactly as in the forward sweep; each thread takes one face,
// recomputes the Roe average, eigenvectors, projections and splitting speeds,
// then runs the reverse pass and scatters the adjoints of the window cells'
// conserved states, physical fluxes and primitive quantities into LDS
// accumulators (ds_add_f64).  After a barrier the cell-level reverse
// pass turns those into conserved-state adjoints, maps ghost cells back to
// their interior source (with the momentum sign flips of wall conditions) and
// adds them to U_bar with global FP64 atomics, so the summation order - and
// the last bits of U_bar - can vary between runs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa_device.h"
#include "tenoaa_internal.h"

#ifndef TENOAA_ADJ_TN_X
#define TENOAA_ADJ_TN_X 64
#endif
#ifndef TENOAA_ADJ_TT_X
#define TENOAA_ADJ_TT_X 2
#endif
#ifndef TENOAA_ADJ_TN_YZ
#define TENOAA_ADJ_TN_YZ 16
#endif
#ifndef TENOAA_ADJ_TT_YZ
#define TENOAA_ADJ_TT_YZ 8
#endif
#ifndef TENOAA_ADJ_WAVES_PER_EU
#define TENOAA_ADJ_WAVES_PER_EU 0
#endif

namespace tenoaa {
namespace {

// Derivative of the frozen reconstruction chosen by `flag` with respect to
// the window values f_{-G+1..G} (w[q] = d fhat / d v[q]).
template <int ORDER>
__device__ __forceinline__ void recon_weights(uint8_t flag, double (&w)[ORDER]) {
  constexpr int G = ORDER / 2;
  constexpr int I = G - 1;
  unroll<ORDER>([&](auto q) { w[q] = 0.0; });
  const int sel = flag & 3;
  if (ORDER == 10 && sel == 3) {
    unroll<10>([&](auto q) {
      constexpr int qq = decltype(q)::value;
      if constexpr (qq < ORDER) w[qq] = lin_coef<10>(qq);
    });
  } else if (sel == 2) {
    constexpr int P = (ORDER == 10) ? 1 : 0;
    unroll<8>([&](auto q) { w[P + q] = lin_coef<8>(q); });
  } else if (sel == 1) {
    constexpr int P = (ORDER == 10) ? 2 : 1;
    unroll<6>([&](auto q) { w[P + q] = lin_coef<6>(q); });
  } else {
    const int dm = (flag >> 2) & 7;
    const double w0 = WFALL.w[dm][0], w1 = WFALL.w[dm][1], w2 = WFALL.w[dm][2];
    constexpr double s6 = 1.0 / 6.0;
    w[I - 2] = w2 * (2.0 * s6);
    w[I - 1] = w0 * (-s6) + w2 * (-7.0 * s6);
    w[I] = w0 * (5.0 * s6) + w1 * (2.0 * s6) + w2 * (11.0 * s6);
    w[I + 1] = w0 * (2.0 * s6) + w1 * (5.0 * s6);
    w[I + 2] = w1 * (-s6);
  }
}

__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }

template <int ORDER, int NDIM, int DIR, int TT, int TN>
__global__ __launch_bounds__(TT* TN)
#if TENOAA_ADJ_WAVES_PER_EU > 0
__attribute__((amdgpu_waves_per_eu(TENOAA_ADJ_WAVES_PER_EU)))
#endif
void sweep_vjp_kernel(AdjointArgs A) {
  constexpr int G = ORDER / 2;
  constexpr int W = ORDER;
  constexpr int NV = NDIM + 2;
  constexpr int NT = (NDIM > 1) ? NDIM - 1 : 1;
  constexpr int NC = TN + W - 1;
  constexpr int NCT = TT * NC;
  constexpr int NTH = TT * TN;
  constexpr int AX_A = (DIR == 0) ? 1 : 0;
  constexpr int AX_B = (DIR == 2) ? 1 : 2;
  using Fr = Frame<NDIM, DIR>;

  // forward per-cell records (as in the forward sweep)
  __shared__ double2 sWF[NV][NCT];
  __shared__ double sUn[NCT], sC[NCT], sSr[NCT], sH[NCT];
  __shared__ double sUt[NT][NCT];
  // adjoint accumulators per tile cell: conserved state, physical flux,
  // velocity (local slots: 0 normal, 1.. tangential), sound speed, enthalpy, sqrt(rho)
  __shared__ double aW[NV][NCT], aF[NV][NCT], aU[NDIM][NCT], aC[NCT], aH[NCT], aS[NCT];

  const int64_t nN = A.n[DIR];
  const int64_t nA = A.n[AX_A];
  const int64_t stride[3] = {1, A.n[0], A.n[0] * A.n[1]};
  const int64_t ncell = A.n[0] * A.n[1] * A.n[2];
  const int64_t f0 = (int64_t)blockIdx.x * TN;
  const int64_t t0 = (int64_t)blockIdx.y * TT;
  const int64_t bcoord = blockIdx.z;
  const double gam = A.gamma;
  const double gm1 = gam - 1.0;

  // ghost mapping of tile cell ct: source cell along the normal and wall kind
  auto map_cell = [&](int ct, int64_t& t, int64_t& l, int& mirror_bc) {
    int tt, nn;
    if (DIR == 0) {
      tt = ct / NC;
      nn = ct % NC;
    } else {
      tt = ct % TT;
      nn = ct / TT;
    }
    t = t0 + tt;
    l = f0 - G + nn;
    mirror_bc = -1;
    if (l < 0 || l >= nN) {
      const int bc = (l < 0) ? A.bc_lo : A.bc_hi;
      if (bc == TENOAA_BC_PERIODIC) {
        l = ((l % nN) + nN) % nN;
      } else if (bc == TENOAA_BC_OUTFLOW) {
        l = (l < 0) ? 0 : nN - 1;
      } else {
        l = (l < 0) ? -l - 1 : 2 * nN - 1 - l;
        mirror_bc = bc;
      }
      if (l < 0) l = 0;
      if (l >= nN) l = nN - 1;
    }
  };

  for (int ct = threadIdx.x; ct < NCT; ct += NTH) {
    int64_t t, l;
    int mbc;
    map_cell(ct, t, l, mbc);
    if (t >= nA) t = nA - 1;
    const int64_t off = l * stride[DIR] + t * stride[AX_A] + bcoord * stride[AX_B];
    double Wc[NV];
    unroll<NV>([&](auto c) { Wc[c] = A.U[c * ncell + off]; });
    if (mbc == TENOAA_BC_SYMMETRY) Wc[1 + DIR] = -Wc[1 + DIR];
    if (mbc == TENOAA_BC_NOSLIP) unroll<NDIM>([&](auto k) { Wc[1 + k] = -Wc[1 + k]; });
    const double rho = Wc[0];
    double u[NDIM];
    double q2 = 0.0;
    unroll<NDIM>([&](auto k) {
      u[k] = Wc[1 + k] / rho;
      q2 = (k == 0) ? u[0] * u[0] : q2 + u[k] * u[k];
    });
    const double E = Wc[NV - 1];
    const double p = gm1 * (E - (0.5 * rho) * q2);
    const double un = u[DIR];
    sWF[0][ct] = make_double2(rho, Wc[1 + DIR]);
    unroll<NDIM>([&](auto k) {
      constexpr int slot = Fr::slot_of_axis(decltype(k)::value);
      sWF[1 + slot][ct] = make_double2(Wc[1 + k], (k == DIR) ? Wc[1 + k] * un + p : Wc[1 + k] * un);
      if constexpr (slot > 0) sUt[slot - 1][ct] = u[k];
    });
    sWF[NV - 1][ct] = make_double2(E, (E + p) * un);
    sUn[ct] = un;
    sC[ct] = sqrt((gam * p) / rho);
    sSr[ct] = sqrt(rho);
    sH[ct] = (E + p) / rho;
    unroll<NV>([&](auto c) {
      aW[c][ct] = 0.0;
      aF[c][ct] = 0.0;
    });
    unroll<NDIM>([&](auto k) { aU[k][ct] = 0.0; });
    aC[ct] = 0.0;
    aH[ct] = 0.0;
    aS[ct] = 0.0;
  }
  __syncthreads();

  int tt, fn;
  if (DIR == 0) {
    tt = threadIdx.x / TN;
    fn = threadIdx.x % TN;
  } else {
    tt = threadIdx.x % TT;
    fn = threadIdx.x / TT;
  }
  const int64_t f = f0 + fn;
  const int64_t t = t0 + tt;
  const bool active = (f < A.nf) && (t < nA);
  const int lbase = (DIR == 0) ? tt * NC + fn : fn * TT + tt;
  constexpr int LSTEP = (DIR == 0) ? 1 : TT;
  const int ia = lbase + (G - 1) * LSTEP, ib = lbase + G * LSTEP;

  int64_t flin = 0;
  {
    int64_t m[3] = {A.n[0], A.n[1], A.n[2]};
    m[DIR] = A.nf;
    const int64_t fstr[3] = {1, m[0], m[0] * m[1]};
    flin = f * fstr[DIR] + t * fstr[AX_A] + bcoord * fstr[AX_B];
  }
  if (active) {
    // seed of the face flux: dU_i = -(F_{i+1} - F_i)/dx gives
    // Fbar_f = (R_f - R_{f-1}) / dx over the cells that exist
    double Fb[NV];  // local frame
    {
      const bool periodic = A.bc_lo == TENOAA_BC_PERIODIC;
      const int64_t base = t * stride[AX_A] + bcoord * stride[AX_B];
      const bool hasR = f < nN;
      const bool hasL = f >= 1 || periodic;
      const int64_t cR = f;
      const int64_t cL = (f >= 1) ? f - 1 : nN - 1;
      unroll<NV>([&](auto c) {
        double r = hasR ? A.R[c * ncell + base + cR * stride[DIR]] : 0.0;
        double lft = hasL ? A.R[c * ncell + base + cL * stride[DIR]] : 0.0;
        const double v = (r - lft) / A.dx;
        int slot;
        if (c == 0) slot = 0;
        else if (c == NV - 1) slot = NV - 1;
        else slot = 1 + Fr::slot_of_axis(c - 1);
        Fb[slot] = v;
      });
    }

    // ---- forward recompute: Roe average and eigenvectors
    const double sa = sSr[ia], sb = sSr[ib];
    const double den = sa + sb;
    const double un = (sa * sUn[ia] + sb * sUn[ib]) / den;
    double ut[NT];
    unroll<NDIM - 1>([&](auto k) { ut[k] = (sa * sUt[k][ia] + sb * sUt[k][ib]) / den; });
    double q2 = 0.0;
    unroll<NDIM>([&](auto a) {
      constexpr int slot = Fr::slot_of_axis(decltype(a)::value);
      double ua;
      if constexpr (slot == 0) ua = un;
      else ua = ut[slot - 1];
      q2 = (a == 0) ? ua * ua : q2 + ua * ua;
    });
    const double Hr = (sa * sH[ia] + sb * sH[ib]) / den;
    const double qq = 0.5 * q2;
    const double c2 = gm1 * (Hr - qq);
    const double cr = sqrt(c2);
    const double b1 = gm1 / c2;
    const double b2 = b1 * qq;
    const double unc = un / cr;
    const double ic = 1.0 / cr;

    // splitting speeds and the cells attaining them
    double am = -1.0, a0 = -1.0, ap = -1.0;
    int jm = 0, j0 = 0, jp = 0;
    unroll<W>([&](auto j) {
      const int li = lbase + j * LSTEP;
      const double u = sUn[li], c = sC[li];
      if (A.splitting == TENOAA_LLF) {
        const double lm = fabs(u - c), l0 = fabs(u), lp = fabs(u + c);
        if (lm > am) { am = lm; jm = j; }
        if (l0 > a0) { a0 = l0; j0 = j; }
        if (lp > ap) { ap = lp; jp = j; }
      } else {
        const double lr = fabs(u) + c;
        if (lr > a0) { a0 = lr; j0 = j; }
      }
    });
    if (A.splitting != TENOAA_LLF) {
      am = ap = a0;
      jm = jp = j0;
    }

    auto left_row = [&](int s, double (&L)[NV]) {
      unroll<NV>([&](auto c) { L[c] = 0.0; });
      if (s == 0 || s == NV - 1) {
        L[0] = (s == 0) ? 0.5 * (b2 + unc) : 0.5 * (b2 - unc);
        L[1] = (s == 0) ? 0.5 * (-b1 * un - ic) : 0.5 * (-b1 * un + ic);
        unroll<NDIM - 1>([&](auto k) { L[2 + k] = 0.5 * (-b1 * ut[k]); });
        L[NV - 1] = 0.5 * b1;
      } else if (s == 1) {
        L[0] = 1.0 - b2;
        L[1] = b1 * un;
        unroll<NDIM - 1>([&](auto k) { L[2 + k] = b1 * ut[k]; });
        L[NV - 1] = -b1;
      } else {
        if constexpr (NDIM >= 2) {
          const double utk = (NDIM == 3 && s == 3) ? ut[NT - 1] : ut[0];
          L[0] = -utk;
          unroll<NV>([&](auto c) {
            if (c == s) L[c] = 1.0;
          });
        }
      }
    };
    auto right_col = [&](int s, double (&Rc)[NV]) {
      unroll<NV>([&](auto c) { Rc[c] = 0.0; });
      if (s == 0 || s == 1 || s == NV - 1) {
        Rc[0] = 1.0;
        Rc[1] = (s == 0) ? un - cr : (s == 1 ? un : un + cr);
        unroll<NDIM - 1>([&](auto k) { Rc[2 + k] = ut[k]; });
        Rc[NV - 1] = (s == 0) ? Hr - un * cr : (s == 1 ? qq : Hr + un * cr);
      } else {
        if constexpr (NDIM >= 2) {
          unroll<NV>([&](auto c) {
            if (c == s) Rc[c] = 1.0;
          });
          Rc[NV - 1] = (NDIM == 3 && s == 3) ? ut[NT - 1] : ut[0];
        }
      }
    };
    auto project = [&](const double (&L)[NV], int j, double& v, double& g) {
      const int li = lbase + j * LSTEP;
      const double2 w0 = sWF[0][li];
      v = L[0] * w0.x;
      g = L[0] * w0.y;
      unroll<NV - 1>([&](auto cc) {
        const double2 w = sWF[cc + 1][li];
        v = fma(L[cc + 1], w.x, v);
        g = fma(L[cc + 1], w.y, g);
      });
    };

    // ---- reverse pass
    double un_b = 0.0, Hr_b = 0.0, qq_b = 0.0, cr_b = 0.0, b1_b = 0.0, b2_b = 0.0, unc_b = 0.0, ic_b = 0.0;
    double ut_b[NT];
    unroll<NT>([&](auto k) { ut_b[k] = 0.0; });
#pragma unroll 1
    for (int s = 0; s < NV; ++s) {
      const double fh = A.fh[(int64_t)s * A.nft + flin];
      // back-projection F = sum_s R[:, s] fh_s
      double Rc[NV];
      right_col(s, Rc);
      double fh_b = 0.0;
      unroll<NV>([&](auto c) { fh_b = fma(Rc[c], Fb[c], fh_b); });
      // adjoints of the R entries (column s)
      if (s == 0 || s == 1 || s == NV - 1) {
        const double r1 = Fb[1] * fh, re = Fb[NV - 1] * fh;
        unroll<NDIM - 1>([&](auto k) { ut_b[k] += Fb[2 + k] * fh; });
        if (s == 0) {
          un_b += r1 - cr * re;
          cr_b += -r1 - un * re;
          Hr_b += re;
        } else if (s == 1) {
          un_b += r1;
          qq_b += re;
        } else {
          un_b += r1 + cr * re;
          cr_b += r1 + un * re;
          Hr_b += re;
        }
      } else {
        const double re = Fb[NV - 1] * fh;
        if (NDIM == 3 && s == 3) ut_b[NT - 1] += re;
        else ut_b[0] += re;
      }
      // reconstructions with frozen weights
      double wp[W], wm[W];
      recon_weights<ORDER>(A.flags[(int64_t)(2 * s) * A.nft + flin], wp);
      recon_weights<ORDER>(A.flags[(int64_t)(2 * s + 1) * A.nft + flin], wm);
      double L[NV];
      left_row(s, L);
      const double alpha = (s == 0) ? am : (s == NV - 1 ? ap : a0);
      const int jstar = (s == 0) ? jm : (s == NV - 1 ? jp : j0);
      double alpha_b = 0.0;
      double Lb[NV];
      unroll<NV>([&](auto c) { Lb[c] = 0.0; });
      unroll<W>([&](auto j) {
        double v, g;
        project(L, j, v, g);
        const double gpb = wp[j] * fh_b;
        const double gmb = wm[W - 1 - j] * fh_b;
        const double g_b = 0.5 * (gpb + gmb);
        const double v_b = 0.5 * alpha * (gpb - gmb);
        alpha_b += 0.5 * v * (gpb - gmb);
        const int li = lbase + j * LSTEP;
        unroll<NV>([&](auto c) {
          const double2 w = sWF[c][li];
          Lb[c] = fma(v_b, w.x, fma(g_b, w.y, Lb[c]));
          if (L[c] != 0.0) {
            lds_add(&aW[c][li], L[c] * v_b);
            lds_add(&aF[c][li], L[c] * g_b);
          }
        });
        __builtin_amdgcn_sched_barrier(0);
      });
      // splitting speed: frozen argmax cell and sign
      {
        const int li = lbase + jstar * LSTEP;
        const double u = sUn[li], c = sC[li];
        if (A.splitting == TENOAA_LLF) {
          const double lam = (s == 0) ? u - c : (s == NV - 1 ? u + c : u);
          const double sg = lam < 0.0 ? -1.0 : 1.0;
          lds_add(&aU[0][li], sg * alpha_b);
          if (s == 0) lds_add(&aC[li], -sg * alpha_b);
          if (s == NV - 1) lds_add(&aC[li], sg * alpha_b);
        } else {
          const double sg = u < 0.0 ? -1.0 : 1.0;
          lds_add(&aU[0][li], sg * alpha_b);
          lds_add(&aC[li], alpha_b);
        }
      }
      // adjoints of the L entries (row s)
      if (s == 0 || s == NV - 1) {
        const double sgn = (s == 0) ? 1.0 : -1.0;
        b2_b += 0.5 * Lb[0];
        unc_b += 0.5 * sgn * Lb[0];
        b1_b += -0.5 * un * Lb[1];
        un_b += -0.5 * b1 * Lb[1];
        ic_b += -0.5 * sgn * Lb[1];
        unroll<NDIM - 1>([&](auto k) {
          b1_b += -0.5 * ut[k] * Lb[2 + k];
          ut_b[k] += -0.5 * b1 * Lb[2 + k];
        });
        b1_b += 0.5 * Lb[NV - 1];
      } else if (s == 1) {
        b2_b -= Lb[0];
        b1_b += un * Lb[1];
        un_b += b1 * Lb[1];
        unroll<NDIM - 1>([&](auto k) {
          b1_b += ut[k] * Lb[2 + k];
          ut_b[k] += b1 * Lb[2 + k];
        });
        b1_b -= Lb[NV - 1];
      } else {
        if (NDIM == 3 && s == 3) ut_b[NT - 1] -= Lb[0];
        else ut_b[0] -= Lb[0];
      }
    }

    // ---- Roe average and eigen-system parameters
    un_b += unc_b / cr;
    cr_b -= unc_b * unc / cr;
    cr_b -= ic_b * ic * ic;
    b1_b += b2_b * qq;
    qq_b += b2_b * b1;
    double c2_b = -b1_b * b1 / c2;
    c2_b += cr_b / (2.0 * cr);
    Hr_b += gm1 * c2_b;
    qq_b -= gm1 * c2_b;
    // qq = |u~|^2 / 2
    un_b += qq_b * un;
    unroll<NDIM - 1>([&](auto k) { ut_b[k] += qq_b * ut[k]; });
    // u~ = (sa ua + sb ub) / den, H~ likewise
    double sa_b = 0.0, sb_b = 0.0;
    {
      const double wa = sa / den, wb = sb / den;
      lds_add(&aU[0][ia], un_b * wa);
      lds_add(&aU[0][ib], un_b * wb);
      sa_b += un_b * (sUn[ia] - un) / den;
      sb_b += un_b * (sUn[ib] - un) / den;
      unroll<NDIM - 1>([&](auto k) {
        lds_add(&aU[1 + k][ia], ut_b[k] * wa);
        lds_add(&aU[1 + k][ib], ut_b[k] * wb);
        sa_b += ut_b[k] * (sUt[k][ia] - ut[k]) / den;
        sb_b += ut_b[k] * (sUt[k][ib] - ut[k]) / den;
      });
      lds_add(&aH[ia], Hr_b * wa);
      lds_add(&aH[ib], Hr_b * wb);
      sa_b += Hr_b * (sH[ia] - Hr) / den;
      sb_b += Hr_b * (sH[ib] - Hr) / den;
      lds_add(&aS[ia], sa_b);
      lds_add(&aS[ib], sb_b);
    }
  }
  __syncthreads();

  // ---- cell-level reverse pass and scatter to U_bar
  for (int ct = threadIdx.x; ct < NCT; ct += NTH) {
    int64_t tc, l;
    int mbc;
    map_cell(ct, tc, l, mbc);
    if (tc >= nA) continue;
    const double2 w0 = sWF[0][ct];
    const double rho = w0.x;
    const double E = sWF[NV - 1][ct].x;
    double m[NDIM], u[NDIM];  // local slots
    unroll<NDIM>([&](auto k) {
      m[k] = sWF[1 + k][ct].x;
      u[k] = m[k] / rho;
    });
    double q2 = 0.0;
    unroll<NDIM>([&](auto k) { q2 += u[k] * u[k]; });
    const double p = gm1 * (E - (0.5 * rho) * q2);
    const double c = sC[ct], H = sH[ct], sr = sSr[ct];
    double rho_b = aW[0][ct], E_b = aW[NV - 1][ct];
    double m_b[NDIM], u_b[NDIM];
    unroll<NDIM>([&](auto k) {
      m_b[k] = aW[1 + k][ct];
      u_b[k] = aU[k][ct];
    });
    double p_b = 0.0;
    // physical flux (Sec. 1): (m_n, m_n u_n + p, m_t u_n, (E + p) u_n)
    {
      const double F0b = aF[0][ct];
      m_b[0] += F0b;
      const double F1b = aF[1][ct];
      m_b[0] += F1b * u[0];
      u_b[0] += F1b * m[0];
      p_b += F1b;
      unroll<NDIM - 1>([&](auto k) {
        const double Fkb = aF[2 + k][ct];
        m_b[1 + k] += Fkb * u[0];
        u_b[0] += Fkb * m[1 + k];
      });
      const double FEb = aF[NV - 1][ct];
      E_b += FEb * u[0];
      p_b += FEb * u[0];
      u_b[0] += FEb * (E + p);
    }
    rho_b += aS[ct] / (2.0 * sr);
    {
      const double Hb = aH[ct];
      E_b += Hb / rho;
      p_b += Hb / rho;
      rho_b -= Hb * H / rho;
    }
    {
      const double tb = aC[ct] / (2.0 * c);  // c = sqrt(gam p / rho)
      p_b += tb * gam / rho;
      rho_b -= tb * (c * c) / rho;
    }
    E_b += gm1 * p_b;
    rho_b -= gm1 * 0.5 * q2 * p_b;
    const double q2_b = -gm1 * 0.5 * rho * p_b;
    unroll<NDIM>([&](auto k) {
      u_b[k] += 2.0 * u[k] * q2_b;
      m_b[k] += u_b[k] / rho;
      rho_b -= u_b[k] * u[k] / rho;
    });
    // back to axis order, undo the wall sign flips, add to the source cell
    double Ub[NV];
    Ub[0] = rho_b;
    Ub[NV - 1] = E_b;
    unroll<NDIM>([&](auto a) { Ub[1 + a] = m_b[Fr::slot_of_axis(decltype(a)::value)]; });
    if (mbc == TENOAA_BC_SYMMETRY) Ub[1 + DIR] = -Ub[1 + DIR];
    if (mbc == TENOAA_BC_NOSLIP) unroll<NDIM>([&](auto k) { Ub[1 + k] = -Ub[1 + k]; });
    const int64_t off = l * stride[DIR] + tc * stride[AX_A] + bcoord * stride[AX_B];
    unroll<NV>([&](auto cc) { unsafeAtomicAdd(&A.Ubar[cc * ncell + off], Ub[cc]); });
  }
}

__global__ void zero_kernel(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// out = a*x + b*y + c*z (element-wise; null operands skipped) for the RK3 chain.
__global__ void axpbypcz_kernel(double* out, double a, const double* x, double b, const double* y, double c,
                                const double* z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * x[i];
    if (y) v = v + b * y[i];
    if (z) v = v + c * z[i];
    out[i] = v;
  }
}

// out = a*x + (c * dt) * z with dt read on the device.
__global__ void axpdtz_kernel(double* out, double a, const double* x, double c, const double* dt, const double* z,
                              int64_t n) {
  const double cd = c * (*dt);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a * x[i] + cd * z[i];
}

}  // namespace

template <int ORDER, int NDIM, int DIR>
static hipError_t launch_vjp_t(const AdjointArgs& a, hipStream_t st) {
  constexpr int TT = (NDIM == 1) ? 1 : (DIR == 0 ? TENOAA_ADJ_TT_X : TENOAA_ADJ_TT_YZ);
  constexpr int TN = (DIR == 0) ? TENOAA_ADJ_TN_X : TENOAA_ADJ_TN_YZ;
  constexpr int AX_A = (DIR == 0) ? 1 : 0;
  constexpr int AX_B = (DIR == 2) ? 1 : 2;
  dim3 grid((unsigned)((a.nf + TN - 1) / TN), (unsigned)((a.n[AX_A] + TT - 1) / TT), (unsigned)a.n[AX_B]);
  hipLaunchKernelGGL((sweep_vjp_kernel<ORDER, NDIM, DIR, TT, TN>), grid, dim3(TT * TN), 0, st, a);
  return hipGetLastError();
}

template <int ORDER>
static hipError_t launch_vjp_ord(int ndim, int dir, const AdjointArgs& a, hipStream_t st) {
  if (ndim == 1) return launch_vjp_t<ORDER, 1, 0>(a, st);
  if (ndim == 2) return dir == 0 ? launch_vjp_t<ORDER, 2, 0>(a, st) : launch_vjp_t<ORDER, 2, 1>(a, st);
  if (dir == 0) return launch_vjp_t<ORDER, 3, 0>(a, st);
  if (dir == 1) return launch_vjp_t<ORDER, 3, 1>(a, st);
  return launch_vjp_t<ORDER, 3, 2>(a, st);
}

hipError_t launch_sweep_vjp(int order, int ndim, int dir, const AdjointArgs& a, hipStream_t st) {
  return order == 10 ? launch_vjp_ord<10>(ndim, dir, a, st) : launch_vjp_ord<8>(ndim, dir, a, st);
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_axpbypcz(double* out, double a, const double* x, double b, const double* y, double c,
                           const double* z, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpbypcz_kernel, dim3(grid_for(n)), dim3(256), 0, st, out, a, x, b, y, c, z, n);
  return hipGetLastError();
}

hipError_t launch_axpdtz(double* out, double a, const double* x, double c, const double* dt, const double* z,
                         int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpdtz_kernel, dim3(grid_for(n)), dim3(256), 0, st, out, a, x, c, dt, z, n);
  return hipGetLastError();
}

}  // namespace tenoaa
