// Adjoint (vector-Jacobian product) of the TENO-AA Euler right-hand side.
//
// For a state U and a seed R = dL/d(dU/dt), one sweep kernel per direction
// accumulates U_bar += (d(dU/dt)_d / dU)^T R with every threshold decision of
// the method frozen at U: the stencil chosen by the cascade and the cut-off
// deltas (Sec. 3.3 of the paper), hence the linear weights of each
// reconstruction; the cell that attains each LLF/Rusanov splitting speed and
// the sign of that speed; with the Roe flux, which side each field
// reconstructs.  Everything else - cell primitives, Roe average,
// eigenvectors, projection, split, back-projection - is differentiated
// exactly.  With the positivity limiter, its factor theta per face (recorded
// by the forward sweep) is frozen as well, and the Lax-Friedrichs flux it
// blends in is differentiated with its speed's cell frozen.
//
// The forward sweep of the same direction runs first and leaves, per face,
// the decision bytes and the per-field fluxes fh_s.  Per block: the tile of
// cells is staged with the forward sweep's arithmetic; each thread takes one
// face, recomputes the Roe average, eigenvectors, projections and splitting
// speeds, then runs the reverse pass and scatters the adjoints of the window
// cells' conserved states, physical fluxes and primitive quantities into LDS
// accumulators (ds_add_f64).  After a barrier the cell-level reverse pass
// turns those into conserved-state adjoints, maps ghost cells back to their
// interior source (with the momentum sign flips of wall conditions) and adds
// them to U_bar (a Dirichlet ghost through the Jacobian of its reflection
// rule; an inflow ghost is a constant; a halo cell, a neighbour piece's, goes
// to the caller's halo-adjoint buffer).
//
// Every sum is taken in a fixed order, so U_bar is the same bit for bit from
// run to run: a wave holds whole pencils of its tile (the LDS records are
// pencil-major in every direction), so each LDS accumulator is added to by
// one wave only, in program order; a ghost position whose source is a domain
// cell of the same tile is summed into that cell's adjoint in window order
// before one add to U_bar; and the tiles of a direction run in launches of
// alternating tiles (the periodic wrap's neighbours apart), so that no two
// tiles of one launch add to the same cell.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa_device.h"
#include "tenoaa_internal.h"
#include "tenoaa_stencil.h"

#ifndef TENOAA_ADJ_TN_X
#define TENOAA_ADJ_TN_X 64
#endif
#ifndef TENOAA_ADJ_TT_X
#define TENOAA_ADJ_TT_X 2
#endif
#ifndef TENOAA_ADJ_TN_YZ
#define TENOAA_ADJ_TN_YZ 64
#endif
#ifndef TENOAA_ADJ_TT_YZ
#define TENOAA_ADJ_TT_YZ 2
#endif
#ifndef TENOAA_ADJ_WAVES_PER_EU
#define TENOAA_ADJ_WAVES_PER_EU 0
#endif

namespace tenoaa {
namespace {

// Derivatives of the frozen reconstructions with respect to the window values
// f_{-G+1..G}: one row per outcome of the cascade.  Rows 0-7: the TENO5
// fallback with delta mask 0-7 (weights d_k delta_k / sum, Sec. 3.3, times the
// three third-order candidates); rows 8, 9, 10, 11: the linear schemes on S3,
// S4, S5 (Sec. 4.1) and S6 (TENO12-AA), stencil S_p starting at v[G - p].
// Row 0 (no small stencil kept) is all zeros: the byte of a side the Roe flux
// does not reconstruct selects it.
constexpr int NROW = 12;
template <int ORDER>
__device__ __forceinline__ double weight_entry(int row, int q) {
  constexpr int G = ORDER / 2;
  constexpr int I = G - 1;
  if (row >= 8) {
    const int p = row - 5;
    const int P = G - p;
    if (p > G || q < P || q >= P + 2 * p) return 0.0;
    return p == 3 ? lin_coef<6>(q - P) : (p == 4 ? lin_coef<8>(q - P) : (p == 5 ? lin_coef<10>(q - P) : lin_coef<12>(q - P)));
  }
  const double w0 = WFALL.w[row][0], w1 = WFALL.w[row][1], w2 = WFALL.w[row][2];
  constexpr double s6 = 1.0 / 6.0;
  if (q == I - 2) return w2 * (2.0 * s6);
  if (q == I - 1) return w0 * (-s6) + w2 * (-7.0 * s6);
  if (q == I) return w0 * (5.0 * s6) + w1 * (2.0 * s6) + w2 * (11.0 * s6);
  if (q == I + 1) return w0 * (2.0 * s6) + w1 * (5.0 * s6);
  if (q == I + 2) return w1 * (-s6);
  return 0.0;
}

// Row of the weight table selected by a decision byte (S6 of TENO12-AA:
// selector 3 with bit 2 set).
template <int ORDER>
__device__ __forceinline__ int weight_row(uint8_t flag) {
  const int sel = flag & 3;
  int large = 7 + sel;
  if constexpr (ORDER == 12) large += (sel == 3) & ((flag >> 2) & 1);
  return sel == 0 ? (flag >> 2) & 7 : large;
}

__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }

// Materialises x in a register here: keeps the compiler from sinking the
// accumulations of a window cell past the next cell (which would keep every
// cell's operands alive until the end of the window).
__device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }

template <int ORDER, int NDIM, int DIR, int TT, int TN, bool GENERAL>
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
  // a wave holds whole pencils (the fixed order of the LDS sums)
  static_assert(TN <= 64 && 64 % TN == 0 && (TT * TN) % 64 == 0, "tile must give each wave whole pencils");

  // forward per-cell records (as in the forward sweep), pencil-major: cell nn
  // of pencil tt at tt * NC + nn
  __shared__ double2 sWF[NV][NCT];
  __shared__ double sUn[NCT], sC[NCT], sSr[NCT], sH[NCT];
  __shared__ double sUt[NT][NCT];
  // adjoint accumulators per tile cell: conserved state, physical flux,
  // velocity (local slots: 0 normal, 1.. tangential), sound speed, enthalpy, sqrt(rho)
  __shared__ double aW[NV][NCT], aF[NV][NCT], aU[NDIM][NCT], aC[NCT], aH[NCT], aS[NCT];
  // derivative weights of the frozen reconstructions, [row][window position]
  __shared__ double sWT[NROW * W];
  for (int e = threadIdx.x; e < NROW * W; e += NTH) sWT[e] = weight_entry<ORDER>(e / W, e % W);

  const int64_t nN = A.n[DIR];
  const int64_t nA = A.n[AX_A];
  const int64_t stride[3] = {1, A.n[0], A.n[0] * A.n[1]};
  const int64_t ncell = A.n[0] * A.n[1] * A.n[2];
  const int64_t f0 = A.f_begin + (A.tile_first + (int64_t)blockIdx.x * A.tile_step) * TN;
  const int64_t t0 = (int64_t)blockIdx.y * TT;
  const int64_t bcoord = blockIdx.z;
  const double gam = A.gamma;
  const double gm1 = gam - 1.0;

  // pencil and position of the ct-th cell a thread stages: along the pencil
  // in x, across the pencils (consecutive in memory) in y and z
  auto cell_of = [&](int ct, int& tt, int& nn) {
    if (DIR == 0) {
      tt = ct / NC;
      nn = ct % NC;
    } else {
      tt = ct % TT;
      nn = ct / TT;
    }
  };
  // ghost mapping of the tile cell at (tt, nn), as in the forward sweep: the
  // source cell along the normal, the boundary kind that makes it a ghost (-1
  // for a domain cell, a periodic or outflow copy, or a cell beyond the G
  // ghost layers that no face reads), the side and the ghost layer 1..G
  auto map_cell = [&](int tt, int nn, int64_t& t, int64_t& l, int& gbc, int& side, int64_t& layer) {
    t = t0 + tt;
    l = f0 - G + nn;
    gbc = -1;
    side = (l < 0) ? 0 : 1;
    layer = (l < 0) ? -l : l - nN + 1;
    if (l < 0 || l >= nN) {
      const int bc = (l < 0) ? A.bc_lo : A.bc_hi;
      if (bc == TENOAA_BC_PERIODIC) {
        l = ((l % nN) + nN) % nN;
      } else if (bc == TENOAA_BC_OUTFLOW || layer > G) {
        l = (l < 0) ? 0 : nN - 1;
      } else {
        l = (l < 0) ? -l - 1 : 2 * nN - 1 - l;
        gbc = bc;
      }
      if (l < 0) l = 0;
      if (l >= nN) l = nN - 1;
    }
  };
  // boundary values of pencil t's cell of the face plane on side `side`
  const int64_t plane = nA * A.n[AX_B];
  auto face_vals = [&](int side, int64_t t) { return A.bcv[side] + t + nA * bcoord; };

  for (int cs = threadIdx.x; cs < NCT; cs += NTH) {
    int tt0, nn0;
    cell_of(cs, tt0, nn0);
    const int ct = tt0 * NC + nn0;
    int64_t t, l, layer;
    int gbc, side;
    map_cell(tt0, nn0, t, l, gbc, side, layer);
    if (t >= nA) t = nA - 1;
    const int64_t off = l * stride[DIR] + t * stride[AX_A] + bcoord * stride[AX_B];
    double Wc[NV];
    unroll<NV>([&](auto c) { Wc[c] = A.U[c * ncell + off]; });
    if (gbc == TENOAA_BC_SYMMETRY) {
      Wc[1 + DIR] = -Wc[1 + DIR];
    } else if (gbc == TENOAA_BC_NOSLIP) {
      unroll<NDIM>([&](auto k) { Wc[1 + k] = -Wc[1 + k]; });
    } else if constexpr (GENERAL) {
      if (gbc == TENOAA_BC_DIRICHLET) {
        dirichlet_ghost<NDIM>(Wc, face_vals(side, t), plane, gm1);
      } else if (gbc == TENOAA_BC_INFLOW) {
        inflow_ghost<NDIM>(Wc, face_vals(side, t) + (layer - 1) * NV * plane, plane, gm1);
      } else if (gbc == TENOAA_BC_HALO) {
        const double* hv = face_vals(side, t) + (layer - 1) * NV * plane;
        unroll<NV>([&](auto c) { Wc[c] = hv[c * plane]; });
      }
    }
    // the same arithmetic as the forward sweep, so that the frozen splitting
    // speeds are attained by the same cells
    const double rho = Wc[0];
    const double ir = div_rn(1.0, rho);
    double u[NDIM];
    double q2 = 0.0;
    unroll<NDIM>([&](auto k) {
      u[k] = Wc[1 + k] * ir;
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
    sC[ct] = sqrt_rn((gam * p) * ir);
    sSr[ct] = sqrt_rn(rho);
    sH[ct] = (E + p) * ir;
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

  const int tt = threadIdx.x / TN;
  const int fn = threadIdx.x % TN;
  const int64_t f = f0 + fn;
  const int64_t t = t0 + tt;
  const bool active = (f < A.nf) && (t < nA);
  const int lbase = tt * NC + fn;
  constexpr int LSTEP = 1;
  const int ia = lbase + (G - 1) * LSTEP, ib = lbase + G * LSTEP;

  // the face's recorded decisions, fluxes and limiter factor, laid out
  // pencil by pencil by the forward sweep (a wave reads consecutive faces)
  const int64_t frec = f + A.nf * (t + nA * bcoord);
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

    // positivity limiter with its factor frozen: F = F_LF + theta (F_H - F_LF),
    // F_LF = (F_a + F_b - a_L (W_b - W_a)) / 2 with a_L = max(|u_n| + c) of the
    // two cells (that cell frozen); F_H continues below with seed theta Fbar
    if (A.theta) {
      const double th = A.theta[frec];
      if (th < 1.0) {
        const double sA = fabs(sUn[ia]) + sC[ia], sB = fabs(sUn[ib]) + sC[ib];
        const bool onA = sA >= sB;
        const double aL = onA ? sA : sB;
        double aLb = 0.0;
        unroll<NV>([&](auto c) {
          const double flb = (1.0 - th) * Fb[c];
          const double2 wa = sWF[c][ia], wb = sWF[c][ib];
          lds_add(&aF[c][ia], 0.5 * flb);
          lds_add(&aF[c][ib], 0.5 * flb);
          lds_add(&aW[c][ia], (0.5 * aL) * flb);
          lds_add(&aW[c][ib], -(0.5 * aL) * flb);
          aLb -= 0.5 * flb * (wb.x - wa.x);
          Fb[c] *= th;
        });
        const int li = onA ? ia : ib;
        lds_add(&aU[0][li], (sUn[li] < 0.0 ? -1.0 : 1.0) * aLb);
        lds_add(&aC[li], aLb);
      }
    }

    // ---- forward recompute: Roe average and eigenvectors
    const double sa = sSr[ia], sb = sSr[ib];
    const double den = sa + sb;
    const double iden = div_rn(1.0, den);
    const double un = (sa * sUn[ia] + sb * sUn[ib]) * iden;
    double ut[NT];
    unroll<NDIM - 1>([&](auto k) { ut[k] = (sa * sUt[k][ia] + sb * sUt[k][ib]) * iden; });
    double q2 = 0.0;
    unroll<NDIM>([&](auto a) {
      constexpr int slot = Fr::slot_of_axis(decltype(a)::value);
      double ua;
      if constexpr (slot == 0) ua = un;
      else ua = ut[slot - 1];
      q2 = (a == 0) ? ua * ua : q2 + ua * ua;
    });
    const double Hr = (sa * sH[ia] + sb * sH[ib]) * iden;
    const double qq = 0.5 * q2;
    const double c2 = gm1 * (Hr - qq);
    const double cr = sqrt_rn(c2);
    const double b1 = div_rn(gm1, c2);
    const double b2 = b1 * qq;
    const double ic = div_rn(1.0, cr);
    const double unc = un * ic;

    // splitting speeds and the cells attaining them
    double am = -1.0, a0 = -1.0, ap = -1.0;
    int jm = 0, j0 = 0, jp = 0;
    unroll<W>([&](auto j) {
      const int li = lbase + j * LSTEP;
      const double u = sUn[li], c = sC[li];
      if (A.splitting != TENOAA_RUSANOV) {  // LLF, also the Roe flux's fallback
        const double lm = fabs(u - c), l0 = fabs(u), lp = fabs(u + c);
        if (lm > am) { am = lm; jm = j; }
        if (l0 > a0) { a0 = l0; j0 = j; }
        if (lp > ap) { ap = lp; jp = j; }
      } else {
        const double lr = fabs(u) + c;
        if (lr > a0) { a0 = lr; j0 = j; }
      }
    });
    if (A.splitting == TENOAA_RUSANOV) {
      am = ap = a0;
      jm = jp = j0;
    }

    // ---- reverse pass
    double un_b = 0.0, Hr_b = 0.0, qq_b = 0.0, cr_b = 0.0, b1_b = 0.0, b2_b = 0.0, unc_b = 0.0, ic_b = 0.0;
    double ut_b[NT];
    unroll<NT>([&](auto k) { ut_b[k] = 0.0; });

    // back-projection F = sum_s R[:, s] fh_s: adjoints of fh_s and of R's entries
    double fhb[NV];
    unroll<NV>([&](auto ss) {
      constexpr int s = decltype(ss)::value;
      constexpr bool shear = (s >= 2 && s <= NV - 2);
      const double fh = A.fh[(int64_t)s * A.nft + frec];
      if constexpr (!shear) {
        const double r1 = (s == 0) ? un - cr : (s == 1 ? un : un + cr);
        const double re = (s == 0) ? Hr - un * cr : (s == 1 ? qq : Hr + un * cr);
        double acc = Fb[0];
        acc = fma(r1, Fb[1], acc);
        unroll<NDIM - 1>([&](auto k) { acc = fma(ut[k], Fb[2 + k], acc); });
        fhb[s] = fma(re, Fb[NV - 1], acc);
        const double r1b = Fb[1] * fh, reb = Fb[NV - 1] * fh;
        unroll<NDIM - 1>([&](auto k) { ut_b[k] += Fb[2 + k] * fh; });
        if constexpr (s == 0) {
          un_b += r1b - cr * reb;
          cr_b += -r1b - un * reb;
          Hr_b += reb;
        } else if constexpr (s == 1) {
          un_b += r1b;
          qq_b += reb;
        } else {
          un_b += r1b + cr * reb;
          cr_b += r1b + un * reb;
          Hr_b += reb;
        }
      } else {
        fhb[s] = fma(ut[s - 2], Fb[NV - 1], Fb[s]);
        ut_b[s - 2] += Fb[NV - 1] * fh;
      }
    });

    // left eigenvector rows: full rows for the acoustic and entropy fields
    // (local slots 0, 1, NV-1 -> rows 0, 1, 2 here), -u_t + e_s for the shear fields
    double L[3][NV];
    unroll<2>([&](auto side) {
      constexpr int r = side == 0 ? 0 : 2;
      const double sg = side == 0 ? 1.0 : -1.0;
      L[r][0] = 0.5 * (b2 + sg * unc);
      L[r][1] = 0.5 * (-b1 * un - sg * ic);
      unroll<NDIM - 1>([&](auto k) { L[r][2 + k] = 0.5 * (-b1 * ut[k]); });
      L[r][NV - 1] = 0.5 * b1;
    });
    L[1][0] = 1.0 - b2;
    L[1][1] = b1 * un;
    unroll<NDIM - 1>([&](auto k) { L[1][2 + k] = b1 * ut[k]; });
    L[1][NV - 1] = -b1;
    // frozen reconstructions: row of the weight table per field and side.
    // The Roe flux reconstructs the unsplit characteristic flux g from one
    // side only where the field's eigenvalue keeps one sign at the face; the
    // other side's byte is then 0 (no real decision has it)
    int rowp[NV], rowm[NV];
    bool one_side[NV];
    unroll<NV>([&](auto ss) {
      constexpr int s = decltype(ss)::value;
      const uint8_t bp = A.flags[(int64_t)(2 * s) * A.nft + frec];
      const uint8_t bm = A.flags[(int64_t)(2 * s + 1) * A.nft + frec];
      rowp[s] = weight_row<ORDER>(bp);
      rowm[s] = weight_row<ORDER>(bm);
      one_side[s] = GENERAL && A.splitting == TENOAA_ROE && (bp == 0 || bm == 0);
    });
    double Lb[3][NV], Lbs[NT];
    unroll<3>([&](auto r) { unroll<NV>([&](auto c) { Lb[r][c] = 0.0; }); });
    unroll<NT>([&](auto k) { Lbs[k] = 0.0; });
    double am_b = 0.0, a0_b = 0.0, ap_b = 0.0;

    unroll<W>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const int li = lbase + j * LSTEP;
      double2 w[NV];
      unroll<NV>([&](auto c) { w[c] = sWF[c][li]; });
      double vb[NV], gb[NV];
      unroll<NV>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        constexpr bool shear = (s >= 2 && s <= NV - 2);
        constexpr int r = (s == 0) ? 0 : (s == 1 ? 1 : 2);
        double v, g;
        if constexpr (!shear) {
          v = L[r][0] * w[0].x;
          g = L[r][0] * w[0].y;
          unroll<NV - 1>([&](auto cc) {
            v = fma(L[r][cc + 1], w[cc + 1].x, v);
            g = fma(L[r][cc + 1], w[cc + 1].y, g);
          });
        } else {
          v = fma(-ut[s - 2], w[0].x, w[s].x);
          g = fma(-ut[s - 2], w[0].y, w[s].y);
        }
        const double cp = sWT[rowp[s] * W + j] * fhb[s];
        const double cm = sWT[rowm[s] * W + (W - 1 - j)] * fhb[s];
        const double alpha = (s == 0) ? am : (s == NV - 1 ? ap : a0);
        const double d = cp - cm;
        // split: f+- = (g +- alpha v) / 2; one-sided Roe: f = g (the unused side's row is zero)
        vb[s] = one_side[s] ? 0.0 : (0.5 * alpha) * d;
        gb[s] = one_side[s] ? cp + cm : 0.5 * (cp + cm);
        const double ab = one_side[s] ? 0.0 : (0.5 * v) * d;
        if constexpr (s == 0) am_b += ab;
        else if constexpr (s == NV - 1) ap_b += ab;
        else a0_b += ab;
        if constexpr (!shear) {
          unroll<NV>([&](auto c) { Lb[r][c] = fma(vb[s], w[c].x, fma(gb[s], w[c].y, Lb[r][c])); });
        } else {
          Lbs[s - 2] = fma(vb[s], w[0].x, fma(gb[s], w[0].y, Lbs[s - 2]));
        }
      });
      // adjoints of this cell's conserved state and flux: L^T (vb, gb)
      unroll<NV>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        double sw = L[0][c] * vb[0] + L[1][c] * vb[1] + L[2][c] * vb[NV - 1];
        double sf = L[0][c] * gb[0] + L[1][c] * gb[1] + L[2][c] * gb[NV - 1];
        if constexpr (c == 0) {
          unroll<NT>([&](auto k) {
            if constexpr (NDIM > 1) {
              sw = fma(-ut[k], vb[2 + k], sw);
              sf = fma(-ut[k], gb[2 + k], sf);
            }
          });
        } else if constexpr (c >= 2 && c <= NV - 2) {
          sw += vb[c];
          sf += gb[c];
        }
        lds_add(&aW[c][li], sw);
        lds_add(&aF[c][li], sf);
      });
      unroll<3>([&](auto r) { unroll<NV>([&](auto c) { pin(Lb[r][c]); }); });
      unroll<NT>([&](auto k) { pin(Lbs[k]); });
      pin(am_b);
      pin(a0_b);
      pin(ap_b);
      __builtin_amdgcn_sched_barrier(0);
    });

    // splitting speeds: frozen argmax cells and signs
    if (A.splitting != TENOAA_RUSANOV) {
      {
        const int li = lbase + jm * LSTEP;
        const double sg = (sUn[li] - sC[li]) < 0.0 ? -1.0 : 1.0;
        lds_add(&aU[0][li], sg * am_b);
        lds_add(&aC[li], -sg * am_b);
      }
      {
        const int li = lbase + j0 * LSTEP;
        const double sg = sUn[li] < 0.0 ? -1.0 : 1.0;
        lds_add(&aU[0][li], sg * a0_b);
      }
      {
        const int li = lbase + jp * LSTEP;
        const double sg = (sUn[li] + sC[li]) < 0.0 ? -1.0 : 1.0;
        lds_add(&aU[0][li], sg * ap_b);
        lds_add(&aC[li], sg * ap_b);
      }
    } else {
      const int li = lbase + j0 * LSTEP;
      const double sg = sUn[li] < 0.0 ? -1.0 : 1.0;
      const double tot = (am_b + a0_b) + ap_b;
      lds_add(&aU[0][li], sg * tot);
      lds_add(&aC[li], tot);
    }

    // adjoints of the L entries
    unroll<2>([&](auto side) {
      constexpr int r = side == 0 ? 0 : 2;
      const double sgn = side == 0 ? 1.0 : -1.0;
      b2_b += 0.5 * Lb[r][0];
      unc_b += 0.5 * sgn * Lb[r][0];
      b1_b += -0.5 * un * Lb[r][1];
      un_b += -0.5 * b1 * Lb[r][1];
      ic_b += -0.5 * sgn * Lb[r][1];
      unroll<NDIM - 1>([&](auto k) {
        b1_b += -0.5 * ut[k] * Lb[r][2 + k];
        ut_b[k] += -0.5 * b1 * Lb[r][2 + k];
      });
      b1_b += 0.5 * Lb[r][NV - 1];
    });
    b2_b -= Lb[1][0];
    b1_b += un * Lb[1][1];
    un_b += b1 * Lb[1][1];
    unroll<NDIM - 1>([&](auto k) {
      b1_b += ut[k] * Lb[1][2 + k];
      ut_b[k] += b1 * Lb[1][2 + k];
    });
    b1_b -= Lb[1][NV - 1];
    unroll<NDIM - 1>([&](auto k) { ut_b[k] -= Lbs[k]; });

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

  // ---- cell-level reverse pass: the conserved-state adjoint Ub of the tile
  // cell at (ttc, nn) with respect to the state it is read from (the source
  // cell, a wall ghost's sign flips undone, a Dirichlet ghost's mirror cell
  // through its rule, or a halo cell); false if it adds nothing (a pencil
  // beyond the grid, an inflow ghost, which does not depend on U, a halo side
  // without its buffer, or a position beyond the G ghost layers, which no
  // face reads)
  auto cell_adjoint = [&](int ttc, int nn, double (&Ub)[NV]) -> bool {
    const int ct = ttc * NC + nn;
    int64_t tc, l, layer;
    int gbc, side;
    map_cell(ttc, nn, tc, l, gbc, side, layer);
    const int64_t lraw = f0 - G + nn;
    if (tc >= nA || ((lraw < 0 || lraw >= nN) && layer > G)) return false;
    if (GENERAL && gbc == TENOAA_BC_INFLOW) return false;
    if (GENERAL && gbc == TENOAA_BC_HALO && !A.hbar[side]) return false;
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
    // back to axis order, undo the wall sign flips
    Ub[0] = rho_b;
    Ub[NV - 1] = E_b;
    unroll<NDIM>([&](auto a) { Ub[1 + a] = m_b[Fr::slot_of_axis(decltype(a)::value)]; });
    if (gbc == TENOAA_BC_SYMMETRY) Ub[1 + DIR] = -Ub[1 + DIR];
    if (gbc == TENOAA_BC_NOSLIP) unroll<NDIM>([&](auto k) { Ub[1 + k] = -Ub[1 + k]; });
    const int64_t off = l * stride[DIR] + tc * stride[AX_A] + bcoord * stride[AX_B];
    if (GENERAL && gbc == TENOAA_BC_DIRICHLET) {
      // through the ghost rule (rho, u, p)_g = 2 (rho, u, p)_face - (rho, u, p)_m
      // back to the mirror cell m: ghost conserved -> ghost primitives, the
      // reflection (-1), mirror primitives -> mirror conserved
      double Wm[NV];
      unroll<NV>([&](auto cc) { Wm[cc] = A.U[cc * ncell + off]; });
      const double* fv = face_vals(side, tc);
      const double rm = Wm[0];
      double um[NDIM], q2m = 0.0;
      unroll<NDIM>([&](auto k) {
        um[k] = Wm[1 + k] / rm;
        q2m += um[k] * um[k];
      });
      const double rg = 2.0 * fv[0] - rm;
      double ug[NDIM], qg = 0.0;
      unroll<NDIM>([&](auto k) {
        ug[k] = 2.0 * fv[(1 + k) * plane] - um[k];
        qg += ug[k] * ug[k];
      });
      double rg_b = Ub[0] + Ub[NV - 1] * (0.5 * qg);
      unroll<NDIM>([&](auto k) { rg_b += Ub[1 + k] * ug[k]; });
      const double pm_b = -Ub[NV - 1] / gm1;
      double Um[NV];
      Um[NV - 1] = gm1 * pm_b;
      Um[0] = -rg_b + gm1 * 0.5 * q2m * pm_b;
      unroll<NDIM>([&](auto k) {
        const double um_b = -(Ub[1 + k] * rg + Ub[NV - 1] * rg * ug[k]);
        Um[1 + k] = um_b / rm - gm1 * um[k] * pm_b;
        Um[0] -= um_b * um[k] / rm;
      });
      unroll<NV>([&](auto cc) { Ub[cc] = Um[cc]; });
    }
    return true;
  };
  // adds Ub to where the tile cell at (ttc, nn) is read from: U_bar, or for a
  // halo cell (a neighbour piece's) the caller's halo-adjoint buffer.  The
  // adds are atomic (performed at L2, where the tiles of later launches read
  // them); their order is fixed as described at the top of this file.
  auto add_to_source = [&](int ttc, int nn, const double (&Ub)[NV]) {
    int64_t tc, l, layer;
    int gbc, side;
    map_cell(ttc, nn, tc, l, gbc, side, layer);
    if (GENERAL && gbc == TENOAA_BC_HALO) {
      double* hb = A.hbar[side] + tc + nA * bcoord + (layer - 1) * NV * plane;
      unroll<NV>([&](auto cc) { unsafeAtomicAdd(&hb[cc * plane], Ub[cc]); });
      return;
    }
    const int64_t off = l * stride[DIR] + tc * stride[AX_A] + bcoord * stride[AX_B];
    unroll<NV>([&](auto cc) { unsafeAtomicAdd(&A.Ubar[cc * ncell + off], Ub[cc]); });
  };
  // every tile cell's adjoint in parallel.  A ghost position whose source is
  // a domain cell of this tile (outflow, wall and Dirichlet ghosts, a
  // periodic image the window wraps onto) is folded into that cell's sum
  // after a barrier - the cell's own adjoint first, then the ghosts in window
  // order - and the sum goes to U_bar.  Every other adjoint goes at once:
  // domain cells of a tile with nothing to fold (distinct cells, and no other
  // tile of this launch touches them), periodic images in another tile, halo
  // cells.  The adjoints to fold wait in the LDS accumulator slots: aW the
  // adjoint, aC the window position + 1 of the cell it folds into (0: none).
  const int64_t lo_w = f0 - G;  // raw position of window cell 0
  auto folds = [&](int bc) {
    return bc == TENOAA_BC_PERIODIC ? nN < NC : (bc != TENOAA_BC_HALO && bc != TENOAA_BC_INFLOW);
  };
  const bool ghosts = (lo_w < 0 && folds(A.bc_lo)) || (lo_w + NC > nN && folds(A.bc_hi));
  auto fold_pos = [&](int ttc, int nn) -> int {
    int64_t tc, l, layer;
    int gbc, side;
    map_cell(ttc, nn, tc, l, gbc, side, layer);
    if (GENERAL && gbc == TENOAA_BC_HALO) return -1;
    const int64_t q = l - lo_w;
    return (q >= 0 && q < NC) ? (int)q : -1;
  };
  for (int cs = threadIdx.x; cs < NCT; cs += NTH) {
    int ttc, nn;
    cell_of(cs, ttc, nn);
    const int ct = ttc * NC + nn;
    const int64_t l = lo_w + nn;
    double Ub[NV];
    const bool has = cell_adjoint(ttc, nn, Ub);
    if (!ghosts) {
      if (has) add_to_source(ttc, nn, Ub);
      continue;
    }
    int q = -1;
    if (has) {
      q = (l >= 0 && l < nN) ? nn : fold_pos(ttc, nn);
      if (q < 0) add_to_source(ttc, nn, Ub);
    }
    unroll<NV>([&](auto cc) { aW[cc][ct] = Ub[cc]; });
    aC[ct] = (double)(q + 1);
  }
  if (ghosts) {
    __syncthreads();
    // ghost positions of the window: [0, gl) low side, [gh, NC) high side
    const int gl = lo_w < 0 ? (int)(-lo_w < NC ? -lo_w : NC) : 0;
    const int gh = lo_w + NC > nN ? (int)(nN - lo_w > 0 ? nN - lo_w : 0) : NC;
    for (int cs = threadIdx.x; cs < NCT; cs += NTH) {
      int ttc, nn;
      cell_of(cs, ttc, nn);
      const int64_t l = lo_w + nn;
      const int ct = ttc * NC + nn;
      if (l < 0 || l >= nN || aC[ct] == 0.0) continue;
      double Ub[NV];
      unroll<NV>([&](auto cc) { Ub[cc] = aW[cc][ct]; });
      const double me = (double)(nn + 1);
      for (int g = 0; g < NC; ++g) {
        if (g == gl && gl < gh) g = gh;  // skip the domain positions
        if (g >= NC) break;
        const int cg = ttc * NC + g;
        if (aC[cg] == me) unroll<NV>([&](auto cc) { Ub[cc] += aW[cc][cg]; });
      }
      add_to_source(ttc, nn, Ub);
    }
  }
}

// The reverse sweep over the faces [a.f_begin, f_end) of a direction in
// tiles of TT pencils x TN faces, in launches of tiles that share no cell: a
// tile's window reaches into its neighbours' only (TN >= 2 G - 1), so the
// even tiles, then the odd ones.  Along a periodic direction the wrap makes
// the first and the last tile neighbours (with an odd count, the last runs on
// its own); when the cells from the last tile's start to the end of the
// direction are fewer than 2 G - 1, it also joins the first tile to the one
// before the last and the second to the last, and the last two run on their own.
template <int ORDER, int NDIM, int DIR, int TT, int TN, bool GENERAL>
hipError_t launch_vjp_tiles(const AdjointArgs& a, int64_t f_end, hipStream_t st) {
  constexpr int AX_A = (DIR == 0) ? 1 : 0;
  constexpr int AX_B = (DIR == 2) ? 1 : 2;
  const int64_t ntile = (f_end - a.f_begin + TN - 1) / TN;
  // narrower tiles (the tail's) come one per pencil
  if (TN < ORDER - 1 && ntile > 1) return hipErrorInvalidValue;
  // tiles [body, ntile) run one per launch; the rest alternate
  int64_t body = ntile;
  if (a.bc_lo == TENOAA_BC_PERIODIC && ntile >= 2) {
    const bool short_last = a.f_begin != 0 || a.n[DIR] - (ntile - 1) * TN < ORDER - 1;
    body = short_last ? ntile - 2 : (ntile % 2 == 0 ? ntile : ntile - 1);
  }
  const int64_t first[4] = {0, 1, body, body + 1};
  const int64_t count[4] = {(body + 1) / 2, body / 2, ntile - body, ntile - body - 1};
  for (int c = 0; c < 4; ++c) {
    if (count[c] <= 0) continue;
    AdjointArgs b = a;
    b.tile_first = first[c];
    b.tile_step = 2;
    const unsigned nb = (unsigned)(c < 2 ? count[c] : 1);
    dim3 grid(nb, (unsigned)((a.n[AX_A] + TT - 1) / TT), (unsigned)a.n[AX_B]);
    hipLaunchKernelGGL((sweep_vjp_kernel<ORDER, NDIM, DIR, TT, TN, GENERAL>), grid, dim3(TT * TN), 0, st, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The whole-tile shapes: x (and 1D) TENOAA_ADJ_TT_X x TENOAA_ADJ_TN_X, y and
// z TENOAA_ADJ_TT_YZ x TENOAA_ADJ_TN_YZ.
template <int ORDER, bool GENERAL>
hipError_t launch_vjp_shape(int ndim, int dir, const AdjointArgs& a, int64_t f_end, hipStream_t st) {
  constexpr int TTX = TENOAA_ADJ_TT_X, TNX = TENOAA_ADJ_TN_X, TTY = TENOAA_ADJ_TT_YZ, TNY = TENOAA_ADJ_TN_YZ;
  if (ndim == 1) return launch_vjp_tiles<ORDER, 1, 0, 1, TNX, GENERAL>(a, f_end, st);
  if (ndim == 2) {
    return dir == 0 ? launch_vjp_tiles<ORDER, 2, 0, TTX, TNX, GENERAL>(a, f_end, st)
                    : launch_vjp_tiles<ORDER, 2, 1, TTY, TNY, GENERAL>(a, f_end, st);
  }
  if (dir == 0) return launch_vjp_tiles<ORDER, 3, 0, TTX, TNX, GENERAL>(a, f_end, st);
  if (dir == 1) return launch_vjp_tiles<ORDER, 3, 1, TTY, TNY, GENERAL>(a, f_end, st);
  return launch_vjp_tiles<ORDER, 3, 2, TTY, TNY, GENERAL>(a, f_end, st);
}

template <bool GENERAL>
hipError_t launch_vjp_kind(int order, int ndim, int dir, const AdjointArgs& a, int64_t f_end, hipStream_t st) {
  if (order == 12) return launch_vjp_shape<12, GENERAL>(ndim, dir, a, f_end, st);
  if (order == 10) return launch_vjp_shape<10, GENERAL>(ndim, dir, a, f_end, st);
  return launch_vjp_shape<8, GENERAL>(ndim, dir, a, f_end, st);
}

}  // namespace
}  // namespace tenoaa
