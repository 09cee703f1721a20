// Device bodies of the forward path, shared by the per-grid kernels
// (tenoaa_kernels.hip) and the batched persistent kernel (tenoaa_batch.hip),
// so that both evaluate every face and cell with the same operations:
//
//   sweep_tile   one tile of faces of one direction: staging of the cell
//                records in LDS (boundary conditions by index mapping, cell
//                primitives and physical flux, Sec. 1), then per face the Roe
//                average and eigenvectors, projection, LLF/Rusanov split,
//                TENO-AA reconstruction of both sides (Sec. 3, 4),
//                back-projection and the optional positivity limiter (Sec. 5);
//   update_cell  flux difference and the SSP-RK3 stage of one cell;
//   cell_speeds  |u_d| + c of one cell for the CFL condition;
//   dt_and_mu    dt = CFL / sum_d a_d/dx_d and the limiter factors.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "tenoaa_device.h"
#include "tenoaa_internal.h"

// 1: a scheduling barrier after each window cell of the projection (tuning)
#ifndef TENOAA_CELL_BARRIER
#define TENOAA_CELL_BARRIER 0
#endif
// > 0: x-sweep waves take patches of this many faces by 64 / it pencils
// instead of 64 faces of one pencil, so that a wave's lanes meet the deep
// cascade together more often (tuning; 0 restores whole-pencil waves)
#ifndef TENOAA_X_PATCH
#define TENOAA_X_PATCH 16
#endif

namespace tenoaa {
namespace {

// Tile geometry of a sweep: TN faces along the direction for each of TT
// pencils; the tile stages TN + W - 1 cells per pencil.
template <int ORDER, int NDIM, int TT, int TN>
struct SweepShape {
  static constexpr int W = ORDER;
  static constexpr int NV = NDIM + 2;
  static constexpr int NT = (NDIM > 1) ? NDIM - 1 : 1;
  static constexpr int NC = TN + W - 1;
  static constexpr int NCT = TT * NC;
  static constexpr int NTH = TT * TN;
  // cells that are one of the two cells of a face of the tile: TN + 1 per pencil
  static constexpr int NFC = TN + 1;
  static constexpr int NFCT = TT * NFC;
  // per-cell records: NV double2 (conserved, flux) + un, c for every staged
  // cell; sqrt(rho), H and the NT tangential velocities for the face cells
  static constexpr int LDS_BYTES = NCT * (16 * NV + 16) + NFCT * 8 * (2 + NT);
};

// Splitting of a sweep, fixed at compile time (TENOAA_LLF, TENOAA_RUSANOV,
// TENOAA_ROE), or SPLIT_RUNTIME: LLF or Rusanov as the arguments say.
constexpr int SPLIT_RUNTIME = -1;

// Dirichlet ghost cell (Appendix A): in primitive variables the ghost is the
// mirror cell reflected through the prescribed face value,
// (rho, u, p)_ghost = 2 (rho, u, p)_face - (rho, u, p)_mirror.  W holds the
// mirror cell's conserved state on entry and the ghost's on return; fv points
// at the face density, its velocities and pressure following at strides of
// `plane`.
template <int NDIM>
__device__ __forceinline__ void dirichlet_ghost(double* W, const double* fv, int64_t plane, double gm1) {
  constexpr int NV = NDIM + 2;
  const double rho = W[0];
  const double ir = div_rn(1.0, rho);
  double u[NDIM];
  double q2 = 0.0;
  unroll<NDIM>([&](auto k) {
    u[k] = W[1 + k] * ir;
    q2 = (k == 0) ? u[0] * u[0] : q2 + u[k] * u[k];
  });
  const double p = gm1 * (W[NV - 1] - (0.5 * rho) * q2);
  const double rg = 2.0 * fv[0] - rho;
  double qg = 0.0;
  unroll<NDIM>([&](auto k) {
    const double ug = 2.0 * fv[(1 + k) * plane] - u[k];
    W[1 + k] = rg * ug;
    qg = (k == 0) ? ug * ug : qg + ug * ug;
  });
  const double pg = 2.0 * fv[(NV - 1) * plane] - p;
  W[0] = rg;
  W[NV - 1] = div_rn(pg, gm1) + (0.5 * rg) * qg;
}

// Prescribed ghost cell (supersonic inflow, where every characteristic enters
// the domain): the conserved state of the primitives at pv (density, then
// velocities and pressure at strides of `plane`).
template <int NDIM>
__device__ __forceinline__ void inflow_ghost(double* W, const double* pv, int64_t plane, double gm1) {
  constexpr int NV = NDIM + 2;
  const double rho = pv[0];
  double q2 = 0.0;
  unroll<NDIM>([&](auto k) {
    const double u = pv[(1 + k) * plane];
    W[1 + k] = rho * u;
    q2 = (k == 0) ? u * u : q2 + u * u;
  });
  W[0] = rho;
  W[NV - 1] = div_rn(pv[(NV - 1) * plane], gm1) + (0.5 * rho) * q2;
}

// One tile of faces.  (bx, by, bz) = (tile index along the direction, tile
// index across it, coordinate along the remaining axis).  `lds` holds at
// least SweepShape::LDS_BYTES bytes, 16-byte aligned; the caller separates
// consecutive tiles that reuse it with a barrier.  `mu` is the limiter factor
// of this direction (used when LIMIT).  ROE selects the Roe flux with entropy
// fix (SPLIT = TENOAA_ROE); SPLIT = TENOAA_LLF or TENOAA_RUSANOV fixes the
// flux splitting, SPLIT_RUNTIME takes it from A.splitting.  AUDIT (LLF or
// Rusanov only) takes each decision live unless A.near_in marks it, replays
// A.frozen where it does, and reports in A.near_out which live decisions lie
// within A.near_tol of a threshold.
template <int ORDER, int NDIM, int DIR, int TT, int TN, bool LIMIT, int SPLIT = SPLIT_RUNTIME, bool AUDIT = false>
__device__ __forceinline__ void sweep_tile(const SweepArgs& A, char* lds, int64_t bx, int64_t by, int64_t bz,
                                           double mu) {
  static_assert(SPLIT == SPLIT_RUNTIME || SPLIT == TENOAA_LLF || SPLIT == TENOAA_RUSANOV || SPLIT == TENOAA_ROE,
                "unknown splitting");
  constexpr bool ROE = SPLIT == TENOAA_ROE;
  static_assert(!(AUDIT && ROE), "the audit sweep splits the fluxes");
  using Sh = SweepShape<ORDER, NDIM, TT, TN>;
  constexpr int G = ORDER / 2;
  constexpr int W = ORDER;
  constexpr int NV = Sh::NV;
  constexpr int NT = Sh::NT;
  constexpr int NC = Sh::NC;
  constexpr int NCT = Sh::NCT;
  constexpr int NFC = Sh::NFC;
  constexpr int NFCT = Sh::NFCT;
  constexpr int AX_A = (DIR == 0) ? 1 : 0;  // transverse axis spread over threads
  constexpr int AX_B = (DIR == 2) ? 1 : 2;  // remaining axis
  using Fr = Frame<NDIM, DIR>;

  // per-cell records: half the (conserved, flux) pairs in the local frame
  // (the splitting's factor 1/2, exact as a power of two, applied once per
  // cell), normal velocity, sound speed; for the face cells also sqrt(rho),
  // enthalpy and the tangential velocities
  double2* const sWF = reinterpret_cast<double2*>(lds);
  double* const sUn = reinterpret_cast<double*>(lds + 16 * NV * NCT);
  double* const sC = sUn + NCT;
  double* const sSr = sC + NCT;
  double* const sH = sSr + NFCT;
  double* const sUt = sH + NFCT;

  const int64_t nN = A.n[DIR];
  const int64_t nA = A.n[AX_A];
  const int64_t stride[3] = {1, A.n[0], A.n[0] * A.n[1]};
  const int64_t ncell = A.n[0] * A.n[1] * A.n[2];
  const int64_t f0 = A.f_begin + bx * TN;
  const int64_t t0 = by * TT;
  const int64_t bcoord = bz;
  const double gam = A.gamma;
  const double gm1 = gam - 1.0;

  // ---- stage the tile: cells f0-G .. f0+TN+G-2 along the normal
  for (int ct = threadIdx.x; ct < NCT; ct += TT * TN) {
    int tt, nn;
    if (DIR == 0) {
      tt = ct / NC;
      nn = ct % NC;
    } else {
      tt = ct % TT;
      nn = ct / TT;
    }
    int64_t t = t0 + tt;
    if (t >= nA) t = nA - 1;
    int64_t l = f0 - G + nn;
    int bc = -1;  // the boundary that makes this a ghost cell, -1 for a domain cell
    const int side = (l < 0) ? 0 : 1;
    const int64_t layer = (l < 0) ? -l : l - nN + 1;  // ghost layer r = 1, 2, ... outward
    if (l < 0 || l >= nN) {
      bc = (l < 0) ? A.bc_lo : A.bc_hi;
      if (bc == TENOAA_BC_PERIODIC) {
        l = ((l % nN) + nN) % nN;
        bc = -1;
      } else if (bc == TENOAA_BC_OUTFLOW || layer > G) {
        // outflow, or a cell beyond the G ghost layers that no face of the tile reads
        l = (l < 0) ? 0 : nN - 1;
        bc = -1;
      } else {
        l = (l < 0) ? -l - 1 : 2 * nN - 1 - l;  // mirror cell
      }
      if (l < 0) l = 0;
      if (l >= nN) l = nN - 1;
    }
    const int64_t off = l * stride[DIR] + t * stride[AX_A] + bcoord * stride[AX_B];
    double Wc[NV];
    unroll<NV>([&](auto c) { Wc[c] = A.U[c * ncell + off]; });
    if (bc >= 0) {
      // values of this pencil's cell of the face plane: the transverse index
      // t, then the remaining axis
      const int64_t plane = nA * A.n[AX_B];
      const double* fv = A.bcv[side] + t + nA * bcoord;
      if (bc == TENOAA_BC_SYMMETRY) {
        Wc[1 + DIR] = -Wc[1 + DIR];
      } else if (bc == TENOAA_BC_NOSLIP) {
        unroll<NDIM>([&](auto k) { Wc[1 + k] = -Wc[1 + k]; });
      } else if (bc == TENOAA_BC_DIRICHLET) {
        dirichlet_ghost<NDIM>(Wc, fv, plane, gm1);
      } else if (bc == TENOAA_BC_INFLOW) {
        inflow_ghost<NDIM>(Wc, fv + (layer - 1) * NV * plane, plane, gm1);
      } else {  // halo: the neighbour piece's conserved state
        unroll<NV>([&](auto c) { Wc[c] = fv[((layer - 1) * NV + c) * plane]; });
      }
    }
    // cell primitives (Sec. 1), axis order
    const double rho = Wc[0];
    const double ir = div_rn(1.0, rho);  // divisions by rho as products with its reciprocal
    double u[NDIM];
    double q2 = 0.0;
    unroll<NDIM>([&](auto k) {
      u[k] = Wc[1 + k] * ir;
      q2 = (k == 0) ? u[0] * u[0] : q2 + u[k] * u[k];
    });
    const double E = Wc[NV - 1];
    const double p = gm1 * (E - (0.5 * rho) * q2);
    const double c = sqrt_rn((gam * p) * ir);
    const double un = u[DIR];
    if (!(rho > 0.0) || !(p > 0.0)) atomicOr(A.status, 1);
    // half the conserved state and physical flux along DIR in the local frame
    sWF[ct] = make_double2(0.5 * rho, 0.5 * Wc[1 + DIR]);
    unroll<NDIM>([&](auto k) {
      constexpr int slot = Fr::slot_of_axis(decltype(k)::value);
      sWF[(1 + slot) * NCT + ct] =
          make_double2(0.5 * Wc[1 + k], 0.5 * ((k == DIR) ? Wc[1 + k] * un + p : Wc[1 + k] * un));
    });
    sWF[(NV - 1) * NCT + ct] = make_double2(0.5 * E, 0.5 * ((E + p) * un));
    sUn[ct] = un;
    sC[ct] = c;
    if (nn >= G - 1 && nn <= G - 1 + TN) {  // one of the two cells of a face of the tile
      const int fc = (DIR == 0) ? tt * NFC + (nn - (G - 1)) : (nn - (G - 1)) * TT + tt;
      sSr[fc] = sqrt_rn(rho);
      sH[fc] = (E + p) * ir;
      unroll<NDIM>([&](auto k) {
        constexpr int slot = Fr::slot_of_axis(decltype(k)::value);
        if constexpr (slot > 0) sUt[(slot - 1) * NFCT + fc] = u[k];
      });
    }
  }
  __syncthreads();

  // ---- one face per thread
  int tt, fn;
  if (DIR == 0) {
#if TENOAA_X_PATCH > 0
    // a wave takes TENOAA_X_PATCH faces of 64 / TENOAA_X_PATCH pencils
    if constexpr (TT * TN % 64 == 0 && TN % TENOAA_X_PATCH == 0 && TT % (64 / TENOAA_X_PATCH) == 0 && TT > 1) {
      constexpr int PW = TENOAA_X_PATCH, PH = 64 / TENOAA_X_PATCH, NPX = TN / PW;
      const int w = threadIdx.x / 64, l = threadIdx.x % 64;
      tt = (w / NPX) * PH + l / PW;
      fn = (w % NPX) * PW + l % PW;
    } else {
      tt = threadIdx.x / TN;
      fn = threadIdx.x % TN;
    }
#else
    tt = threadIdx.x / TN;
    fn = threadIdx.x % TN;
#endif
  } else {
    tt = threadIdx.x % TT;
    fn = threadIdx.x / TT;
  }
  const int64_t f = f0 + fn;
  const int64_t t = t0 + tt;
  if (f >= A.nf || t >= nA) return;
  // LDS index of window cell j (cells f-G .. f+G-1)
  const int lbase = (DIR == 0) ? tt * NC + fn : fn * TT + tt;
  constexpr int LSTEP = (DIR == 0) ? 1 : TT;
  const int ia = lbase + (G - 1) * LSTEP, ib = lbase + G * LSTEP;
  // index of the face's two cells among the face-cell records
  const int fa = (DIR == 0) ? tt * NFC + fn : fn * TT + tt, fb = fa + LSTEP;

  // Roe average (Sec. 5: characteristic decomposition at the face)
  const double sa = sSr[fa], sb = sSr[fb];
  const double den = sa + sb;
  const double iden = div_rn(1.0, den);  // the Roe weights' denominator, inverted once
  const double un = (sa * sUn[ia] + sb * sUn[ib]) * iden;
  double ut[NT];
  unroll<NDIM - 1>([&](auto k) { ut[k] = (sa * sUt[k * NFCT + fa] + sb * sUt[k * NFCT + fb]) * iden; });
  double q2 = 0.0;  // |u|^2 summed in axis order
  unroll<NDIM>([&](auto a) {
    constexpr int slot = Fr::slot_of_axis(decltype(a)::value);
    double ua;
    if constexpr (slot == 0) ua = un;
    else ua = ut[slot - 1];
    q2 = (a == 0) ? ua * ua : q2 + ua * ua;
  });
  const double Hr = (sa * sH[fa] + sb * sH[fb]) * iden;
  const double qq = 0.5 * q2;
  const double c2 = gm1 * (Hr - qq);
  const double cr = sqrt_rn(c2);
  const double b1 = div_rn(gm1, c2);
  const double b2 = b1 * qq;
  const double ic = div_rn(1.0, cr);
  const double unc = un * ic;
  // splitting speeds over the window
  double am = 0.0, a0 = 0.0, ap = 0.0;
  auto llf_speeds = [&]() {  // LLF, also the Roe flux's fallback
    unroll<W>([&](auto j) {
      const int li = lbase + j * LSTEP;
      const double u = sUn[li], c = sC[li];
      am = fmax(am, fabs(u - c));
      a0 = fmax(a0, fabs(u));
      ap = fmax(ap, fabs(u + c));
    });
  };
  auto rusanov_speeds = [&]() {
    unroll<W>([&](auto j) {
      const int li = lbase + j * LSTEP;
      a0 = fmax(a0, fabs(sUn[li]) + sC[li]);
    });
    am = ap = a0;
  };
  if constexpr (SPLIT == TENOAA_LLF || ROE) {
    llf_speeds();
  } else if constexpr (SPLIT == TENOAA_RUSANOV) {
    rusanov_speeds();
  } else {
    if (A.splitting == TENOAA_LLF) llf_speeds();
    else rusanov_speeds();
  }

  int64_t flin;
  {
    int64_t m[3] = {A.n[0], A.n[1], A.n[2]};
    m[DIR] = A.nf;
    const int64_t fstr[3] = {1, m[0], m[0] * m[1]};
    flin = f * fstr[DIR] + t * fstr[AX_A] + bcoord * fstr[AX_B];
  }
  // the recording for the reverse sweep is pencil by pencil (the same as grid
  // order along x)
  const int64_t frec = A.rec_pencil_major ? f + A.nf * (t + nA * bcoord) : flin;
  uint8_t* const flag_out = A.flags ? A.flags + frec : nullptr;
  const uint8_t* const frozen = A.frozen ? A.frozen + flin : nullptr;

  // One characteristic field s (a compile-time constant, so its eigenvector
  // row, splitting speed and projection form are fixed in the code): the
  // projection of the window, the split and the reconstructions of both
  // sides.  Returns fh_s.
  auto field = [&](auto sc) -> double {
    constexpr int s = decltype(sc)::value;
    constexpr bool shear = (s >= 2 && s <= NV - 2);
    // left eigenvector row s (local frame), the reading of the Roe eigenvectors
    double L[NV];
    if constexpr (s == 0 || s == NV - 1) {
      L[0] = (s == 0) ? 0.5 * (b2 + unc) : 0.5 * (b2 - unc);
      L[1] = (s == 0) ? 0.5 * (-b1 * un - ic) : 0.5 * (-b1 * un + ic);
      unroll<NDIM - 1>([&](auto k) { L[2 + k] = 0.5 * (-b1 * ut[k]); });
      L[NV - 1] = 0.5 * b1;
    } else if constexpr (s == 1) {
      L[0] = 1.0 - b2;
      L[1] = b1 * un;
      unroll<NDIM - 1>([&](auto k) { L[2 + k] = b1 * ut[k]; });
      L[NV - 1] = -b1;
    }
    // shear field s: the tangential momentum of local slot s less u_t rho
    [[maybe_unused]] double mut = 0.0;
    if constexpr (shear) mut = -ut[s - 2];
    const double alpha = (s == 0) ? am : (s == NV - 1 ? ap : a0);
    // Roe flux with entropy fix: where the field's eigenvalue keeps one
    // strict sign at both cells of the face, the unsplit characteristic flux
    // is reconstructed from the upwind side alone; elsewhere LLF
    int upwind = 0;  // 0: split, 1: + side only, 2: - side only
    if constexpr (ROE) {
      if (frozen) {
        // replay: the side the recorded decisions reconstruct (the other's byte is 0)
        const uint8_t bp = frozen[(int64_t)(s * 2 + 0) * A.nft], bm = frozen[(int64_t)(s * 2 + 1) * A.nft];
        upwind = bm == 0 ? 1 : (bp == 0 ? 2 : 0);
      } else {
        constexpr double ka = (s == 0) ? -1.0 : (s == NV - 1 ? 1.0 : 0.0);
        const double la = sUn[ia] + ka * sC[ia], lb = sUn[ib] + ka * sC[ib];
        upwind = (la > 0.0 && lb > 0.0) ? 1 : ((la < 0.0 && lb < 0.0) ? 2 : 0);
      }
    }
    // projection of the window's (halved) state and flux on field s, then the split
    double gp[W], gm[W];
    unroll<W>([&](auto j) {
      const int li = lbase + j * LSTEP;
      double v, g;
      if constexpr (!shear) {
        const double2 w0 = sWF[li];
        v = L[0] * w0.x;
        g = L[0] * w0.y;
        unroll<NV - 1>([&](auto cc) {
          const double2 w = sWF[(cc + 1) * NCT + li];
          v = fma(L[cc + 1], w.x, v);
          g = fma(L[cc + 1], w.y, g);
        });
      } else {
        // the row's other entries are zero and its entry at slot s is one
        const double2 w0 = sWF[li];
        const double2 ws = sWF[s * NCT + li];
        v = mut * w0.x + ws.x;
        g = mut * w0.y + ws.y;
      }
      // v, g are half the projections: the split 1/2 (g +- alpha v) is one fma
      if (!ROE || upwind == 0) {
        gp[j] = fma(alpha, v, g);
        gm[W - 1 - j] = fma(-alpha, v, g);  // mirrored for the - side
      } else {
        gp[j] = 2.0 * g;
        gm[W - 1 - j] = 2.0 * g;
      }
#if TENOAA_CELL_BARRIER
      __builtin_amdgcn_sched_barrier(0);
#endif
    });
    uint8_t flp = 0, flm = 0;
    double hp, hm;
    if constexpr (AUDIT) {
      // live decisions except where near_in marks a replayed one
      const int64_t op = (int64_t)(s * 2 + 0) * A.nft, om = (int64_t)(s * 2 + 1) * A.nft;
      const uint8_t* nin = A.near_in ? A.near_in + flin : nullptr;
      uint8_t np = 1, nm = 1;
      if (nin && nin[op]) {
        flp = frozen[op];
        hp = replay_recon<ORDER>(gp, flp);
      } else {
        hp = teno_aa<ORDER, true>(gp, flp, &np, A.near_tol);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (nin && nin[om]) {
        flm = frozen[om];
        hm = replay_recon<ORDER>(gm, flm);
      } else {
        hm = teno_aa<ORDER, true>(gm, flm, &nm, A.near_tol);
      }
      if (A.near_out) {
        A.near_out[flin + op] = np;
        A.near_out[flin + om] = nm;
      }
    } else if (frozen) {
      // replay recorded decisions
      flp = frozen[(int64_t)(s * 2 + 0) * A.nft];
      flm = frozen[(int64_t)(s * 2 + 1) * A.nft];
      hp = replay_recon<ORDER>(gp, flp);
      hm = replay_recon<ORDER>(gm, flm);
    } else if constexpr (ROE) {
      hp = 0.0;
      hm = 0.0;
      if (upwind != 2) hp = teno_aa<ORDER>(gp, flp);
      __builtin_amdgcn_sched_barrier(0);
      if (upwind != 1) hm = teno_aa<ORDER>(gm, flm);
    } else {
      hp = teno_aa<ORDER>(gp, flp);
      // keep the two reconstructions from being interleaved (register pressure)
      __builtin_amdgcn_sched_barrier(0);
      hm = teno_aa<ORDER>(gm, flm);
    }
    if (flag_out) {
      flag_out[(int64_t)(s * 2 + 0) * A.nft] = flp;
      flag_out[(int64_t)(s * 2 + 1) * A.nft] = flm;
    }
    const double fh = (!ROE || upwind == 0) ? hp + hm : (upwind == 1 ? hp : hm);
    if (A.fh_out) A.fh_out[(int64_t)s * A.nft + frec] = fh;
    return fh;
  };
  // every field its own code; a scheduling barrier between two fields keeps
  // their working sets from overlapping (register pressure)
  double fhs[NV];
  unroll<NV>([&](auto sc) {
    fhs[sc] = field(sc);
    __builtin_amdgcn_sched_barrier(0);
  });

  // back-projection F = sum_s R[:, s] fh_s, accumulated over s in order; the
  // zero entries of a shear field's column add nothing (skipped) and its unit
  // entry is an addition
  double Fh[NV];  // back-projected flux, local frame
  {
    const double fa = fhs[0];
    Fh[0] = fa;
    Fh[1] = (un - cr) * fa;
    unroll<NDIM - 1>([&](auto k) { Fh[2 + k] = ut[k] * fa; });
    Fh[NV - 1] = (Hr - un * cr) * fa;
    const double fe = fhs[1];
    Fh[0] = Fh[0] + fe;
    Fh[1] = fma(un, fe, Fh[1]);
    unroll<NDIM - 1>([&](auto k) { Fh[2 + k] = fma(ut[k], fe, Fh[2 + k]); });
    Fh[NV - 1] = fma(qq, fe, Fh[NV - 1]);
    unroll<NDIM - 1>([&](auto k) {
      const double fk = fhs[2 + k];
      Fh[2 + k] = Fh[2 + k] + fk;
      Fh[NV - 1] = fma(ut[k], fk, Fh[NV - 1]);
    });
    const double fz = fhs[NV - 1];
    Fh[0] = Fh[0] + fz;
    Fh[1] = fma(un + cr, fz, Fh[1]);
    unroll<NDIM - 1>([&](auto k) { Fh[2 + k] = fma(ut[k], fz, Fh[2 + k]); });
    Fh[NV - 1] = fma(Hr + un * cr, fz, Fh[NV - 1]);
  }

  if constexpr (LIMIT) {
    // Positivity limiter (reading of Hu, Adams & Shu 2013, applied in Sec. 5.3).
    const double sA = fabs(sUn[ia]) + sC[ia];
    const double sB = fabs(sUn[ib]) + sC[ib];
    const double aL = (sA >= sB) ? sA : sB;
    double FL[NV];
    unroll<NV>([&](auto c) {
      // the records hold half the state and flux: this is 1/2 (F_a + F_b - aL (U_b - U_a))
      const double2 wa = sWF[c * NCT + ia], wb = sWF[c * NCT + ib];
      FL[c] = (wa.y + wb.y) - aL * (wb.x - wa.x);
    });
    // pressure of X; EXACT selects correctly rounded divisions, otherwise
    // the compiler's (within an ulp), and `scale` bounds the terms of p
    auto pressure = [&](const double (&X)[NV], auto exact, double& scale) {
      const double rho = X[0];
      const double ir = decltype(exact)::value ? div_rn(1.0, rho) : 1.0 / rho;
      double q = 0.0;
      unroll<NDIM>([&](auto a) {
        const double ua = X[1 + Fr::slot_of_axis(decltype(a)::value)] * ir;
        q = (a == 0) ? ua * ua : q + ua * ua;
      });
      const double k = (0.5 * rho) * q;
      scale = fabs(X[NV - 1]) + fabs(k);
      return gm1 * (X[NV - 1] - k);
    };
    double th_r = 1.0;
    unroll<2>([&](auto side) {
      const int li = side == 0 ? ia : ib;
      const double sg = side == 0 ? -1.0 : 1.0;
      const double r = 2.0 * sWF[li].x;
      const double rL = r + (sg * mu) * FL[0];
      const double rH = r + (sg * mu) * Fh[0];
      const double eps = rL < 1e-13 ? rL : 1e-13;
      if (rH < eps) {
        const double th = div_rn(rL - eps, rL - rH);
        th_r = th < th_r ? th : th_r;
      }
    });
    double Fs[NV];
    unroll<NV>([&](auto c) { Fs[c] = (th_r < 1.0) ? FL[c] + th_r * (Fh[c] - FL[c]) : Fh[c]; });
    double th_p = 1.0;
    unroll<2>([&](auto side) {
      const int li = side == 0 ? ia : ib;
      const double sg = side == 0 ? -1.0 : 1.0;
      double XL[NV], XS[NV];
      unroll<NV>([&](auto c) {
        const double x = 2.0 * sWF[c * NCT + li].x;
        XL[c] = x + (sg * mu) * FL[c];
        XS[c] = x + (sg * mu) * Fs[c];
      });
      // The test pS < eps with the compiler's divisions differs from the exact
      // one only if pS is within ~1e-15 of the pressures' term scale of eps;
      // outside a 1e-12 band the limiter certainly leaves this side alone.
      double sL, sS;
      const double pLf = pressure(XL, std::false_type{}, sL);
      const double pSf = pressure(XS, std::false_type{}, sS);
      const double epsf = pLf < 1e-13 ? pLf : 1e-13;
      if (pSf < epsf + 1e-12 * (sL + sS)) {
        const double pL = pressure(XL, std::true_type{}, sL);
        const double pS = pressure(XS, std::true_type{}, sS);
        const double eps = pL < 1e-13 ? pL : 1e-13;
        const double th = (pS < eps) ? div_rn(pL - eps, pL - pS) : 1.0;
        th_p = th < th_p ? th : th_p;
      }
    });
    unroll<NV>([&](auto c) { Fh[c] = (th_p < 1.0) ? FL[c] + th_p * (Fs[c] - FL[c]) : Fs[c]; });
    // for the adjoint: the flux is F_LF + theta (F_H - F_LF) with theta = theta_rho theta_p
    if (A.theta_out) A.theta_out[frec] = th_r * th_p;
  } else {
    (void)mu;
  }

  // store in axis order
  A.F[flin] = Fh[0];
  A.F[(int64_t)(NV - 1) * A.nft + flin] = Fh[NV - 1];
  unroll<NDIM>([&](auto a) {
    constexpr int slot = Fr::slot_of_axis(decltype(a)::value);
    A.F[(int64_t)(1 + a) * A.nft + flin] = Fh[1 + slot];
  });
}

// |u_d| + c of one cell (state Wc, conserved, axis order) folded into amax;
// `bad` is set for a non-physical state.
template <int NDIM>
__device__ __forceinline__ void cell_speeds(const double (&Wc)[NDIM + 2], double gam, double (&amax)[NDIM],
                                            bool& bad) {
  constexpr int NV = NDIM + 2;
  const double rho = Wc[0];
  const double ir = div_rn(1.0, rho);
  double u[NDIM];
  double q2 = 0.0;
  unroll<NDIM>([&](auto k) {
    u[k] = Wc[1 + k] * ir;
    q2 = (k == 0) ? u[0] * u[0] : q2 + u[k] * u[k];
  });
  const double p = (gam - 1.0) * (Wc[NV - 1] - (0.5 * rho) * q2);
  const double c = sqrt_rn((gam * p) * ir);
  if (!(rho > 0.0) || !(p > 0.0)) bad = true;
  unroll<NDIM>([&](auto d) { amax[d] = dmax(amax[d], fabs(u[d]) + c); });
}

// Flux difference and SSP-RK3 stage of cell idx = co[0] + n0 (co[1] + n1 co[2])
// (MODE 0: dU/dt; 1-3: stage).  The new state of the cell is left in Wn.
template <int NDIM, int MODE>
__device__ __forceinline__ void update_cell(const UpdateArgs& A, int64_t idx, const int64_t (&co)[3], double dt,
                                            double (&Wn)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  const int64_t ncell = A.n[0] * A.n[1] * A.n[2];
  int64_t fl[3], fr[3];
  unroll<NDIM>([&](auto d) {
    int64_t m[3] = {A.n[0], A.n[1], A.n[2]};
    m[d] = A.nf[d];
    const int64_t fs[3] = {1, m[0], m[0] * m[1]};
    int64_t c2[3] = {co[0], co[1], co[2]};
    fl[d] = c2[0] * fs[0] + c2[1] * fs[1] + c2[2] * fs[2];
    int64_t r = co[d] + 1;
    if (r == A.nf[d]) r = 0;  // periodic wrap (nf == n)
    c2[d] = r;
    fr[d] = c2[0] * fs[0] + c2[1] * fs[1] + c2[2] * fs[2];
  });
  unroll<NV>([&](auto c) {
    double du = 0.0;
    unroll<NDIM>([&](auto d) {
      const double* F = A.F[d] + (int64_t)c * A.nft[d];
      du = du - (F[fr[d]] - F[fl[d]]) * A.rdx[d];
    });
    const int64_t e = (int64_t)c * ncell + idx;
    double v;
    if (MODE == 0) {
      v = du;
    } else if (MODE == 1) {
      v = A.Un[e] + dt * du;
    } else if (MODE == 2) {
      v = 0.75 * A.Un[e] + 0.25 * A.Us[e] + (0.25 * dt) * du;
    } else {
      v = (1.0 / 3.0) * A.Un[e] + (2.0 / 3.0) * A.Us[e] + ((2.0 / 3.0) * dt) * du;
    }
    A.out[e] = v;
    Wn[c] = v;
  });
}

// Division of 32-bit unsigned integers by an invariant divisor d >= 1 with a
// multiply-high and a shift (Granlund and Montgomery): m and l from
// fastdiv_make on the host.
struct FastDiv {
  uint32_t m, l;
};
__device__ __forceinline__ uint32_t fastdiv(uint32_t n, FastDiv f) {
  return (uint32_t)(((uint64_t)__umulhi(f.m, n) + n) >> f.l);
}

// dt = cfl / sum_d a_d/dx_d (reading of the multi-dimensional CFL condition)
// unless dt_given > 0; limiter factors mu_d = 2 S / a_d with
// S = sum_d (dt/dx_d) a_d.
__device__ __forceinline__ void dt_and_mu(const unsigned long long* amax_bits, int ndim, const double* dx,
                                          double cfl, double dt_given, double& dt, double* mu) {
  double a[3];
  for (int d = 0; d < 3; ++d) a[d] = d < ndim ? __longlong_as_double((long long)amax_bits[d]) : 0.0;
  dt = dt_given;
  if (!(dt > 0.0)) {
    double s = div_rn(a[0], dx[0]);
    for (int d = 1; d < ndim; ++d) s = s + div_rn(a[d], dx[d]);
    dt = div_rn(cfl, s);
  }
  double Ssum = div_rn(dt, dx[0]) * a[0];
  for (int d = 1; d < ndim; ++d) Ssum = Ssum + div_rn(dt, dx[d]) * a[d];
  for (int d = 0; d < 3; ++d) mu[d] = (d < ndim) ? div_rn(2.0 * Ssum, a[d]) : 0.0;
}

}  // namespace
}  // namespace tenoaa
