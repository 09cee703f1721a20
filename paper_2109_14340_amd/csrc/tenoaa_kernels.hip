// TENO-AA8/10 Euler right-hand side: HIP kernels for gfx950 (FP64 VALU).
//
// One sweep kernel per direction evaluates every face flux of that direction:
// a block stages a tile of cells (plus the reconstruction halo, with the
// boundary conditions applied by index mapping) in LDS as per-cell records
// (conserved state and physical flux in the face's local frame, normal and
// tangential velocity, sound speed, sqrt(rho), enthalpy), then each thread
// takes one face: Roe average and eigenvectors (Sec. 5 of the paper),
// projection of the window onto one characteristic field at a time, LLF or
// Rusanov splitting, the scalar TENO-AA reconstruction of both split sides
// (Sec. 3, 4), back-projection and the optional positivity limiter.  Face
// fluxes go to a face array; a separate element-wise kernel forms the flux
// difference and the SSP-RK3 stage.
//
// Bit-for-bit agreement with the reference evaluation.  Every value that
// feeds a threshold decision (the split characteristic fluxes) is computed
// with one fixed order of IEEE operations: no contraction (this file is built
// with -ffp-contract=off), fma only where written, correctly rounded division
// and square root.  The smoothness indicators, the scale-separation test and
// the C_T bucket may differ from a reference evaluation by a few ulps, which
// can only move a decision that lies within ~1e-14 of its threshold.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "tenoaa_device.h"
#include "tenoaa_internal.h"

// Launch-shape tunables (overridable at build time).
#ifndef TENOAA_WAVES_PER_EU
#define TENOAA_WAVES_PER_EU 0
#endif
#ifndef TENOAA_TN_X
#define TENOAA_TN_X 64
#endif
#ifndef TENOAA_TT_X
#define TENOAA_TT_X 4
#endif
#ifndef TENOAA_TN_YZ
#define TENOAA_TN_YZ 16
#endif
#ifndef TENOAA_TT_YZ
#define TENOAA_TT_YZ 16
#endif
#ifndef TENOAA_CELL_BARRIER
#define TENOAA_CELL_BARRIER 0
#endif

namespace tenoaa {
namespace {

// ------------------------------------------------------------ sweep kernel
template <int ORDER, int NDIM, int DIR, int TT, int TN, bool LIMIT>
__global__ __launch_bounds__(TT* TN)
#if TENOAA_WAVES_PER_EU > 0
__attribute__((amdgpu_waves_per_eu(TENOAA_WAVES_PER_EU)))
#endif
void sweep_kernel(SweepArgs A) {
  constexpr int G = ORDER / 2;
  constexpr int W = ORDER;
  constexpr int NV = NDIM + 2;
  constexpr int NT = (NDIM > 1) ? NDIM - 1 : 1;
  constexpr int NC = TN + W - 1;  // cells along the normal in the tile
  constexpr int NCT = TT * NC;
  constexpr int AX_A = (DIR == 0) ? 1 : 0;  // transverse axis spread over threads
  constexpr int AX_B = (DIR == 2) ? 1 : 2;  // remaining axis (blockIdx.z)
  using Fr = Frame<NDIM, DIR>;

  // per-cell records: (conserved, flux) pairs in the local frame, then
  // normal velocity, sound speed, sqrt(rho), enthalpy, tangential velocities
  __shared__ double2 sWF[NV][NCT];
  __shared__ double sUn[NCT], sC[NCT], sSr[NCT], sH[NCT];
  __shared__ double sUt[NT][NCT];

  const int64_t nN = A.n[DIR];
  const int64_t nA = A.n[AX_A];
  const int64_t stride[3] = {1, A.n[0], A.n[0] * A.n[1]};
  const int64_t ncell = A.n[0] * A.n[1] * A.n[2];
  const int64_t f0 = (int64_t)blockIdx.x * TN;
  const int64_t t0 = (int64_t)blockIdx.y * TT;
  const int64_t bcoord = blockIdx.z;
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
    bool mirror = false;
    int bc = -1;
    if (l < 0 || l >= nN) {
      bc = (l < 0) ? A.bc_lo : A.bc_hi;
      if (bc == TENOAA_BC_PERIODIC) {
        l = ((l % nN) + nN) % nN;
      } else if (bc == TENOAA_BC_OUTFLOW) {
        l = (l < 0) ? 0 : nN - 1;
      } else {
        l = (l < 0) ? -l - 1 : 2 * nN - 1 - l;
        mirror = true;
      }
      if (l < 0) l = 0;
      if (l >= nN) l = nN - 1;
    }
    const int64_t off = l * stride[DIR] + t * stride[AX_A] + bcoord * stride[AX_B];
    double Wc[NV];
    unroll<NV>([&](auto c) { Wc[c] = A.U[c * ncell + off]; });
    if (mirror) {
      if (bc == TENOAA_BC_SYMMETRY) {
        Wc[1 + DIR] = -Wc[1 + DIR];
      } else {
        unroll<NDIM>([&](auto k) { Wc[1 + k] = -Wc[1 + k]; });
      }
    }
    // cell primitives (Sec. 1), axis order
    const double rho = Wc[0];
    double u[NDIM];
    double q2 = 0.0;
    unroll<NDIM>([&](auto k) {
      u[k] = Wc[1 + k] / rho;
      q2 = (k == 0) ? u[0] * u[0] : q2 + u[k] * u[k];
    });
    const double E = Wc[NV - 1];
    const double p = gm1 * (E - (0.5 * rho) * q2);
    const double c = sqrt((gam * p) / rho);
    const double H = (E + p) / rho;
    const double sr = sqrt(rho);
    const double un = u[DIR];
    if (!(rho > 0.0) || !(p > 0.0)) atomicOr(A.status, 1);
    // conserved state and physical flux along DIR in the local frame
    sWF[0][ct] = make_double2(rho, Wc[1 + DIR]);
    unroll<NDIM>([&](auto k) {
      constexpr int slot = Fr::slot_of_axis(decltype(k)::value);
      sWF[1 + slot][ct] = make_double2(Wc[1 + k], (k == DIR) ? Wc[1 + k] * un + p : Wc[1 + k] * un);
      if constexpr (slot > 0) sUt[slot - 1][ct] = u[k];
    });
    sWF[NV - 1][ct] = make_double2(E, (E + p) * un);
    sUn[ct] = un;
    sC[ct] = c;
    sSr[ct] = sr;
    sH[ct] = H;
  }
  __syncthreads();

  // ---- one face per thread
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
  if (f >= A.nf || t >= nA) return;
  // LDS index of window cell j (cells f-G .. f+G-1)
  const int lbase = (DIR == 0) ? tt * NC + fn : fn * TT + tt;
  constexpr int LSTEP = (DIR == 0) ? 1 : TT;
  const int ia = lbase + (G - 1) * LSTEP, ib = lbase + G * LSTEP;

  // Roe average (Sec. 5: characteristic decomposition at the face)
  const double sa = sSr[ia], sb = sSr[ib];
  const double den = sa + sb;
  const double un = (sa * sUn[ia] + sb * sUn[ib]) / den;
  double ut[NT];
  unroll<NDIM - 1>([&](auto k) { ut[k] = (sa * sUt[k][ia] + sb * sUt[k][ib]) / den; });
  double q2 = 0.0;  // |u|^2 summed in axis order
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
  // splitting speeds over the window
  double am = 0.0, a0 = 0.0, ap = 0.0;
  unroll<W>([&](auto j) {
    const int li = lbase + j * LSTEP;
    const double u = sUn[li], c = sC[li];
    if (A.splitting == TENOAA_LLF) {
      am = dmax(am, fabs(u - c));
      a0 = dmax(a0, fabs(u));
      ap = dmax(ap, fabs(u + c));
    } else {
      a0 = dmax(a0, fabs(u) + c);
    }
  });
  if (A.splitting != TENOAA_LLF) am = ap = a0;

  int64_t flin;
  {
    int64_t m[3] = {A.n[0], A.n[1], A.n[2]};
    m[DIR] = A.nf;
    const int64_t fstr[3] = {1, m[0], m[0] * m[1]};
    flin = f * fstr[DIR] + t * fstr[AX_A] + bcoord * fstr[AX_B];
  }
  uint8_t* const flag_out = A.flags ? A.flags + flin : nullptr;
  const uint8_t* const frozen = A.frozen ? A.frozen + flin : nullptr;

  double Fh[NV];  // back-projected flux, local frame
  unroll<NV>([&](auto c) { Fh[c] = 0.0; });
#pragma unroll 1
  for (int s = 0; s < NV; ++s) {
    const bool shear = (s >= 2 && s <= NV - 2);
    const bool acoustic = (s == 0 || s == NV - 1);
    const double sgn = (s == 0) ? 1.0 : -1.0;  // u - c field: +, u + c field: -
    // left eigenvector row s (local frame), the reading of the Roe eigenvectors
    double L[NV];
    if (acoustic) {
      L[0] = (s == 0) ? 0.5 * (b2 + unc) : 0.5 * (b2 - unc);
      L[1] = (s == 0) ? 0.5 * (-b1 * un - ic) : 0.5 * (-b1 * un + ic);
      unroll<NDIM - 1>([&](auto k) { L[2 + k] = 0.5 * (-b1 * ut[k]); });
      L[NV - 1] = 0.5 * b1;
    } else {
      L[0] = 1.0 - b2;
      L[1] = b1 * un;
      unroll<NDIM - 1>([&](auto k) { L[2 + k] = b1 * ut[k]; });
      L[NV - 1] = -b1;
    }
    (void)sgn;
    double mut = 0.0;
    int sl = 2;
    if constexpr (NDIM == 3) {
      mut = (s == 3) ? -ut[1] : -ut[0];
      sl = s;
    } else if constexpr (NDIM == 2) {
      mut = -ut[0];
    }
    const double alpha = (s == 0) ? am : (s == NV - 1 ? ap : a0);
    // projection of the window's state and flux on field s, then the split
    double gp[W], gm[W];
    unroll<W>([&](auto j) {
      const int li = lbase + j * LSTEP;
      double v, g;
      if (!shear) {
        const double2 w0 = sWF[0][li];
        v = L[0] * w0.x;
        g = L[0] * w0.y;
        unroll<NV - 1>([&](auto cc) {
          const double2 w = sWF[cc + 1][li];
          v = fma(L[cc + 1], w.x, v);
          g = fma(L[cc + 1], w.y, g);
        });
      } else {
        const double2 w0 = sWF[0][li];
        const double2 ws = sWF[sl][li];
        v = mut * w0.x + ws.x;
        g = mut * w0.y + ws.y;
      }
      gp[j] = 0.5 * fma(alpha, v, g);
      gm[W - 1 - j] = 0.5 * fma(-alpha, v, g);  // mirrored for the - side
#if TENOAA_CELL_BARRIER
      __builtin_amdgcn_sched_barrier(0);
#endif
    });
    uint8_t flp = 0, flm = 0;
    double hp, hm;
    if (frozen) {
      // replay recorded decisions
      flp = frozen[(int64_t)(s * 2 + 0) * A.nft];
      flm = frozen[(int64_t)(s * 2 + 1) * A.nft];
      hp = replay_recon<ORDER>(gp, flp);
      hm = replay_recon<ORDER>(gm, flm);
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
    const double fh = hp + hm;
    if (A.fh_out) A.fh_out[(int64_t)s * A.nft + flin] = fh;
    // back-projection F = sum_s R[:, s] fh_s, accumulated over s in order
    double r1 = 0.0, re = 0.0;
    if (s == 0) {
      r1 = un - cr;
      re = Hr - un * cr;
    } else if (s == NV - 1) {
      r1 = un + cr;
      re = Hr + un * cr;
    } else if (s == 1) {
      r1 = un;
      re = qq;
    } else {
      if constexpr (NDIM == 3) re = (s == 3) ? ut[1] : ut[0];
      else if constexpr (NDIM == 2) re = ut[0];
    }
    const double r0 = shear ? 0.0 : 1.0;
    if (s == 0) {
      Fh[0] = r0 * fh;
      Fh[1] = r1 * fh;
      unroll<NDIM - 1>([&](auto k) { Fh[2 + k] = ut[k] * fh; });
      Fh[NV - 1] = re * fh;
    } else {
      Fh[0] = fma(r0, fh, Fh[0]);
      Fh[1] = fma(r1, fh, Fh[1]);
      unroll<NDIM - 1>([&](auto k) {
        const double rk = shear ? (s == 2 + (int)k ? 1.0 : 0.0) : ut[k];
        Fh[2 + k] = fma(rk, fh, Fh[2 + k]);
      });
      Fh[NV - 1] = fma(re, fh, Fh[NV - 1]);
    }
  }

  if (LIMIT) {
    // Positivity limiter (reading of Hu, Adams & Shu 2013, applied in Sec. 5.3).
    const double mu = A.mu[DIR];
    const double sA = fabs(sUn[ia]) + sC[ia];
    const double sB = fabs(sUn[ib]) + sC[ib];
    const double aL = (sA >= sB) ? sA : sB;
    double FL[NV];
    unroll<NV>([&](auto c) {
      const double2 wa = sWF[c][ia], wb = sWF[c][ib];
      FL[c] = 0.5 * ((wa.y + wb.y) - aL * (wb.x - wa.x));
    });
    auto pressure = [&](const double (&X)[NV]) {
      const double rho = X[0];
      double q = 0.0;
      unroll<NDIM>([&](auto a) {
        const double ua = X[1 + Fr::slot_of_axis(decltype(a)::value)] / rho;
        q = (a == 0) ? ua * ua : q + ua * ua;
      });
      return gm1 * (X[NV - 1] - (0.5 * rho) * q);
    };
    double th_r = 1.0;
    unroll<2>([&](auto side) {
      const int li = side == 0 ? ia : ib;
      const double sg = side == 0 ? -1.0 : 1.0;
      const double r = sWF[0][li].x;
      const double rL = r + (sg * mu) * FL[0];
      const double rH = r + (sg * mu) * Fh[0];
      const double eps = rL < 1e-13 ? rL : 1e-13;
      const double th = (rH < eps) ? (rL - eps) / (rL - rH) : 1.0;
      th_r = th < th_r ? th : th_r;
    });
    double Fs[NV];
    unroll<NV>([&](auto c) { Fs[c] = (th_r < 1.0) ? FL[c] + th_r * (Fh[c] - FL[c]) : Fh[c]; });
    double th_p = 1.0;
    unroll<2>([&](auto side) {
      const int li = side == 0 ? ia : ib;
      const double sg = side == 0 ? -1.0 : 1.0;
      double X[NV];
      unroll<NV>([&](auto c) { X[c] = sWF[c][li].x + (sg * mu) * FL[c]; });
      const double pL = pressure(X);
      unroll<NV>([&](auto c) { X[c] = sWF[c][li].x + (sg * mu) * Fs[c]; });
      const double pS = pressure(X);
      const double eps = pL < 1e-13 ? pL : 1e-13;
      const double th = (pS < eps) ? (pL - eps) / (pL - pS) : 1.0;
      th_p = th < th_p ? th : th_p;
    });
    unroll<NV>([&](auto c) { Fh[c] = (th_p < 1.0) ? FL[c] + th_p * (Fs[c] - FL[c]) : Fs[c]; });
  }

  // store in axis order
  A.F[flin] = Fh[0];
  A.F[(int64_t)(NV - 1) * A.nft + flin] = Fh[NV - 1];
  unroll<NDIM>([&](auto a) {
    constexpr int slot = Fr::slot_of_axis(decltype(a)::value);
    A.F[(int64_t)(1 + a) * A.nft + flin] = Fh[1 + slot];
  });
}

// --------------------------------------------------- flux difference / RK
template <int NDIM, int MODE>
__global__ __launch_bounds__(256) void update_kernel(UpdateArgs A) {
  constexpr int NV = NDIM + 2;
  const int64_t ncell = A.n[0] * A.n[1] * A.n[2];
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ncell;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t co[3];
    co[0] = idx % A.n[0];
    co[1] = (idx / A.n[0]) % A.n[1];
    co[2] = idx / (A.n[0] * A.n[1]);
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
    const double dt = (MODE == 0) ? 0.0 : *A.dt;
    unroll<NV>([&](auto c) {
      double du = 0.0;
      unroll<NDIM>([&](auto d) {
        const double* F = A.F[d] + (int64_t)c * A.nft[d];
        du = du - (F[fr[d]] - F[fl[d]]) / A.dx[d];
      });
      const int64_t e = (int64_t)c * ncell + idx;
      if (MODE == 0) {
        A.out[e] = du;
      } else if (MODE == 1) {
        A.out[e] = A.Un[e] + dt * du;
      } else if (MODE == 2) {
        A.out[e] = 0.75 * A.Un[e] + 0.25 * A.Us[e] + (0.25 * dt) * du;
      } else {
        A.out[e] = (1.0 / 3.0) * A.Un[e] + (2.0 / 3.0) * A.Us[e] + ((2.0 / 3.0) * dt) * du;
      }
    });
  }
}

// ---------------------------------------------------------- wave speeds / dt
__global__ void init_scalars_kernel(Scalars* S) {
  if (threadIdx.x == 0) {
    S->amax_bits[0] = S->amax_bits[1] = S->amax_bits[2] = 0ull;
  }
}

template <int NDIM>
__global__ __launch_bounds__(256) void wave_speed_kernel(const double* U, int64_t ncell, double gam, Scalars* S,
                                                         int* status) {
  constexpr int NV = NDIM + 2;
  double amax[NDIM];
  unroll<NDIM>([&](auto d) { amax[d] = 0.0; });
  bool bad = false;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ncell;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double Wc[NV];
    unroll<NV>([&](auto c) { Wc[c] = U[c * ncell + idx]; });
    const double rho = Wc[0];
    double u[NDIM];
    double q2 = 0.0;
    unroll<NDIM>([&](auto k) {
      u[k] = Wc[1 + k] / rho;
      q2 = (k == 0) ? u[0] * u[0] : q2 + u[k] * u[k];
    });
    const double p = (gam - 1.0) * (Wc[NV - 1] - (0.5 * rho) * q2);
    const double c = sqrt((gam * p) / rho);
    if (!(rho > 0.0) || !(p > 0.0)) bad = true;
    unroll<NDIM>([&](auto d) { amax[d] = dmax(amax[d], fabs(u[d]) + c); });
  }
  if (bad) atomicOr(status, 1);
  __shared__ double red[NDIM][256];
  unroll<NDIM>([&](auto d) { red[d][threadIdx.x] = amax[d]; });
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      unroll<NDIM>([&](auto d) { red[d][threadIdx.x] = dmax(red[d][threadIdx.x], red[d][threadIdx.x + s]); });
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    unroll<NDIM>([&](auto d) {
      // non-negative doubles order like their bit patterns
      atomicMax(&S->amax_bits[d], (unsigned long long)__double_as_longlong(red[d][0]));
    });
  }
}

// dt = cfl / sum_d a_d/dx_d unless *dt_dev > 0; limiter mu_d = 2 S / a_d with
// S = sum_d (dt/dx_d) a_d.
__global__ void finalize_dt_kernel(Scalars* S, int ndim, double dx0, double dx1, double dx2, double cfl,
                                   double* dt_dev, double dt_fixed) {
  if (threadIdx.x != 0) return;
  const double dx[3] = {dx0, dx1, dx2};
  double a[3];
  for (int d = 0; d < 3; ++d) a[d] = __longlong_as_double((long long)S->amax_bits[d]);
  double dt = dt_fixed;
  if (!(dt > 0.0) && dt_dev) dt = *dt_dev;
  if (!(dt > 0.0)) {
    double s = a[0] / dx[0];
    for (int d = 1; d < ndim; ++d) s = s + a[d] / dx[d];
    dt = cfl / s;
  }
  if (dt_dev) *dt_dev = dt;
  S->dt = dt;
  double Ssum = (dt / dx[0]) * a[0];
  for (int d = 1; d < ndim; ++d) Ssum = Ssum + (dt / dx[d]) * a[d];
  for (int d = 0; d < 3; ++d) S->mu[d] = (d < ndim) ? (2.0 * Ssum) / a[d] : 0.0;
}

}  // namespace

// ------------------------------------------------------------ host launchers
template <int ORDER, int NDIM, int DIR, bool LIMIT>
static hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t st) {
  constexpr int TT = (NDIM == 1) ? 1 : (DIR == 0 ? TENOAA_TT_X : TENOAA_TT_YZ);
  constexpr int TN = (DIR == 0) ? TENOAA_TN_X : TENOAA_TN_YZ;
  constexpr int AX_A = (DIR == 0) ? 1 : 0;
  constexpr int AX_B = (DIR == 2) ? 1 : 2;
  dim3 grid((unsigned)((a.nf + TN - 1) / TN), (unsigned)((a.n[AX_A] + TT - 1) / TT), (unsigned)a.n[AX_B]);
  hipLaunchKernelGGL((sweep_kernel<ORDER, NDIM, DIR, TT, TN, LIMIT>), grid, dim3(TT * TN), 0, st, a);
  return hipGetLastError();
}

template <int ORDER, int NDIM, int DIR>
static hipError_t launch_sweep_o(const SweepArgs& a, bool limit, hipStream_t st) {
  return limit ? launch_sweep_t<ORDER, NDIM, DIR, true>(a, st) : launch_sweep_t<ORDER, NDIM, DIR, false>(a, st);
}

template <int ORDER>
static hipError_t launch_sweep_ord(int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st) {
  if (ndim == 1) return launch_sweep_o<ORDER, 1, 0>(a, limit, st);
  if (ndim == 2) {
    return dir == 0 ? launch_sweep_o<ORDER, 2, 0>(a, limit, st) : launch_sweep_o<ORDER, 2, 1>(a, limit, st);
  }
  if (dir == 0) return launch_sweep_o<ORDER, 3, 0>(a, limit, st);
  if (dir == 1) return launch_sweep_o<ORDER, 3, 1>(a, limit, st);
  return launch_sweep_o<ORDER, 3, 2>(a, limit, st);
}

hipError_t launch_sweep(int order, int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st) {
  return order == 10 ? launch_sweep_ord<10>(ndim, dir, a, limit, st) : launch_sweep_ord<8>(ndim, dir, a, limit, st);
}

template <int NDIM>
static hipError_t launch_update_n(int mode, const UpdateArgs& a, hipStream_t st) {
  const int64_t ncell = a.n[0] * a.n[1] * a.n[2];
  int64_t blocks = (ncell + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  dim3 g((unsigned)blocks);
  switch (mode) {
    case 0: hipLaunchKernelGGL((update_kernel<NDIM, 0>), g, dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL((update_kernel<NDIM, 1>), g, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((update_kernel<NDIM, 2>), g, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((update_kernel<NDIM, 3>), g, dim3(256), 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_update(int ndim, int mode, const UpdateArgs& a, hipStream_t st) {
  if (ndim == 1) return launch_update_n<1>(mode, a, st);
  if (ndim == 2) return launch_update_n<2>(mode, a, st);
  return launch_update_n<3>(mode, a, st);
}

hipError_t launch_wave_speeds(int ndim, const double* U, int64_t ncell, double gam, Scalars* S, int* status,
                              hipStream_t st) {
  hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, st, S);
  int64_t blocks = (ncell + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (ndim == 1) hipLaunchKernelGGL(wave_speed_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, U, ncell, gam, S, status);
  if (ndim == 2) hipLaunchKernelGGL(wave_speed_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, st, U, ncell, gam, S, status);
  if (ndim == 3) hipLaunchKernelGGL(wave_speed_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, st, U, ncell, gam, S, status);
  return hipGetLastError();
}

hipError_t launch_finalize_dt(Scalars* S, int ndim, const double* dx, double cfl, double* dt_dev, double dt_fixed,
                              hipStream_t st) {
  hipLaunchKernelGGL(finalize_dt_kernel, dim3(1), dim3(64), 0, st, S, ndim, dx[0], dx[1], dx[2], cfl, dt_dev,
                     dt_fixed);
  return hipGetLastError();
}

}  // namespace tenoaa
