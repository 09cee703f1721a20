// Drives every entry point of the oracle (oracle/tenoaa_oracle.cpp, compiled
// into this program) over small grids of every dimension, boundary type,
// order, splitting and limiter setting, so that a build with the address and
// undefined-behaviour sanitizers checks its indexing and arithmetic.  Test
// infrastructure: tests/test_oracle_sanitize.py builds and runs it on the CPU.
#include "../oracle/tenoaa_oracle.cpp"

#include <cstdio>
#include <vector>

namespace {

// Smooth positive state with a jump: rho, p in [0.5, 2.5], velocities in [-0.5, 0.5].
std::vector<double> make_state(int ndim, const int64_t n[3], double gam, unsigned seed) {
  const int nv = ndim + 2;
  const int64_t nc = n[0] * n[1] * n[2];
  std::vector<double> U(nv * nc);
  for (int64_t k = 0; k < n[2]; ++k)
    for (int64_t j = 0; j < n[1]; ++j)
      for (int64_t i = 0; i < n[0]; ++i) {
        const int64_t c = i + n[0] * (j + n[1] * k);
        const double x = (i + 0.5) / n[0], y = (j + 0.5) / n[1], z = (k + 0.5) / n[2];
        const double ph = 0.37 * seed;
        double rho = 1.5 + 0.5 * std::sin(6.283 * x + ph) * std::cos(6.283 * y) + (x > 0.6 ? 0.4 : 0.0);
        double p = 1.5 + 0.5 * std::cos(6.283 * (x + z) + ph) - (y > 0.55 ? 0.3 : 0.0);
        double u[3] = {0.4 * std::sin(6.283 * y + ph), 0.3 * std::cos(6.283 * z), 0.2 * std::sin(6.283 * x)};
        double q = 0.0;
        U[c] = rho;
        for (int d = 0; d < ndim; ++d) {
          U[(1 + d) * nc + c] = rho * u[d];
          q += u[d] * u[d];
        }
        U[(nv - 1) * nc + c] = p / (gam - 1.0) + 0.5 * rho * q;
      }
  return U;
}

int failures = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

}  // namespace

int main() {
  const double gam = 1.4;
  const int orders[3] = {8, 10, 12};
  // boundary kinds per case: periodic, outflow, symmetry, no-slip, Dirichlet, inflow
  for (int ndim = 1; ndim <= 3; ++ndim) {
    const int nv = ndim + 2;
    int64_t n[3] = {1, 1, 1};
    const int64_t sizes[3] = {ndim == 1 ? 24 : (ndim == 2 ? 14 : 8), ndim == 2 ? 13 : 9, 7};
    for (int d = 0; d < ndim; ++d) n[d] = sizes[d];
    const int64_t nc = n[0] * n[1] * n[2];
    std::vector<double> U = make_state(ndim, n, gam, ndim);
    for (int bc = 0; bc <= 5; ++bc) {
      for (int oi = 0; oi < 3; ++oi) {
        const int order = orders[oi];
        const int G = order / 2;
        bool fits = true;
        for (int d = 0; d < ndim; ++d) fits = fits && n[d] >= G;
        if (!fits) continue;
        or_grid g{};
        g.ndim = ndim;
        g.bc_sets = 1;
        std::vector<std::vector<double>> bv;
        for (int d = 0; d < 3; ++d) {
          g.n[d] = n[d];
          g.dx[d] = d < ndim ? 1.0 / n[d] : 1.0;
          g.bc_lo[d] = d < ndim ? bc : 0;
          g.bc_hi[d] = d < ndim ? (bc == 0 ? 0 : 1) : 0;  // mixed: the high side is outflow
          if (d < ndim && (bc == 4 || bc == 5)) {
            int64_t plane = 1;
            for (int e = 0; e < ndim; ++e)
              if (e != d) plane *= n[e];
            const int layers = bc == 5 ? G : 1;
            std::vector<double> v((size_t)layers * nv * plane);
            for (int l = 0; l < layers; ++l)
              for (int c = 0; c < nv; ++c)
                for (int64_t q = 0; q < plane; ++q)
                  v[((size_t)l * nv + c) * plane + q] = (c == 0 || c == nv - 1) ? 1.0 + 0.01 * l : 0.1;
            bv.push_back(v);
            g.bc_values[d][0] = bv.back().data();
          }
        }
        for (int split = 0; split <= 2; ++split) {
          for (int pos = 0; pos <= 1; ++pos) {
            std::vector<double> dU(nv * nc);
            const int64_t nflag = or_flags_size(&g);
            std::vector<uint8_t> fl(nflag);
            std::vector<double> mg(nflag);
            const double dt = or_dt(&g, gam, 0.4, U.data());
            check(or_rhs(&g, order, split, pos, gam, U.data(), dU.data(), pos ? dt : 0.0, fl.data(), mg.data()) == 0,
                  "or_rhs");
            std::vector<int64_t> cells = {0, nc / 2, nc - 1};
            std::vector<double> out(cells.size() * nv);
            double amax[3];
            or_wave_speeds(&g, gam, U.data(), amax);
            check(or_rhs_cells(&g, order, split, pos, gam, U.data(), pos ? dt : 0.0, amax, (int64_t)cells.size(),
                               cells.data(), out.data()) == 0,
                  "or_rhs_cells");
            std::vector<double> V(nv * nc), jv(nv * nc), r(nv * nc);
            for (int64_t q = 0; q < nv * nc; ++q) V[q] = std::sin(0.1 * q);
            check(or_rhs_jvp(&g, order, split, gam, U.data(), V.data(), fl.data(), r.data(), jv.data()) == 0,
                  "or_rhs_jvp");
            std::vector<double> Us = U;
            double dts = 0.0;
            std::vector<uint8_t> fl3(3 * nflag);
            std::vector<double> mg3(3 * nflag);
            check(or_step(&g, order, split, pos, gam, 0.4, Us.data(), &dts, fl3.data(), mg3.data()) == 0, "or_step");
            check(or_step_jvp(&g, order, split, pos, gam, U.data(), V.data(), dts, fl3.data(), jv.data()) == 0,
                  "or_step_jvp");
          }
        }
      }
    }
  }
  for (int oi = 0; oi < 3; ++oi) {
    const int64_t n = 40;
    std::vector<double> u(n), du(n);
    std::vector<uint8_t> f(n), f3(3 * n);
    for (int64_t i = 0; i < n; ++i) u[i] = std::exp(-std::pow((i - 20.0) / 4.0, 2)) + (i > 30 ? 1.0 : 0.0);
    check(or_advect_rhs(orders[oi], n, 1.0 / n, u.data(), du.data(), f.data()) == 0, "or_advect_rhs");
    check(or_advect_step(orders[oi], n, 1.0 / n, 0.2 / n, u.data(), f3.data()) == 0, "or_advect_step");
  }
  for (int k = 0; k <= 6; ++k) {
    double fv[12];
    for (int j = 0; j < 12; ++j) fv[j] = std::sin(0.7 * j) + (j > 6 ? 1.0 : 0.0);
    (void)or_beta(k, fv);
    (void)or_candidate_flux(k, fv + 5);
  }
  for (int order : orders) {
    double fv[12];
    for (int j = 0; j < 12; ++j) fv[j] = j * j * 0.01;
    uint8_t fl;
    double mg;
    (void)or_teno(order, fv, &fl, &mg);
  }
  std::printf("oracle sanitize driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
