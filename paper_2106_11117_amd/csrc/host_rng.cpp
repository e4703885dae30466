// Per-sample random inputs on the host: Philox4x64-10 counter-based streams,
// Box-Muller normals for the block log wave speeds, the pulse centre, and the
// per-sample step count of the CFL rule.  Built with -ffp-contract=off so
// that every operation rounds exactly once (reproducible bit for bit).
#include <cmath>

#include "host.h"

namespace lts {

// Philox4x64-10 as defined by Salmon, Moraes, Dror and Shaw ("Parallel random
// numbers: as easy as 1, 2, 3", SC'11): 10 rounds of two 64x64->128-bit
// multiplications with a Feistel-like word permutation, the key bumped by the
// Weyl constants (golden ratio and sqrt(3)-1 in 64-bit fixed point) between
// rounds.
static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const unsigned __int128 p = (unsigned __int128)a * b;
  hi = (uint64_t)(p >> 64);
  lo = (uint64_t)p;
}

void philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static inline double to_uniform(uint64_t x) {
  // ((x >> 12) + 0.5) * 2^-52: every value is exact and lies in (0, 1)
  return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

void philox_uniforms(uint64_t seed, int64_t i, int32_t level, uint64_t purpose, int n, double* u) {
  const uint64_t key[2] = {seed, 0};
  for (int j = 0; 4 * j < n; ++j) {
    const uint64_t ctr[4] = {(uint64_t)j, (uint64_t)i, (uint64_t)(uint32_t)level, purpose};
    uint64_t w[4];
    philox4x64_10(ctr, key, w);
    for (int k = 0; k < 4 && 4 * j + k < n; ++k) u[4 * j + k] = to_uniform(w[k]);
  }
}

std::string gen_samples(uint64_t seed, int32_t sample_level, int64_t first_index, int32_t n,
                        const lts_sample_rule& rule, double h_mesh, double* g, double* kappa,
                        double* x0, int32_t* n_steps, double* dt) {
  const int nb = rule.n_blocks;
  if (nb < 2 || nb > 255 || (nb % 2)) return "rule.n_blocks must be even and in 2..254";
  if (n < 0 || first_index < 0) return "n and first_index must be >= 0";
  if (sample_level < 0) return "sample_level must be >= 0";
  if (!(rule.sigma >= 0.0) || !(rule.T > 0.0) || !(rule.cfl > 0.0) || !(h_mesh > 0.0))
    return "sigma >= 0, T > 0, cfl > 0 and h_mesh > 0 required";
  if (!(rule.width > 0.0)) return "width must be > 0";
  const double pi2 = 2.0 * M_PI;
  double u[256], z[256];
  for (int s = 0; s < n; ++s) {
    const int64_t i = first_index + s;
    philox_uniforms(seed, i, sample_level, 0, nb, u);
    for (int k = 0; k < nb; k += 2) {
      const double r = std::sqrt(-2.0 * std::log(u[k]));
      const double t = pi2 * u[k + 1];
      z[k] = r * std::cos(t);
      z[k + 1] = r * std::sin(t);
    }
    double cmax = 0.0;
    for (int b = 0; b < nb; ++b) {
      const double gb = rule.sigma * z[b];
      if (g) g[(size_t)s * nb + b] = gb;
      if (kappa) kappa[(size_t)s * nb + b] = std::exp(2.0 * gb);
      const double cb = std::exp(gb);
      if (b == 0 || cb > cmax) cmax = cb;
    }
    double up[2];
    philox_uniforms(seed, i, sample_level, 1, 2, up);
    if (x0) {
      x0[2 * s] = rule.px_lo + (rule.px_hi - rule.px_lo) * up[0];
      x0[2 * s + 1] = rule.py_lo + (rule.py_hi - rule.py_lo) * up[1];
    }
    const double ns = std::ceil((rule.T * cmax) / (rule.cfl * h_mesh));
    if (!(ns >= 1.0) || ns > 2.0e9) return "step count out of range";
    if (n_steps) n_steps[s] = (int32_t)ns;
    if (dt) dt[s] = rule.T / ns;
  }
  return "";
}

// ---------------------------------------------------------------------------
// Stabilized Chebyshev constants (Sec. 3.3): delta = 1 + nu/p^2,
// omega = 2 T_p'(delta)/T_p(delta), beta_k = T_{k-1}/T_{k+1},
// beta_{k+1/2} = T_k/T_{k+1} at delta, with T_p' = p U_{p-1}.  Evaluated by the
// three-term recurrences in extended precision.
void cheb_constants(int p, double nu, double& delta, double& omega, std::vector<double>& beta,
                    std::vector<double>& beta_half) {
  const long double d = 1.0L + (long double)nu / ((long double)p * (long double)p);
  std::vector<long double> T(p + 2), U(p + 1);
  T[0] = 1.0L;
  T[1] = d;
  for (int k = 2; k <= p + 1; ++k) T[k] = 2.0L * d * T[k - 1] - T[k - 2];
  U[0] = 1.0L;
  if (p >= 1) U[1] = 2.0L * d;
  for (int k = 2; k <= p; ++k) U[k] = 2.0L * d * U[k - 1] - U[k - 2];
  delta = (double)d;
  omega = (double)(2.0L * ((long double)p * U[p - 1]) / T[p]);
  beta.assign(p, 0.0);
  beta_half.assign(p, 0.0);
  for (int k = 1; k < p; ++k) {
    beta[k] = (double)(T[k - 1] / T[k + 1]);
    beta_half[k] = (double)(T[k] / T[k + 1]);
  }
}

void step_coefficients(const HostLevel& L, double dt, double* out) {
  const int p = L.p;
  const double c1 = 0.5 * (dt / p) * (dt / p) * (2.0 * p * p / (L.omega * L.delta));
  out[1] = c1;
  // a_m: d_m = a_m w on a DOF that neither is in P nor touches P.  The scalar
  // recurrence runs in extended precision (its binary64 evaluation loses up to
  // ~1e-14 relative for p = 64); a_p = -dt^2/2 up to the rounding of the constants.
  long double a_prev = 0.0L, a = -(long double)c1;
  for (int m = 1; m < p; ++m) {
    const double c2 = (dt / p) * (dt / p) * (2.0 * p * p / L.omega) * L.beta_half[m];
    out[1 + m] = c2;
    const long double an = (1.0L + L.beta[m]) * a - (long double)L.beta[m] * a_prev - c2;
    a_prev = a;
    a = an;
  }
  out[0] = (double)a;
}

}  // namespace lts
