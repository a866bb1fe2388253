// sampling.cpp -- the MPPI control perturbations of Sec. IV-A drawn from a
// seed, on the host in FP64.
//
// The perturbation of rollout k at step n of MPPI iteration i is sigma * z
// with z standard normal. The uniforms come from the counter-based generator
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011), keyed by the seed, with counter
// (n / 4, k, i, 0); each of its four 64-bit outputs w gives a 53-bit uniform
// from its top bits. The normals come from the Box-Muller transform (Box and
// Muller 1958): the pair of outputs (w0, w1) gives steps 4j and 4j+1, the
// pair (w2, w3) steps 4j+2 and 4j+3, as r cos t and r sin t with
// r = sqrt(-2 ln u_a), u_a = (top53(w_a) + 1) 2^-53 in (0, 1], and
// t = 2 pi u_b, u_b = top53(w_b) 2^-53 in [0, 1). Every value is a pure
// function of (seed, i, k, n), so any subset of rollouts or steps is drawn
// identically wherever and in whatever order it is drawn.
#include <cmath>
#include <cstdint>

#include "host_common.h"

namespace vpm {
namespace {

// Philox4x64 round multipliers and Weyl key increments (Salmon et al., Table 2).
constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ULL;
constexpr uint64_t kMul1 = 0xCA5A826395121157ULL;
constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73BULL;

inline void mul_hi_lo(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
  const unsigned __int128 p = static_cast<unsigned __int128>(a) * b;
  hi = static_cast<uint64_t>(p >> 64);
  lo = static_cast<uint64_t>(p);
}

// Ten rounds of the Philox S-box network on counter c with key k.
void philox4x64_10(const uint64_t c_in[4], const uint64_t k_in[2], uint64_t out[4]) {
  uint64_t c0 = c_in[0], c1 = c_in[1], c2 = c_in[2], c3 = c_in[3];
  uint64_t k0 = k_in[0], k1 = k_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += kWeyl0;
      k1 += kWeyl1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul_hi_lo(kMul0, c0, hi0, lo0);
    mul_hi_lo(kMul1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

constexpr double kTwoPi = 6.283185307179586;       // the double nearest 2 pi
constexpr double kTwoM53 = 1.0 / 9007199254740992.0;  // 2^-53

}  // namespace

void sample_eps(uint64_t seed, int iteration, int K, int H, double sigma, double *out) {
  const uint64_t key[2] = {seed, 0};
  for (int k = 0; k < K; ++k) {
    double *row = out + static_cast<size_t>(k) * H;
    for (int j = 0; 4 * j < H; ++j) {
      const uint64_t ctr[4] = {static_cast<uint64_t>(j), static_cast<uint64_t>(k),
                               static_cast<uint64_t>(iteration), 0};
      uint64_t w[4];
      philox4x64_10(ctr, key, w);
      for (int p = 0; p < 2; ++p) {
        const double ua = static_cast<double>((w[2 * p] >> 11) + 1) * kTwoM53;
        const double ub = static_cast<double>(w[2 * p + 1] >> 11) * kTwoM53;
        const double r = std::sqrt(-2.0 * std::log(ua));
        const double t = kTwoPi * ub;
        const int n = 4 * j + 2 * p;
        if (n < H) row[n] = sigma * (r * std::cos(t));
        if (n + 1 < H) row[n + 1] = sigma * (r * std::sin(t));
      }
    }
  }
}

}  // namespace vpm

extern "C" {

VPM_API int vpm_sample_eps(uint64_t seed, int32_t iteration, int32_t K, int32_t H,
                           double sigma, double *out) {
  if (K < 1 || H < 1 || iteration < 0)
    return vpm::fail(VPM_EINVAL, "K and H must be >= 1 and iteration >= 0");
  if (!(std::isfinite(sigma) && sigma >= 0.0))
    return vpm::fail(VPM_EINVAL, "sigma must be finite and >= 0");
  if (!out) return vpm::fail(VPM_EINVAL, "out is NULL");
  vpm::sample_eps(seed, iteration, K, H, sigma, out);
  return VPM_OK;
}

}  // extern "C"
