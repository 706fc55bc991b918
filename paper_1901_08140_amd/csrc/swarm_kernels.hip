// Device code of the MI355X electron-swarm library: rate-table build, the persistent
// per-electron null-collision kernels (FP64 and FP32-mixed), and the deterministic tally
// reductions.  Method: "Betaboltz: a Monte-Carlo simulation tool for gas scattering
// processes" (arXiv 1901.08140), section "Theoretical framework" (eqs. freetime,
// frequency, random_time, null_fraction, delta_energy_ela, delta_energy_ine), section
// "Extension of the cross-section tables" and section "Determination of swarm attributes".
//
// Layout of the work: one electron per lane, its whole state in registers; the total
// rate table of the instance is staged in LDS as (F[g], F[g+1]-F[g]) pairs on an octave
// grid so that the per-trial null test is one LDS read and one FMA; the per-channel
// running sums are read from global memory (L2) only at real collisions.  Random numbers
// come from Philox4x32-10 keyed by the run seed with counter (block, stream tag, electron
// id), so any electron's history is independent of scheduling.
//
// Built with -ffp-contract=off: every fused multiply-add below is written explicitly, so
// the arithmetic of an electron is the same in every launch shape.

#include <hip/hip_runtime.h>

#include <math.h>

#include "swarm_internal.hpp"
#include "unit_log.hpp"

namespace swarm_impl {
namespace {

constexpr double kQe = 1.602176634e-19;     // C
constexpr double kMe = 9.1093837015e-31;    // kg
constexpr double kAmu = 1.66053906660e-27;  // kg
constexpr double kPi = 3.14159265358979323846;
constexpr double kHartreeEV = 27.211386245988;   // Hartree energy in eV (CODATA 2018)
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kKb = 1.380649e-23;         // J/K
constexpr double kC = 299792458.0;           // m/s

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplications
// (v_mad_u64_u32 on CDNA) and xors; the key schedule adds the Weyl constants per round.
// ---------------------------------------------------------------------------------------
struct W4 { uint32_t x, y, z, w; };

// a ^ b ^ k in one gfx950 three-input bitwise operation (truth table 0x96 = odd parity)
__device__ __forceinline__ uint32_t xor3_k(uint32_t a, uint32_t b, uint32_t k) {
  return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// Rounds 2..10 of Philox4x32-10 (the first round is done by the caller); k0, k1 are the
// keys of round 2.
__device__ __forceinline__ W4 philox_rounds9(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 1; i < 10; ++i) {
    const uint64_t p0 = static_cast<uint64_t>(c0) * 0xD2511F53u;
    const uint64_t p1 = static_cast<uint64_t>(c2) * 0xCD9E8D57u;
    const uint32_t n0 = xor3_k(static_cast<uint32_t>(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3_k(static_cast<uint32_t>(p0 >> 32), c3, k1);
    c1 = static_cast<uint32_t>(p1);
    c3 = static_cast<uint32_t>(p0);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ W4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                      uint32_t k0, uint32_t k1) {
  const uint64_t p0 = static_cast<uint64_t>(c0) * 0xD2511F53u;
  const uint64_t p1 = static_cast<uint64_t>(c2) * 0xCD9E8D57u;
  const uint32_t n0 = xor3_k(static_cast<uint32_t>(p1 >> 32), c1, k0);
  const uint32_t n2 = xor3_k(static_cast<uint32_t>(p0 >> 32), c3, k1);
  return philox_rounds9(n0, static_cast<uint32_t>(p1), n2, static_cast<uint32_t>(p0),
                        k0 + 0x9E3779B9u, k1 + 0xBB67AE85u);
}

enum : uint32_t { TAG_TRIAL_HI = 0, TAG_TRIAL_LO = 1, TAG_SCAT_HI = 2, TAG_SCAT_LO = 3,
                  TAG_INIT_HI = 4, TAG_INIT_LO = 5, TAG_CHILD = 6, TAG_THERMAL_HI = 7,
                  TAG_THERMAL_LO = 8 };

struct Key { uint32_t k0, k1; };

__device__ __forceinline__ W4 draw(Key key, uint64_t id, uint32_t tag, uint32_t block) {
  return philox10(block, tag, static_cast<uint32_t>(id), static_cast<uint32_t>(id >> 32), key.k0, key.k1);
}

// The first Philox round of a trial block: counter word 2 (the electron id's low half)
// is the same for every block of the electron, so its product is precomputed once per
// electron (a = hi(M1 id_lo) ^ tag ^ k0, b = lo(M1 id_lo)); only M0 * block is new.
struct TrialPre { uint32_t a, b, idhi; };

__device__ __forceinline__ TrialPre trial_pre(Key key, uint64_t id, uint32_t tag) {
  const uint64_t p1 = static_cast<uint64_t>(static_cast<uint32_t>(id)) * 0xCD9E8D57u;
  return {static_cast<uint32_t>(p1 >> 32) ^ tag ^ key.k0, static_cast<uint32_t>(p1),
          static_cast<uint32_t>(id >> 32)};
}

__device__ __forceinline__ W4 draw_trial(Key key, TrialPre pre, uint32_t block) {
  const uint64_t p0 = static_cast<uint64_t>(block) * 0xD2511F53u;
  const uint32_t n2 = xor3_k(static_cast<uint32_t>(p0 >> 32), pre.idhi, key.k1);
  return philox_rounds9(pre.a, pre.b, n2, static_cast<uint32_t>(p0), key.k0 + 0x9E3779B9u,
                        key.k1 + 0xBB67AE85u);
}

// Uniforms on [0,1).  FP64: 53 bits, the HI word on top of the upper 21 bits of the LO
// word (exact: both parts are integers scaled by powers of two).  FP32: the top 24 bits of
// the HI word, i.e. the FP64 uniform truncated.
__device__ __forceinline__ double uni(uint32_t hi, uint32_t lo, double) {
  return fma(static_cast<double>(hi), 0x1.0p-32, static_cast<double>(lo >> 11) * 0x1.0p-53);
}
__device__ __forceinline__ float uni(uint32_t hi, uint32_t, float) {
  return static_cast<float>(hi >> 8) * 0x1.0p-24f;
}
// 1 - u for the FP64 uniform of (hi, lo), formed directly: 1 - lo' 2^-53 and then minus
// hi 2^-32 are both exact, so this equals 1 - uni(hi, lo) bit for bit, one step shorter.
__device__ __forceinline__ double one_minus_uni(uint32_t hi, uint32_t lo) {
  return fma(static_cast<double>(hi), -0x1.0p-32, fma(static_cast<double>(lo >> 11), -0x1.0p-53, 1.0));
}

// Flight-time increment -ln(1-u)/nu' (eq. random_time) in FP64, cT = 1/nu': 1-u is exact,
// and its logarithm comes from the table-driven unit_log (about 20 instructions where the
// library logarithm takes about 85), with the table staged in LDS.  The FP32 trial forms
// its own from the 24-bit word (one_trial).
__device__ __forceinline__ double flight(double one_minus_u, double cT, const double* __restrict__ logtab) {
  return -unit_log(one_minus_u, logtab) * cT;
}

__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }

// sin/cos of 2 pi u for u in [0,1): FP32 through the hardware unit (input in revolutions);
// FP64 as sin/cos of pi (2u), whose argument reduction is exact, so none of the general
// large-argument reduction is needed.
__device__ __forceinline__ void sincos_rev(float u, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(u);
  *c = __builtin_amdgcn_cosf(u);
}
__device__ __forceinline__ void sincos_rev(double u, double* s, double* c) {
  sincospi(2.0 * u, s, c);
}

// Anisotropic scattering (section "Theoretical framework", eqs. collision_angle and
// collision_angle_xi).  For molecules xi solves sigma_mt/sigma_el = (1 - xi)/(2 xi^2)
// ((1 + xi) ln((1 + xi)/(1 - xi)) - 2 xi); the right side falls from 1 at xi = 0 to 0 at
// xi = 1, so bisection on (0, 1) in binary64 converges to it.
__device__ double mt_over_el_of_xi(double xi) {
  if (xi <= 0.0) return 1.0;
  return (1.0 - xi) / (2.0 * xi * xi) * ((1.0 + xi) * log((1.0 + xi) / (1.0 - xi)) - 2.0 * xi);
}
__device__ double xi_of_ratio(double r) {
  if (r >= 1.0) return 0.0;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (mt_over_el_of_xi(mid) > r) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// cos(theta) from the uniform u: screened Coulomb with the energy before the collision in
// Hartree units, or the xi form.
__device__ __forceinline__ double scatter_cos(int scat, double xi, double eps, double u) {
  if (scat == SWARM_SCATTER_SCREENED_COULOMB) {
    const double e = eps / kHartreeEV;
    return 1.0 - 2.0 * u / (1.0 + 8.0 * e * (1.0 - u));
  }
  return 1.0 - 2.0 * u * (1.0 - xi) / (1.0 + xi * (1.0 - 2.0 * u));
}
// (FP32: the quotient through the hardware reciprocal, within an ulp of the division)
__device__ __forceinline__ float scatter_cos(int scat, float xi, float eps, float u) {
  if (scat == SWARM_SCATTER_SCREENED_COULOMB) {
    const float e = eps * static_cast<float>(1.0 / kHartreeEV);
    return 1.0f - 2.0f * u * __builtin_amdgcn_rcpf(1.0f + 8.0f * e * (1.0f - u));
  }
  return 1.0f - 2.0f * u * (1.0f - xi) * __builtin_amdgcn_rcpf(1.0f + xi * (1.0f - 2.0f * u));
}

// The unit vector at polar angle theta (cos given) and azimuth 2 pi u_phi about the unit
// vector d = (a, b, c): the rotation of direction cosines with s = sqrt(a^2 + b^2),
//   (a cos + sin (a c cos phi - b sin phi)/s, b cos + sin (b c cos phi + a sin phi)/s,
//    c cos - s sin cos phi), and (sin cos phi, sin sin phi, c cos) when d is along z.
template <typename R>
__device__ __forceinline__ void rotate_dir(R a, R b, R c, R cos_t, R u_phi, R* nx, R* ny, R* nz) {
  const R sin_t = sqrt_(fmax(R(0), (R(1) - cos_t) * (R(1) + cos_t)));
  R sp, cp;
  sincos_rev(u_phi, &sp, &cp);
  const R s = sqrt_(a * a + b * b);
  if (s > R(0)) {
    *nx = a * cos_t + sin_t * (a * c * cp - b * sp) / s;
    *ny = b * cos_t + sin_t * (b * c * cp + a * sp) / s;
    *nz = c * cos_t - s * sin_t * cp;
  } else {
    *nx = sin_t * cp;
    *ny = sin_t * sp;
    *nz = c * cos_t;
  }
}
// FP32: 1/s from the hardware reciprocal square root and s = s^2 (1/s), instead of a square
// root and two divisions
template <>
__device__ __forceinline__ void rotate_dir<float>(float a, float b, float c, float cos_t, float u_phi,
                                                  float* nx, float* ny, float* nz) {
  const float sin_t = sqrt_(fmaxf(0.0f, (1.0f - cos_t) * (1.0f + cos_t)));
  float sp, cp;
  sincos_rev(u_phi, &sp, &cp);
  const float s2 = fmaf(b, b, a * a);
  if (s2 > 0.0f) {
    const float inv = rsqrt_(s2);
    const float k = sin_t * inv;
    *nx = fmaf(a, cos_t, k * (a * c * cp - b * sp));
    *ny = fmaf(b, cos_t, k * (b * c * cp + a * sp));
    *nz = fmaf(c, cos_t, -(s2 * inv) * sin_t * cp);
  } else {
    *nx = sin_t * cp;
    *ny = sin_t * sp;
    *nz = c * cos_t;
  }
}

// Isotropic unit vector: cos(Theta) = 1 - 2u, Phi = 2 pi u'.  With u a multiple of the
// precision's 2^-24 or 2^-53 below 1, 1 - 2u, 1 - ct = 2u and 1 + ct are exact and not
// negative, so one FMA forms ct and sin(Theta) needs no clamp.
template <typename R>
__device__ __forceinline__ void iso_dir(R uc, R up, R* nx, R* ny, R* nz) {
  const R ct = fma_(R(-2), uc, R(1));
  const R st = sqrt_((R(1) - ct) * (R(1) + ct));
  R s, c;
  sincos_rev(up, &s, &c);
  *nx = st * c;
  *ny = st * s;
  *nz = ct;
}

// The same from the scattering word in FP32: 1 - 2u = 1 - (w >> 8) 2^-23 by one FMA, exact
// as above, so the result equals iso_dir's to the bit.
__device__ __forceinline__ void iso_dir_u24(uint32_t w, float up, float* nx, float* ny, float* nz) {
  const float ct = fmaf(static_cast<float>(w >> 8), -0x1.0p-23f, 1.0f);
  const float st = sqrt_((1.0f - ct) * (1.0f + ct));
  float s, c;
  sincos_rev(up, &s, &c);
  *nx = st * c;
  *ny = st * s;
  *nz = ct;
}

template <typename R> struct Pair;
template <> struct Pair<float> { using T = float2; };
template <> struct Pair<double> { using T = double2; };

// Interpolated value F[g] + w (F[g+1] - F[g]) from a (F, dF) pair.
__device__ __forceinline__ float lerp_pair(float2 q, float w) { return fmaf(w, q.y, q.x); }
__device__ __forceinline__ double lerp_pair(double2 q, double w) { return q.x + w * q.y; }

// =======================================================================================
// Table build (create time): raw tables -> extension -> rates on the octave grid ->
// running sums over channels -> pairs for the kernels; then the trial frequency and the
// field constants.  One thread per grid node.
// =======================================================================================

// Cross-section of raw channel c at eps with the extension rules of section "Extension of
// the cross-section tables": elastic constant to the left of the table; inelastic zero
// below threshold, with a (threshold, 0) point in front of a table that starts above it;
// to the right the power law A eps^K through the last two points (zero if either is 0);
// linear interpolation between points.
__device__ double sigma_ext(const InstanceDesc& d, int c, double eps) {
  const double* e = d.raw_e + d.raw_off[c];
  const double* s = d.raw_s + d.raw_off[c];
  const int n = d.raw_n[c];
  const int kind = d.raw_kind[c];
  const double thr = d.raw_thr[c];
  bool lead = false;                       // virtual first point (thr, 0)
  if (kind != SWARM_ELASTIC) {
    if (eps < thr) return 0.0;
    lead = e[0] > thr;
  }
  const double e_first = lead ? thr : e[0];
  const double s_first = lead ? 0.0 : s[0];
  if (eps <= e_first) return s_first;
  if (eps > e[n - 1]) {
    const double e1 = e[n - 2], e2 = e[n - 1], s1 = s[n - 2], s2 = s[n - 1];
    if (!(s1 > 0.0) || !(s2 > 0.0)) return 0.0;
    const double K = log(s2 / s1) / log(e2 / e1);
    const double A = s2 / pow(e2, K);
    return A * pow(eps, K);
  }
  if (lead && eps <= e[0]) {
    const double t = (eps - thr) / (e[0] - thr);
    return 0.0 + (s[0] - 0.0) * t;
  }
  // smallest i >= 1 with e[i] >= eps (binary search; e[0] < eps <= e[n-1])
  int lo = 1, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (e[mid] < eps) lo = mid + 1; else hi = mid;
  }
  const double t = (eps - e[lo - 1]) / (e[lo] - e[lo - 1]);
  return s[lo - 1] + (s[lo] - s[lo - 1]) * t;
}

__global__ void k_build_rates(InstanceDesc* desc) {
  const InstanceDesc& d = *desc;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.G) return;
  const int P = 1 << d.p_log2;
  const int o = g / P, i = g % P;
  const double eps = ldexp(1.0 + static_cast<double>(i) / P, d.emin + o);
  const double ej = eps * kQe;
  const double speed = d.relativistic ? sqrt(2.0 * ej / kMe * (1.0 + ej / (2.0 * kMe * kC * kC))) / (1.0 + ej / (kMe * kC * kC))
                                      : sqrt(2.0 * ej / kMe);
  double acc = 0.0;
  for (int c = 0; c < d.nc; ++c) {
    const int comp = d.raw_comp[c];
    const double dens = d.comp_frac[comp] * d.N;
    // eq. frequency: nu_c = n_k sigma_c(eps) v, eps in joule, v = sqrt(2 eps / m); the
    // relativistic mover takes the true speed |u|/gamma, |u| = sqrt(2 eps/m (1 + eps/(2 m c^2)))
    // the proper speed and gamma = 1 + eps/(m c^2)
    acc += dens * sigma_ext(d, c, eps) * speed;
    d.cum_cm[static_cast<size_t>(c) * d.G + g] = acc;
  }
  d.nodes[g] = eps;
}

// Pairs (F[g], F[g+1]-F[g]) of every running sum (node major) and of the total rate.  The
// running sums are padded like the LDS table of the total rate: row 0 holds (F[0], 0) for
// energies below the grid, row g+1 node g, and row G (the top node, difference zero) serves
// energies at or above the top, so the padded index of a trial selects the row directly.
// The FP32 differences are stored times 2^-(23-p), because the FP32 weight is taken as the
// integer of the low 23-p mantissa bits (see lds_rate): an exact power-of-two scale, so every
// product w (F[g+1]-F[g]) keeps its value to the bit.
__global__ void k_build_pairs(InstanceDesc* desc) {
  const InstanceDesc& d = *desc;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(d.G) * d.nc) return;
  const int g = static_cast<int>(idx / d.nc), c = static_cast<int>(idx % d.nc);
  const double* F = d.cum_cm + static_cast<size_t>(c) * d.G;
  const double f0 = F[g];
  const double df = g + 1 < d.G ? F[g + 1] - f0 : 0.0;
  const float df32 = static_cast<float>(df) * ldexpf(1.0f, d.p_log2 - 23);
  d.cum64[idx + d.nc] = make_double2(f0, df);
  d.cum32[idx + d.nc] = make_float2(static_cast<float>(f0), df32);
  if (g == 0) {
    d.cum64[c] = make_double2(f0, 0.0);
    d.cum32[c] = make_float2(static_cast<float>(f0), 0.0f);
  }
  if (c == d.nc - 1) {
    d.nu64[g] = make_double2(f0, df);
    d.nu32[g] = make_float2(static_cast<float>(f0), df32);
  }
}

// Trial frequency (maximum of the total rate, raised by 2^-20 so that the interpolated
// rate never exceeds it: the paper's LazyTrialFrequency), channel constants and field
// constants.  One work-group; fixed-order reduction.
__global__ void k_build_constants(InstanceDesc* desc) {
  InstanceDesc& d = *desc;
  __shared__ double smax[256];
  __shared__ int szero[256];
  const double* F = d.cum_cm + static_cast<size_t>(d.nc - 1) * d.G;
  double m = 0.0;
  int zero = 0;
  for (int g = threadIdx.x; g < d.G; g += blockDim.x) {
    m = fmax(m, F[g]);
    zero |= !(F[g] > 0.0);
  }
  smax[threadIdx.x] = m;
  szero[threadIdx.x] = zero;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      szero[threadIdx.x] |= szero[threadIdx.x + s];
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < d.nc; c += blockDim.x) {
    const int comp = d.raw_comp[c];
    const double M = d.comp_mass_amu[comp] * kAmu;
    const double mm = kMe;
    ChannelDev ch;
    ch.kind = d.raw_kind[c];
    ch.comp = comp;
    ch.thr = d.raw_thr[c];
    ch.onset = ch.thr * ((mm + M) / M);
    ch.c_ela = 2.0 * mm * M / ((mm + M) * (mm + M));
    ch.c_M = M / (mm + M);
    ch.c_mM = (mm + M) / M;
    ch.thr_f = static_cast<float>(ch.thr);
    ch.c_ela_f = static_cast<float>(ch.c_ela);
    ch.c_M_f = static_cast<float>(ch.c_M);
    ch.c_mM_f = static_cast<float>(ch.c_mM);
    ch.scat = d.comp_scat[comp];
    ch.xi = ch.scat == SWARM_SCATTER_CONSTANT_XI ? xi_of_ratio(d.comp_ratio[comp]) : 0.0;
    ch.xi_f = static_cast<float>(ch.xi);
    d.chan[c] = ch;
    ThermalChannel th;
    th.mass = M;
    th.sigma = sqrt(kKb * d.T_K / M);
    th.loss = (ch.kind == SWARM_EXCITATION || ch.kind == SWARM_IONIZATION) ? 2.0 * (ch.thr * kQe) / (mm + M) * (M / mm)
                                                                           : 0.0;
    th.cM = M / (mm + M);
    d.chan_th[c] = th;
  }
  if (threadIdx.x == 0) {
    const double numax = smax[0];
    d.numax = numax;
    double nup = (1.0 + 0x1.0p-20) * numax;
    int ok = szero[0] ? -1 : 1;
    if (d.user_majorant > 0.0) {
      if (d.user_majorant < numax) ok = -2;
      nup = d.user_majorant;
    }
    d.built_ok = ok;
    d.majorant = nup;
    d.inv_majorant = 1.0 / nup;
    d.majorant_f = static_cast<float>(nup);
    d.cT_f = static_cast<float>(kLn2 / nup);
    d.c_eps = 0.5 * kMe / kQe;
    d.c_speed = sqrt(2.0 * kQe / kMe);
    // (relativistic mover: the proper speed gamma |v|)
    d.speed0 = sqrt(2.0 * d.eps0 * kQe / kMe * (d.relativistic ? 1.0 + d.eps0 * kQe / (2.0 * kMe * kC * kC) : 1.0));
    d.az = -kQe * d.E / kMe;
    d.omega = kQe * d.B / kMe;
    d.bx = sin(d.B_angle);
    d.bz = cos(d.B_angle);
    d.vDy = d.B > 0.0 ? d.E * d.B * d.bx / (d.B * d.B) : 0.0;   // (E z^ x B b^)/B^2 = (0, E sin th / B, 0)
    d.apar = d.az * d.bz;
    {
      // relativistic mover in E and B: the generator M (k = -e/m; E along z, B in the xz
      // plane) and the invariants of the field, l1^2 - l2^2 = k^2 (E^2/c^2 - B^2) and
      // l1 l2 = k^2 |E.B|/c (the smaller of l1^2, l2^2 from their product, no cancellation)
      const double k = -kQe / kMe, k2 = k * k;
      const double Bx = d.B * d.bx, Bz = d.B * d.bz;
      d.rel_kEc = k * d.E / kC;
      d.rel_kBx = k * Bx;
      d.rel_kBz = k * Bz;
      const double F1 = (d.E / kC) * (d.E / kC) - d.B * d.B, F2 = d.E * Bz / kC;
      const double sq = sqrt(F1 * F1 + 4.0 * F2 * F2);
      double l1s, l2s;
      if (F1 >= 0.0) {
        l1s = 0.5 * k2 * (F1 + sq);
        l2s = l1s > 0.0 ? k2 * k2 * F2 * F2 / l1s : 0.0;
      } else {
        l2s = 0.5 * k2 * (sq - F1);
        l1s = k2 * k2 * F2 * F2 / l2s;
      }
      const double sum = l1s + l2s;
      d.rel_l1 = sqrt(l1s);
      d.rel_l2 = sqrt(l2s);
      d.rel_p1 = sum > 0.0 ? l1s / sum : 0.5;
      d.rel_p2 = sum > 0.0 ? l2s / sum : 0.5;
      d.rel_K = sum > 0.0 ? l1s * l2s / sum : 0.0;
    }
    // FP32 velocity <-> energy constants.  A lane's speed after a collision is c_speed
    // sqrt(eps'), and the next trials read its energy back as c_eps (vx^2 + vy^2) + (sceps vz)^2.
    // With each constant rounded on its own, that round trip loses 1e-7 of the energy per
    // collision, which a gas losing little energy per collision (2 m/M) accumulates into a
    // mean-energy bias of 1e-7 M/(2m).  c_speed is moved by at most 16 units in the last place
    // so that c_eps c_speed^2 and (sceps c_speed)^2 both equal 1 to about 1e-8.
    {
      const float base = static_cast<float>(d.c_speed);
      float best_cs = base, best_sc = static_cast<float>(sqrt(d.c_eps)), best_ce = static_cast<float>(d.c_eps);
      double best_r = 1e300;
      float cs = base;
      for (int i = 0; i < 16; ++i) cs = nextafterf(cs, 0.0f);
      for (int i = 0; i <= 32; ++i, cs = nextafterf(cs, 1e30f)) {
        const double c = static_cast<double>(cs);
        const float sc = static_cast<float>(1.0 / c);
        const float ce = static_cast<float>(1.0 / (c * c));
        const double r1 = fabs(static_cast<double>(ce) * c * c - 1.0);
        const double r2 = fabs(static_cast<double>(sc) * static_cast<double>(sc) * c * c - 1.0);
        const double r = fmax(r1, r2);
        if (r < best_r) { best_r = r; best_cs = cs; best_sc = sc; best_ce = ce; }
      }
      d.c_speed_f = best_cs;
      d.c_eps_f = best_ce;
      d.sceps_f = best_sc;
    }
    d.speed0_f = static_cast<float>(d.speed0);
    d.az_f = static_cast<float>(d.az);
    d.omega_rev_f = static_cast<float>(d.omega / (2.0 * kPi));
    d.bx_f = static_cast<float>(d.bx);
    d.bz_f = static_cast<float>(d.bz);
    d.vDy_f = static_cast<float>(d.vDy);
    d.apar_f = static_cast<float>(d.apar);
    const double sc = static_cast<double>(d.sceps_f);
    d.aze_f = static_cast<float>(d.az * sc);
    d.apare_f = static_cast<float>(d.apar * sc);
    d.nup24_f = d.majorant_f * 0x1.0p-24f;
    d.Pf_d = static_cast<double>(1 << d.p_log2);
    d.twoPf_d = 2.0 * d.Pf_d;
    d.Pf_f = static_cast<float>(d.Pf_d);
    d.twoPf_f = static_cast<float>(d.twoPf_d);
  }
}

// Binned trial frequency: the nu' of every bin, the largest total rate on its cells (a
// cell's largest rate is at one of its end nodes; table entry 0 holds node 0 alone and entry
// G the top node alone) raised by 2^-20 and capped at the constant value.  One thread per
// bin, after k_build_constants.
__global__ void k_build_bins(InstanceDesc* desc) {
  const InstanceDesc& d = *desc;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n_bins) return;
  const double* F = d.cum_cm + static_cast<size_t>(d.nc - 1) * d.G;
  double m = 0.0;
  for (int i = d.bin_first[k]; i < d.bin_first[k + 1]; ++i) {
    const int g = i == 0 ? 0 : i - 1;
    m = fmax(m, F[g]);
    if (i >= 1 && g + 1 < d.G) m = fmax(m, F[g + 1]);
  }
  const double v = fmin((1.0 + 0x1.0p-20) * m, d.majorant);
  d.bin_nup64[k] = v;
  d.bin_nup32[k] = static_cast<float>(v);
}

// Mark record slots as empty (id = all ones): real-secondaries runs that stop early leave
// slots of queued secondaries unwritten, and the reductions skip empty slots.
__global__ void k_mark_empty(swarm_record* r, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    r[i].id = ~0ull;
    r[i].flags = 0u;
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// =======================================================================================
// Per-electron null-collision loop.
// =======================================================================================

// Instance constants in the working precision, loaded once per work item.
template <typename R>
struct Consts {
  R nup, cT, c_eps, c_speed, speed0, az, omega, bx, bz, vDy, apar;
  R omega_rev;   // omega / (2 pi): the gyration phase in revolutions
  R inv_omega;   // 1 / omega (B > 0), divided once per work item instead of per collision
  R aze, apare;  // accelerations in energy units (FP32: times sqrt(m/2e); FP64: plain)
  R nup24;       // FP32: nu' 2^-24 (x = R nu' straight from the 24-bit integer)
  R Pf, twoPf;   // grid points per octave, and twice that, as floating point
  R sceps;       // FP32: sqrt(m/2e)
  R zeta1;       // variable trial frequency: 1 + zeta
  R eps0;        // initial energy of the primaries (eV)
  bool magnetic; // B > 0 (kernels built for B may also serve B = 0 instances)
  bool variable; // a per-lane trial frequency: the variable or the binned strategy
  bool binned;   // the binned strategy
  bool thermal;  // moving targets
  bool relativistic;  // relativistic mover (FP64): lanes hold u = gamma v
  double rel_kEc, rel_kBx, rel_kBz;       // relativistic in E and B: the generator M
  double rel_l1, rel_l2, rel_p1, rel_p2, rel_K;   // and its invariants
  uint32_t grace0;
  int G, nc, off, p;
  int off1;      // off - 1: raw index of entry 0 of the padded LDS table
  int off1G;     // off1 + G: raw index of its last entry
  float e_lo, e_hi;   // FP32: the float just below 2^emin, and 2^emax (the clamp of the index;
                      // e_hi is held in a vector register, see load_consts)
  uint32_t wmask;     // FP32: the low 23-p mantissa bits (the interpolation weight, unscaled)
  uint32_t n_coll, quantum;
  Key key;
  const typename Pair<R>::T* cum;
  const ChannelDev* chan;
  const double* logtab;    // FP64: the logarithm table of the flight times, in LDS
  const ThermalChannel* chan_th;
  bool cum_lds;            // the running sums are staged in LDS (else: global memory)
  const int32_t* bin_of;   // binned: bin of every padded table entry
  const R* bin_nup;        // binned: nu' of every bin
};

template <typename R>
__device__ __forceinline__ Consts<R> load_consts(const InstanceDesc& d) {
  Consts<R> c;
  if constexpr (sizeof(R) == 8) {
    c.nup = d.majorant; c.cT = d.inv_majorant; c.c_eps = d.c_eps; c.c_speed = d.c_speed;
    c.speed0 = d.speed0; c.az = d.az; c.omega = d.omega; c.bx = d.bx; c.bz = d.bz; c.vDy = d.vDy;
    c.apar = d.apar; c.omega_rev = d.omega * (0.5 / kPi);
    c.cum = reinterpret_cast<const typename Pair<R>::T*>(d.cum64);
    c.off = (1023 + d.emin) << d.p_log2;
  } else {
    c.nup = d.majorant_f; c.cT = d.cT_f; c.c_eps = d.c_eps_f; c.c_speed = d.c_speed_f;
    c.speed0 = d.speed0_f; c.az = d.az_f; c.omega = static_cast<float>(d.omega); c.bx = d.bx_f;
    c.bz = d.bz_f; c.vDy = d.vDy_f; c.apar = d.apar_f; c.omega_rev = d.omega_rev_f;
    c.cum = reinterpret_cast<const typename Pair<R>::T*>(d.cum32);
    c.off = (127 + d.emin) << d.p_log2;
  }
  if constexpr (sizeof(R) == 8) {
    c.aze = d.az; c.apare = d.apar; c.nup24 = 0.0; c.sceps = 1.0;
    c.Pf = d.Pf_d; c.twoPf = d.twoPf_d;
  } else {
    c.aze = d.aze_f; c.apare = d.apare_f; c.nup24 = d.nup24_f; c.sceps = d.sceps_f;
    c.Pf = d.Pf_f; c.twoPf = d.twoPf_f;
  }
  c.magnetic = d.B > 0.0;
  c.inv_omega = c.magnetic ? R(1) / c.omega : R(0);
  c.variable = d.trial_strategy != SWARM_TRIAL_CONSTANT;
  c.binned = d.trial_strategy == SWARM_TRIAL_BINNED;
  c.thermal = d.thermal_targets != 0;
  c.relativistic = d.relativistic != 0;
  c.rel_kEc = d.rel_kEc; c.rel_kBx = d.rel_kBx; c.rel_kBz = d.rel_kBz;
  c.rel_l1 = d.rel_l1; c.rel_l2 = d.rel_l2; c.rel_p1 = d.rel_p1; c.rel_p2 = d.rel_p2; c.rel_K = d.rel_K;
  c.bin_of = d.bin_of;
  if constexpr (sizeof(R) == 8) c.bin_nup = d.bin_nup64;
  else c.bin_nup = d.bin_nup32;
  c.grace0 = d.trial_grace;
  c.zeta1 = static_cast<R>(1.0 + d.trial_zeta);
  c.eps0 = static_cast<R>(d.eps0);
  c.G = d.G; c.nc = d.nc; c.p = d.p_log2;
  c.n_coll = d.n_collisions; c.quantum = d.quantum;
  c.key = {static_cast<uint32_t>(d.seed), static_cast<uint32_t>(d.seed >> 32)};
  c.chan = d.chan;
  c.chan_th = d.chan_th;
  c.cum_lds = false;
  c.off1 = c.off - 1;
  c.off1G = c.off1 + c.G;
  c.wmask = (1u << (23 - d.p_log2)) - 1u;
  c.e_lo = __uint_as_float((static_cast<uint32_t>(127 + d.emin) << 23) - 1u);
  // The median-of-three of the index clamp can read one scalar operand only; a copy the
  // compiler cannot rematerialise keeps the other bound in a vector register for the whole
  // work item instead of a move in every trial.
  const float e_hi = __uint_as_float(static_cast<uint32_t>(127 + d.emax) << 23);
  asm("v_mov_b32 %0, %1" : "=v"(c.e_hi) : "s"(e_hi));
  return c;
}

// Real-collision count at which a lane stops in this launch: the budget, or with a quantum
// (resumable epochs) the count after `quantum` more collisions, summed in 64 bits so that a
// large quantum cannot wrap around.
template <typename R>
__device__ __forceinline__ uint32_t stop_count(uint32_t k, const Consts<R>& C) {
  if (!C.quantum) return C.n_coll;
  const uint64_t q = static_cast<uint64_t>(k) + C.quantum;
  return q < C.n_coll ? static_cast<uint32_t>(q) : C.n_coll;
}

template <typename R>
struct Lane {
  double rx, ry, rz, t;     // anchor (state right after the last real collision), FP64
  R vx, vy, vz;             // anchor velocity
  R T;                      // flight time since the anchor
  R nup, cT, nup24;         // trial frequency nu', flight-time scale (FP32 ln2/nu', FP64
                            // 1/nu') and FP32 nu' 2^-24
  uint32_t grace, nfail;    // variable strategy: trials left before nu' is renewed; fails
  R q0;                     // B = 0: vx^2 + vy^2;  B != 0: |vD|^2 + |u0|^2
  R vpar;                   // B != 0: v0 . b
  R u0x, u0y, u0z;          // B != 0: v0 - (v0.b) b - vD
  R w0x, w0y, w0z;          // B != 0: b x u0
  R Bc, Bs;                 // B != 0: 2 vD.u0, 2 vD.w0
  R e_q0, e_vz, e_vpar, e_Bc, e_Bs;  // the same in energy units (FP32 scaled by m/2e)
  double se, sep;           // sums of energies before / after real collisions
  uint64_t id;
  int64_t rec;              // record slot
  uint32_t block, k, k_start, k_stop, G, D, nforb, nover, flags;
  uint32_t nfirst;          // blocks whose first trial was not null (real or forbidden)
  int state;
  int trace_slot, n_ev;
  R p_eps, p_x;             // pending real-collision candidate: energy and x = R nu'
  int p_gi;                 // its raw table index (padded index + off1, see lds_rate)
  R p_w;                    // and interpolation weight
  uint32_t p_sub;            // 0/1: first or second trial of block `block - 1`
  TrialPre pre_hi, pre_lo;  // first-round Philox terms of the trial streams
  W4 sh, sl;                // scattering block k (SCAT_HI / SCAT_LO words)
};

template <typename R>
__device__ __forceinline__ void set_id(Lane<R>& L, const Consts<R>& C, uint64_t id) {
  L.id = id;
  L.pre_hi = trial_pre(C.key, id, TAG_TRIAL_HI);
  if constexpr (sizeof(R) == 8) L.pre_lo = trial_pre(C.key, id, TAG_TRIAL_LO);
}

// Velocity-dependent constants of the flight that starts at the anchor.  FP32 keeps the
// quantities the per-trial energy needs in energy units (velocities times sqrt(m/2e)),
// so that eps = |v(T)|^2 m/2e costs no extra multiplication per trial.
template <typename R, bool HB>
__device__ __forceinline__ void set_anchor(Lane<R>& L, const Consts<R>& C) {
  if (!HB || !C.magnetic) {
    if constexpr (sizeof(R) == 4) L.q0 = fmaf(L.vy, L.vy, L.vx * L.vx);
    else L.q0 = L.vx * L.vx + L.vy * L.vy;
    if constexpr (sizeof(R) == 4) {
      L.e_q0 = C.c_eps * L.q0;
      L.e_vz = C.sceps * L.vz;
    } else {
      L.e_q0 = L.q0;
      L.e_vz = L.vz;
    }
  } else {
    L.vpar = L.vx * C.bx + L.vz * C.bz;
    L.u0x = (L.vx - C.bx * L.vpar);
    L.u0y = (L.vy - C.vDy);
    L.u0z = (L.vz - C.bz * L.vpar);
    L.w0x = -(C.bz * L.u0y);
    L.w0y = C.bz * L.u0x - C.bx * L.u0z;
    L.w0z = C.bx * L.u0y;
    L.q0 = C.vDy * C.vDy + (L.u0x * L.u0x + L.u0y * L.u0y + L.u0z * L.u0z);
    L.Bc = R(2) * C.vDy * L.u0y;
    L.Bs = R(2) * C.vDy * L.w0y;
    if constexpr (sizeof(R) == 4) {
      L.e_q0 = C.c_eps * L.q0;
      L.e_Bc = C.c_eps * L.Bc;
      L.e_Bs = C.c_eps * L.Bs;
      L.e_vpar = C.sceps * L.vpar;
    } else {
      L.e_q0 = L.q0;
      L.e_Bc = L.Bc;
      L.e_Bs = L.Bs;
      L.e_vpar = L.vpar;
    }
  }
}

// Energy (eV) during free flight, eps = (m/2e) |v(T)|^2 (classical motion in uniform E
// and B).
// Relativistic motion in uniform static E and B (the paper's UniformFieldRelativisticChin),
// FP64.  In proper time tau the 4-velocity Y = (w, u) = (gamma c, u) obeys dY/dtau = M Y,
// M (w, u) = k (E.u/c, E w/c + u x B), k = -e/m.  M^2 has the eigenvalues l1^2 and -l2^2 (from
// the field invariants), so exp(M tau) = a0 + a1 M + a2 M^2 + a3 M^3 with
//   a0 = 1 + K (Ch - Ct), a1 = tau + K (Sh - St), a2 = p1 Ch + p2 Ct, a3 = p1 Sh + p2 St,
//   p1 = l1^2/(l1^2 + l2^2), p2 = l2^2/(l1^2 + l2^2), K = l1^2 l2^2/(l1^2 + l2^2),
//   Ch = (cosh l1 tau - 1)/l1^2, Ct = (1 - cos l2 tau)/l2^2,
//   Sh = (sinh(l1 tau)/l1 - tau)/l1^2, St = (tau - sin(l2 tau)/l2)/l2^2,
// and its integral over [0, tau] has b0 = tau + K (Sh - St), b1 = tau^2/2 + K (Qh - Qt),
// b2 = p1 Sh + p2 St, b3 = p1 Qh + p2 Qt with Qh = (Ch - tau^2/2)/l1^2, Qt = (tau^2/2 - Ct)/l2^2.
// The C, S, Q functions are tau^n g(l tau) with g taken from its series for small arguments
// (their tau -> 0 limits tau^2/2, tau^3/6, tau^4/24 without cancellation).  With l1 = l2 = 0
// (no field, or crossed fields with |E| = c|B|) p1 = p2 = 1/2 and K = 0 give the polynomial
// exp of the nilpotent M.  The laboratory time of a flight fixes tau through c t(tau) = b0 Y0^0
// + ... + b3 Y3^0 (Newton; d(c t)/dtau = w > 0).

// g_n(x) = (cosh x - sum_{j<n, j even} x^j/j!) / x^n for n = 2, 4 and (sinh x - x)/x^3 (n = 3),
// and their trigonometric partners with alternating signs, from the series for |x| < 1.
__device__ __forceinline__ void rel_coeffs(double x, bool hyperbolic, double* c2, double* c3, double* c4) {
  const double x2 = x * x;
  if (fabs(x) < 1.0) {
    const double s = hyperbolic ? x2 : -x2;
    // sum_n s^n / (2n + k)! for k = 2, 3, 4, n = 0..9
    double a2 = 0.0, a3 = 0.0, a4 = 0.0;
    double t = 1.0;
    double d2 = 2.0, d3 = 6.0, d4 = 24.0;   // (k)!
    for (int n = 0; n < 10; ++n) {
      a2 += t / d2; a3 += t / d3; a4 += t / d4;
      t *= s;
      d2 *= (2 * n + 3) * (2 * n + 4);
      d3 *= (2 * n + 4) * (2 * n + 5);
      d4 *= (2 * n + 5) * (2 * n + 6);
    }
    *c2 = a2; *c3 = a3; *c4 = a4;
  } else if (hyperbolic) {
    const double ch = cosh(x), sh = sinh(x);
    *c2 = (ch - 1.0) / x2;
    *c3 = (sh - x) / (x2 * x);
    *c4 = (ch - 1.0 - 0.5 * x2) / (x2 * x2);
  } else {
    double sn, cs;
    sincos(x, &sn, &cs);
    *c2 = (1.0 - cs) / x2;
    *c3 = (x - sn) / (x2 * x);
    *c4 = (cs - 1.0 + 0.5 * x2) / (x2 * x2);
  }
}

// State after a flight of laboratory duration T from the anchor: proper velocity u and, if
// wanted, the displacement.  The anchor holds u0; M^k Y0 are formed by the map above.
__device__ __forceinline__ void rel_eb_state(const Lane<double>& L, const Consts<double>& C, double T, double* u,
                                             double* dr) {
  const double c = kC;
  double y[4][4];   // y[k] = M^k Y0 as (w, u_x, u_y, u_z)
  y[0][1] = L.vx; y[0][2] = L.vy; y[0][3] = L.vz;
  y[0][0] = c * sqrt(1.0 + (L.vx * L.vx + L.vy * L.vy + L.vz * L.vz) / (c * c));
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    const double* a = y[k - 1];
    y[k][0] = C.rel_kEc * a[3];
    y[k][1] = C.rel_kBz * a[2];
    y[k][2] = C.rel_kBx * a[3] - C.rel_kBz * a[1];
    y[k][3] = C.rel_kEc * a[0] - C.rel_kBx * a[2];
  }
  double a0, a1, a2, a3, b0, b1, b2, b3;
  auto coeffs = [&](double tau) {
    double g2, g3, g4, t2, t3, t4;
    rel_coeffs(C.rel_l1 * tau, true, &g2, &g3, &g4);
    rel_coeffs(C.rel_l2 * tau, false, &t2, &t3, &t4);
    const double tt = tau * tau;
    const double Ch = tt * g2, Sh = tt * tau * g3, Qh = tt * tt * g4;
    const double Ct = tt * t2, St = tt * tau * t3, Qt = tt * tt * t4;
    a0 = 1.0 + C.rel_K * (Ch - Ct);
    a1 = tau + C.rel_K * (Sh - St);
    a2 = C.rel_p1 * Ch + C.rel_p2 * Ct;
    a3 = C.rel_p1 * Sh + C.rel_p2 * St;
    b0 = a1;
    b1 = 0.5 * tt + C.rel_K * (Qh - Qt);
    b2 = a3;
    b3 = C.rel_p1 * Qh + C.rel_p2 * Qt;
  };
  // Proper time of the flight: f(tau) = c t(tau) - c T = 0 on [0, T] (dt/dtau = gamma >= 1),
  // f increasing with f' = w.  Newton from T c / w0, with a bisection of the bracket instead
  // whenever the Newton step would leave it, would not halve the step before, or the
  // hyperbolic functions overflow (gamma can grow like exp(l1 tau): Newton alone would crawl
  // down from a far guess by about 1/l1 per step).  Every path ends within 200 steps.
  double lo = 0.0, hi = T, tau = fmin(T * c / y[0][0], T), step = T, step_old = T;
  for (int it = 0; it < 200 && T > 0.0; ++it) {
    coeffs(tau);
    const double f = (b0 * y[0][0] + b1 * y[1][0] + b2 * y[2][0] + b3 * y[3][0]) - c * T;
    const double w = a0 * y[0][0] + a1 * y[1][0] + a2 * y[2][0] + a3 * y[3][0];
    const bool ok = isfinite(f) && isfinite(w) && w > 0.0;
    if (!ok || f > 0.0) hi = tau; else lo = tau;
    const double newton = ok ? tau - f / w : -1.0;
    step_old = step;
    if (!ok || !(newton >= lo && newton <= hi) || fabs(2.0 * f) > fabs(step_old * w)) {
      step = 0.5 * (hi - lo);
      tau = lo + step;
    } else {
      step = tau - newton;
      tau = newton;
    }
    if (fabs(step) <= 1e-12 * tau || hi - lo <= 1e-15 * hi) break;
  }
  coeffs(tau);
#pragma unroll
  for (int i = 1; i < 4; ++i) {
    u[i - 1] = a0 * y[0][i] + a1 * y[1][i] + a2 * y[2][i] + a3 * y[3][i];
    if (dr) dr[i - 1] = b0 * y[0][i] + b1 * y[1][i] + b2 * y[2][i] + b3 * y[3][i];
  }
}

// With the relativistic mover (EXT == 2, FP64) the lane holds the proper velocity u = gamma v
// (with B = 0 it grows like v does classically), and the kinetic energy is (gamma - 1) m c^2 =
// m |u|^2 / (gamma + 1), gamma = sqrt(1 + |u|^2/c^2).
template <typename R, bool HB, int EXT = 0>
__device__ __forceinline__ R energy_at(const Lane<R>& L, const Consts<R>& C, R T) {
  if constexpr (EXT == 2 && HB && sizeof(R) == 8) {
    if (C.relativistic && C.magnetic) {
      double u[3];
      rel_eb_state(L, C, T, u, nullptr);
      const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      return C.c_eps * (2.0 * u2) / (1.0 + sqrt(1.0 + u2 * (1.0 / (kC * kC))));
    }
  }
  if (!HB || !C.magnetic) {
    const R vz = fma_(C.aze, T, L.e_vz);
    if constexpr (sizeof(R) == 4) {
      return fmaf(vz, vz, L.e_q0);
    } else {
      const double u2 = fma(vz, vz, L.e_q0);
      if constexpr (EXT == 2) {
        if (C.relativistic) return C.c_eps * (2.0 * u2) / (1.0 + sqrt(1.0 + u2 * (1.0 / (kC * kC))));
      }
      return C.c_eps * u2;
    }
  } else {
    R s, c;
    if constexpr (sizeof(R) == 4) {
      const float x = __builtin_amdgcn_fractf(C.omega_rev * T);
      s = __builtin_amdgcn_sinf(x);
      c = __builtin_amdgcn_cosf(x);
    } else {
      sincospi(2.0 * C.omega_rev * T, &s, &c);     // omega T = pi (2 omega_rev T)
    }
    const R vp = fma_(C.apare, T, L.e_vpar);
    const R v2 = fma_(vp, vp, fma_(L.e_Bs, s, fma_(L.e_Bc, c, L.e_q0)));
    if constexpr (sizeof(R) == 4) return v2;
    else return C.c_eps * v2;
  }
}

// Total rate at eps from the LDS table, which is padded with an (F[0], 0) entry in front:
// entry g+1 holds node g, entry 0 serves energies below the grid and entry G (the top
// node, whose difference is zero) energies at or above 2^emax, so the clamped index needs
// no select on the weight.  Index and weight are exact: the node index comes from the
// exponent and leading mantissa bits, and w = frac(2 P mant) = frac((2 mant - 1) P) (the
// product by the power of two 2P is exact).  FP32 takes the weight as the integer of the low
// 23-p mantissa bits, w 2^(23-p), against differences stored times 2^-(23-p): the same
// products, one instruction fewer.  The raw index (exponent and leading mantissa
// bits, clamped to [off1, off1 + G]) is returned; the padded index is raw - off1, and the
// table is read through a base moved back by off1 entries (one address instruction).  A
// negative energy (the rounding of a near-zero one in the expanded magnetic form) takes entry
// 0, as below the grid.  With MED3 the FP32 trial clamps the energy instead, to [the float
// below 2^emin, 2^emax], whose indices are off1 and off1 + G: one median-of-three instead of
// a maximum and a minimum, for a vector register that holds the upper bound (taken where the
// kernel has one to spare: B = 0 with the constant trial frequency).
template <bool MED3 = false>
__device__ __forceinline__ int raw_index(float eps, const Consts<float>& C) {
  if constexpr (MED3)
    return static_cast<int>(__float_as_uint(__builtin_amdgcn_fmed3f(eps, C.e_lo, C.e_hi)) >> (23 - C.p));
  else
    return min(max(static_cast<int>(__float_as_uint(eps)) >> (23 - C.p), C.off1), C.off1G);
}
template <bool MED3 = false>
__device__ __forceinline__ int raw_index(double eps, const Consts<double>& C) {
  const int32_t hi = static_cast<int32_t>(static_cast<uint64_t>(__double_as_longlong(eps)) >> 32);
  return min(max(hi >> (20 - C.p), C.off1), C.off1G);    // arithmetic shift: negative -> entry 0
}
template <bool MED3 = false>
__device__ __forceinline__ float lds_rate(const float2* __restrict__ s_nu, float eps, const Consts<float>& C,
                                         int* raw_out, float* w_out) {
  const int raw = raw_index<MED3>(eps, C);
  const float w = static_cast<float>(__float_as_uint(eps) & C.wmask);
  const float2 q = (s_nu - C.off1)[raw];
  *raw_out = raw;
  *w_out = w;
  return fmaf(w, q.y, q.x);
}
template <bool MED3 = false>
__device__ __forceinline__ double lds_rate(const double2* __restrict__ s_nu, double eps, const Consts<double>& C,
                                          int* raw_out, double* w_out) {
  const int raw = raw_index(eps, C);
  const double w = __builtin_amdgcn_fract(__builtin_amdgcn_frexp_mant(eps) * C.twoPf);
  const double2 q = (s_nu - C.off1)[raw];
  *raw_out = raw;
  *w_out = w;
  return q.x + w * q.y;
}

// Trial frequency of a lane.  The constant strategy (the paper's LazyTrialFrequency or a
// fixed value) uses the instance's nu'.  The adaptive strategies of section "Trial
// frequency strategies" keep a per-lane nu', capped at the constant value (which can never
// fail), renewed after every `grace` trials and set anew after every fail: the variable
// strategy (VariableTrialFrequency) takes nu' = (1 + zeta) nu(eps) from the total rate at
// the current energy, the binned one (BinnedTrialFrequency) the nu' of the energy's bin.
template <typename R>
__device__ __forceinline__ void constant_trial_frequency(Lane<R>& L, const Consts<R>& C) {
  L.nup = C.nup;
  L.cT = C.cT;
  L.nup24 = C.nup24;
}
template <typename R>
__device__ __forceinline__ void apply_trial_frequency(Lane<R>& L, R v) {
  L.nup = v;
  if constexpr (sizeof(R) == 4) {
    L.cT = 0.693147180559945309f / v;
    L.nup24 = v * 0x1.0p-24f;
  } else {
    L.cT = 1.0 / v;
    L.nup24 = 0.0;
  }
}
// The lane's nu'.  FP32 lanes read it back from nu' 2^-24 (exact: a power-of-two scale), so
// the compiler need not keep both in registers.
template <typename R>
__device__ __forceinline__ R lane_nup(const Lane<R>& L) {
  if constexpr (sizeof(R) == 4) return L.nup24 * 0x1.0p24f;
  else return L.nup;
}

template <typename R>
__device__ __forceinline__ void set_trial_frequency(Lane<R>& L, const Consts<R>& C, R v) {
  if (v < C.nup) apply_trial_frequency(L, v);
  else constant_trial_frequency(L, C);     // at the cap: exactly the constant strategy
}

// Lane flag (never stored in a record): a binned retry is running, from a fail until the
// next real collision or renewal.
constexpr uint32_t kRetryFlag = 0x80000000u;

// Renewal (and first value) at energy eps with total rate nu and padded table entry `entry`.
template <typename R>
__device__ __forceinline__ void renew_trial_frequency(Lane<R>& L, const Consts<R>& C, R nu, int entry) {
  set_trial_frequency(L, C, C.binned ? C.bin_nup[C.bin_of[entry]] : C.zeta1 * nu);
  L.grace = C.grace0;
  L.flags &= ~kRetryFlag;
}

// After a fail at the candidate's energy (rate nu), with the lane back at its anchor.
// Variable: (1 + zeta) nu from the rate that failed.  Binned: the largest nu' of the bins
// from the anchor energy's bin to the failing energy's bin; a fail during that retry, where
// the paper throws, sets record flag 16 and takes the constant nu'.
template <typename R, bool HB, int EXT>
__device__ __forceinline__ void fail_trial_frequency(Lane<R>& L, const Consts<R>& C, R nu) {
  if (!C.binned) {
    set_trial_frequency(L, C, C.zeta1 * nu);
  } else if (L.flags & kRetryFlag) {
    L.flags |= 16u;
    constant_trial_frequency(L, C);
  } else {
    const int a = C.bin_of[raw_index(energy_at<R, HB, EXT>(L, C, R(0)), C) - C.off1];
    const int f = C.bin_of[L.p_gi - C.off1];
    R v = R(0);
    for (int k = min(a, f); k <= max(a, f); ++k) v = C.bin_nup[k] > v ? C.bin_nup[k] : v;
    set_trial_frequency(L, C, v);
    L.flags |= kRetryFlag;
  }
  L.grace = C.grace0;
}
// EXT: what the kernel is built for.  0: constant trial frequency, targets at rest, classical
// motion (nu' in the instance constants, no per-lane frequency).  1: also the adaptive trial
// frequencies.  2: also moving targets and the relativistic mover.  Each level serves every
// instance of the levels below it.
template <typename R, int EXT>
__device__ __forceinline__ void start_trial_frequency(Lane<R>& L, const Consts<R>& C,
                                                      const typename Pair<R>::T* __restrict__ s_nu, R eps) {
  L.nfail = 0;
  if constexpr (EXT) {
    if (C.variable) {
      int raw;
      R w;
      const R nu = lds_rate(s_nu, eps, C, &raw, &w);
      renew_trial_frequency(L, C, nu, raw - C.off1);
    } else {
      constant_trial_frequency(L, C);
    }
  }
}

// Velocity and displacement after a flight of duration T from the anchor (the same
// equations of motion, written per component).
template <typename R, bool HB, int EXT = 0>
__device__ __forceinline__ void move_full(const Lane<R>& L, const Consts<R>& C, R T,
                                          R* vx, R* vy, R* vz, double* rx, double* ry, double* rz) {
  if constexpr (EXT == 2 && sizeof(R) == 8) {
    if (HB && C.relativistic && C.magnetic) {
      double u[3], dr[3];
      rel_eb_state(L, C, T, u, dr);
      *vx = u[0]; *vy = u[1]; *vz = u[2];
      *rx = L.rx + dr[0]; *ry = L.ry + dr[1]; *rz = L.rz + dr[2];
      return;
    }
    if (C.relativistic) {
      // Relativistic, B = 0 (the lane holds u = gamma v): u_z grows by a T; z advances by
      // c^2 (gamma1 - gamma0)/a = (u_z0 + u_z1) T / (gamma0 + gamma1), and x, y by
      // u_x (c/a) (asinh(u_z1/A) - asinh(u_z0/A)), A^2 = c^2 + u_x^2 + u_y^2, with the
      // difference taken as one asinh of c a T (gamma0 - u_z0 (u_z0 + u_z1)/(c^2 (gamma0 +
      // gamma1))) / A^2 (no cancellation).  Without a field, straight at u0/gamma0.
      const double c2 = kC * kC, a = C.az;
      const double uz0 = L.vz, uz1 = L.vz + a * T;
      const double up2 = L.vx * L.vx + L.vy * L.vy;
      const double g0 = sqrt(1.0 + (up2 + uz0 * uz0) / c2), g1 = sqrt(1.0 + (up2 + uz1 * uz1) / c2);
      *vx = L.vx; *vy = L.vy; *vz = uz1;
      double sx;
      if (a == 0.0) {
        sx = T / g0;
      } else {
        const double arg = kC * a * T * (g0 - uz0 * (uz0 + uz1) / (c2 * (g0 + g1))) / (c2 + up2);
        sx = kC / a * asinh(arg);
      }
      *rx = L.rx + L.vx * sx;
      *ry = L.ry + L.vy * sx;
      *rz = L.rz + (uz0 + uz1) * T / (g0 + g1);
      return;
    }
  }
  if (!HB || !C.magnetic) {
    *vx = L.vx;
    *vy = L.vy;
    *vz = L.vz + C.az * T;
    if constexpr (sizeof(R) == 8) {
      *rx = L.rx + L.vx * T;
      *ry = L.ry + L.vy * T;
      *rz = (L.rz + L.vz * T) + C.az * (0.5 * T * T);
    } else {
      *rx = L.rx + static_cast<double>(L.vx * T);
      *ry = L.ry + static_cast<double>(L.vy * T);
      *rz = L.rz + static_cast<double>(fma_(C.az * 0.5f * T, T, L.vz * T));
    }
  } else {
    R s, c, sh;
    if constexpr (sizeof(R) == 4) {
      const float x = __builtin_amdgcn_fractf(C.omega_rev * T);
      s = __builtin_amdgcn_sinf(x);
      c = __builtin_amdgcn_cosf(x);
      sh = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(0.5f * C.omega_rev * T));
    } else {
      const double ph = 2.0 * C.omega_rev * T;      // omega T / pi
      sincospi(ph, &s, &c);
      sh = sinpi(0.5 * ph);
    }
    const R omc = R(2) * sh * sh;   // 1 - cos(wT)
    const R px = C.bx * L.vpar, pz = C.bz * L.vpar;       // v_par0
    const R ax = C.bx * C.apar, az = C.bz * C.apar;       // a_par
    *vx = ((px + ax * T) + R(0)) + (L.u0x * c + L.w0x * s);
    *vy = ((R(0) + R(0) * T) + C.vDy) + (L.u0y * c + L.w0y * s);
    *vz = ((pz + az * T) + R(0)) + (L.u0z * c + L.w0z * s);
    const R hT2 = R(0.5) * T * T;
    const R inv_w = C.inv_omega;
    const R dx = ((px + R(0)) * T + ax * hT2) + (L.u0x * s + L.w0x * omc) * inv_w;
    const R dy = ((R(0) + C.vDy) * T + R(0) * hT2) + (L.u0y * s + L.w0y * omc) * inv_w;
    const R dz = ((pz + R(0)) * T + az * hT2) + (L.u0z * s + L.w0z * omc) * inv_w;
    *rx = L.rx + static_cast<double>(dx);
    *ry = L.ry + static_cast<double>(dy);
    *rz = L.rz + static_cast<double>(dz);
  }
}

// Start a primary: at the origin, energy eps0, isotropic direction from the INIT stream.
template <typename R, bool HB, int EXT>
__device__ __forceinline__ void init_primary(Lane<R>& L, const Consts<R>& C,
                                             const typename Pair<R>::T* __restrict__ s_nu, uint64_t id) {
  const W4 h = draw(C.key, id, TAG_INIT_HI, 0);
  W4 l = {0, 0, 0, 0};
  if constexpr (sizeof(R) == 8) l = draw(C.key, id, TAG_INIT_LO, 0);
  R nx, ny, nz;
  iso_dir<R>(uni(h.x, l.x, R(0)), uni(h.y, l.y, R(0)), &nx, &ny, &nz);
  L.vx = C.speed0 * nx;
  L.vy = C.speed0 * ny;
  L.vz = C.speed0 * nz;
  L.rx = L.ry = L.rz = 0.0;
  L.t = 0.0;
  set_id(L, C, id);
  L.k = L.k_start = 0;
  L.block = 0;
  L.G = L.D = L.nforb = L.nover = L.nfirst = L.flags = 0;
  L.se = L.sep = 0.0;
  L.T = R(0);
  set_anchor<R, HB>(L, C);
  start_trial_frequency<R, EXT>(L, C, s_nu, C.eps0);
}

template <typename R>
__device__ __forceinline__ void write_record(const InstanceDesc& d, const Lane<R>& L) {
  swarm_record r;
  r.id = L.id;
  r.flags = L.flags & ~kRetryFlag;
  r.k_start = L.k_start;
  r.k_end = L.k;
  r.G = L.G;
  r.D = L.D;
  r.n_forbidden = L.nforb;
  r.n_over = L.nover;
  r.n_fail = L.nfail;
  // null trials: two per block, less the unused second trials (first trial not null),
  // less the real collisions, forbidden picks and fails of this electron
  r.n_null = 2ull * L.block - L.nfirst - (L.k - L.k_start) - L.nforb - L.nfail;
  r.blocks = L.block;
  r.r[0] = L.rx; r.r[1] = L.ry; r.r[2] = L.rz;
  r.t = L.t;
  r.sum_eps = L.se;
  r.sum_epsp = L.sep;
  d.records[L.rec] = r;
}

// Resumable state of a lane at a real-collision boundary (the anchor, T = 0): written at the
// end of a serving epoch, or when a real-secondaries launch parks an electron for the next.
template <typename R, int EXT>
__device__ __forceinline__ SavedState saved_of(const Lane<R>& L, const Consts<R>& C) {
  SavedState s;
  s.r[0] = L.rx; s.r[1] = L.ry; s.r[2] = L.rz;
  s.t = L.t;
  s.v[0] = L.vx; s.v[1] = L.vy; s.v[2] = L.vz;
  s.sum_eps = L.se;
  s.sum_epsp = L.sep;
  s.id = L.id;
  s.block = L.block; s.k = L.k; s.k_start = L.k_start; s.G = L.G; s.D = L.D;
  s.n_forb = L.nforb; s.n_over = L.nover; s.n_first = L.nfirst;
  s.started = 1; s.pad = L.flags;
  s.nup = static_cast<double>(EXT ? lane_nup(L) : C.nup);
  s.grace = EXT ? L.grace : 0u;
  s.n_fail = L.nfail;
  return s;
}

template <typename R, int EXT>
__device__ __forceinline__ void save_state(const InstanceDesc& d, const Lane<R>& L, const Consts<R>& C,
                                           int64_t e) {
  d.saved[e] = saved_of<R, EXT>(L, C);
}

template <typename R, bool HB, int EXT>
__device__ __forceinline__ void load_saved(const SavedState& s, Lane<R>& L, const Consts<R>& C) {
  L.rx = s.r[0]; L.ry = s.r[1]; L.rz = s.r[2];
  L.t = s.t;
  L.vx = static_cast<R>(s.v[0]); L.vy = static_cast<R>(s.v[1]); L.vz = static_cast<R>(s.v[2]);
  L.se = s.sum_eps; L.sep = s.sum_epsp;
  set_id(L, C, s.id);
  L.block = s.block; L.k = s.k; L.k_start = s.k_start; L.G = s.G; L.D = s.D;
  L.nforb = s.n_forb; L.nover = s.n_over; L.nfirst = s.n_first; L.flags = s.pad;
  L.T = R(0);
  if constexpr (EXT) {
    // the same derived values as when nu' was set (at the cap: the constant strategy's)
    const R v = static_cast<R>(s.nup);
    if (C.variable && v < C.nup) apply_trial_frequency(L, v);
    else constant_trial_frequency(L, C);
    L.grace = s.grace;
  }
  L.nfail = s.n_fail;
  set_anchor<R, HB>(L, C);
}

template <typename R, bool HB, int EXT>
__device__ __forceinline__ void load_state(const InstanceDesc& d, Lane<R>& L, const Consts<R>& C, int64_t e) {
  const SavedState s = d.saved[e];
  load_saved<R, HB, EXT>(s, L, C);
}

template <bool TR>
__device__ __forceinline__ int find_trace(const InstanceDesc& d, uint64_t id) {
  if constexpr (!TR) {
    return -1;
  } else {
    for (int i = 0; i < d.n_trace; ++i)
      if (d.trace_ids[i] == id) return i;
    return -1;
  }
}

template <typename R, bool TR>
__device__ __forceinline__ void trace_event(const InstanceDesc& d, Lane<R>& L, int type, int ch,
                                            R eps, R epsp, double t, double rx, double ry, double rz) {
  if constexpr (TR) {
    if (L.trace_slot >= 0 && L.n_ev < d.max_events) {
      swarm_event ev;
      ev.id = L.id; ev.type = type; ev.channel = ch; ev.k = L.k; ev.block = L.block - 1u;
      ev.sub = L.p_sub; ev.pad = 0; ev.eps = static_cast<double>(eps);
      ev.epsp = static_cast<double>(epsp); ev.t = t; ev.r[0] = rx; ev.r[1] = ry; ev.r[2] = rz;
      d.trace_out[static_cast<int64_t>(L.trace_slot) * d.max_events + L.n_ev] = ev;
      L.n_ev += 1;
      d.trace_count[L.trace_slot] = L.n_ev;
    }
  }
}

// One trial from the words (hf, lf) of the flight time and (hr, lr) of the real/null test:
// the flight time grows by -ln(1-u)/nu' (eq. random_time), the energy at the new time is
// looked up in the LDS rate table, and the trial is real when x = u_r nu' < nu(eps)
// (eq. null_fraction).  Leaves eps, x and the table position in the candidate fields.
template <typename R, bool HB, int EXT>
__device__ __forceinline__ bool one_trial(Lane<R>& L, const Consts<R>& C,
                                          const typename Pair<R>::T* __restrict__ s_nu,
                                          uint32_t hf, uint32_t hr, uint32_t lf, uint32_t lr) {
  if constexpr (sizeof(R) == 4) {
    // u = (hf >> 8) 2^-24: -ln(1-u)/nu' = -log2(1 - u) ln2/nu', with 1 - u formed exactly
    // by one FMA (a 24-bit integer times 2^-24 subtracted from 1)
    const float l2 = __builtin_amdgcn_logf(fmaf(static_cast<float>(hf >> 8), -0x1.0p-24f, 1.0f));
    L.T = fmaf(l2, -(EXT ? L.cT : C.cT), L.T);
    L.p_x = static_cast<float>(hr >> 8) * (EXT ? L.nup24 : C.nup24);    // = u_r nu' exactly
  } else {
    L.T = L.T + flight(one_minus_uni(hf, lf), EXT ? L.cT : C.cT, C.logtab);
    L.p_x = uni(hr, lr, R(0)) * (EXT ? L.nup : C.nup);
  }
  L.p_eps = energy_at<R, HB, EXT>(L, C, L.T);
  const R nu = lds_rate<!HB && EXT == 0>(s_nu, L.p_eps, C, &L.p_gi, &L.p_w);
  // Not null when x < nu.  That includes nu > nu' (then x < nu' < nu), a fail of an
  // adaptive strategy, which the collision phase tells apart.
  const bool hit = L.p_x < nu;
  if (EXT && C.variable) {
    L.grace -= 1u;
    if (!hit && L.grace == 0u) renew_trial_frequency(L, C, nu, L.p_gi - C.off1);   // after a null
  }
  return hit;
}

// One random-number block = two candidate trials (eq. random_time for the flight time,
// eq. null_fraction for the real/null test with x = R nu' < nu(eps)).  A non-null
// outcome of the first trial leaves the second unused.  The total rate comes from the
// LDS pair table.  A lane that finds a real candidate is READY at once: its scattering
// words are drawn in the collision phase, where all the wave's waiting lanes draw them in
// one generator call (drawing them in a trial pass would keep the lane out of trials for a
// pass).
template <typename R, bool HB, int EXT>
__device__ __forceinline__ void trial_block(Lane<R>& L, const Consts<R>& C,
                                            const typename Pair<R>::T* __restrict__ s_nu) {
  if (L.block >= kMaxBlocks) {
    L.flags |= 4u;
    L.state = ST_STOPPED;    // stopped at the cap: recorded and flagged
    return;
  }
  const W4 h = draw_trial(C.key, L.pre_hi, L.block);
  W4 l = {0, 0, 0, 0};
  if constexpr (sizeof(R) == 8) l = draw_trial(C.key, L.pre_lo, L.block);
  L.block += 1;
  // The trial writes the candidate fields of the lane directly: a lane that finds a real
  // candidate stops writing them until it is served, so they need no copy, and the second
  // trial runs only on the lanes whose first one was null.
  bool hit = one_trial<R, HB, EXT>(L, C, s_nu, h.x, h.y, l.x, l.y);
  const bool second = !hit;
  if (second) hit = one_trial<R, HB, EXT>(L, C, s_nu, h.z, h.w, l.z, l.w);
  L.p_sub = second ? 1u : 0u;
  L.state = hit ? ST_READY : ST_ACTIVE;
}

// Scattering block k of the lane's electron (SCAT_HI, and SCAT_LO in FP64), through the
// precomputed first round of its trial stream (the tags differ by a constant in word 1).
template <typename R>
__device__ __forceinline__ void draw_scattering(Lane<R>& L, const Consts<R>& C) {
  TrialPre ph = L.pre_hi;
  ph.a ^= (TAG_TRIAL_HI ^ TAG_SCAT_HI);
  L.sh = draw_trial(C.key, ph, L.k);
  if constexpr (sizeof(R) == 8) {
    TrialPre pl = L.pre_lo;
    pl.a ^= (TAG_TRIAL_LO ^ TAG_SCAT_LO);
    L.sl = draw_trial(C.key, pl, L.k);
  } else {
    L.sl = W4{0, 0, 0, 0};
  }
}

// Outcome of serving a pending candidate.
constexpr int kScanChannels = 8;   // up to this many channels, selection scans the whole row

// Few channels (2 <= nc <= N + 1): the first c with x < C_c(eps), or nc - 1 (the last channel
// needs no test), by a backward scan over the row of running sums fetched at once.  The loads
// are unconditional so that they all issue before the first wait: one memory round trip.  From
// global memory they use one address and immediate offsets (the table keeps kScanChannels
// spare pairs after its last row, so entries past the row stay inside the buffer); from LDS the
// indices are clamped to the row.
template <typename R, int N>
__device__ __forceinline__ int first_channel_below(const Consts<R>& C, const typename Pair<R>::T* row, R x, R w) {
  using PT = typename Pair<R>::T;
  const int last = C.nc - 2;
  PT q[N];
  if (C.cum_lds) {
#pragma unroll
    for (int c = 0; c < N; ++c) q[c] = row[min(c, last)];
  } else {
    const __attribute__((address_space(1))) PT* grow = (const __attribute__((address_space(1))) PT*)(row);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      q[c].x = grow[c].x;
      q[c].y = grow[c].y;
    }
  }
  int lo = C.nc - 1;
#pragma unroll
  for (int c = N - 1; c >= 0; --c)
    if (c <= last && x < lerp_pair(q[c], w)) lo = c;
  return lo;
}
enum : int { RC_CONTINUE = 0, RC_STOP = 1 };

// Moving targets (section "Effect of gas temperature").  The target velocity of collision k
// has three normal components of spread sqrt(kT/M), from the four uniforms of the THERMAL
// block by Box-Muller.  moving_target() returns the centre-of-momentum velocity Vcm = (m V1 +
// M V2)/(m + M) and the electron's squared speed in that frame after the threshold loss,
// |V1 - Vcm|^2 - 2 eps_k M / ((m + M) m) (negative: the process cannot happen).  FP64 lanes
// compute in binary64; FP32 lanes in binary32 (hardware log, sqrt, sin and cos), with V1 -
// Vcm as (M/(m + M)) (V1 - V2) and the threshold compared in binary64, as for the onset.
template <typename R>
__device__ __forceinline__ void moving_target(const Lane<R>& L, const Consts<R>& C, int c,
                                              R vx, R vy, R vz, double* vcm, double* g2) {
  const ThermalChannel th = C.chan_th[c];
  const W4 h = draw(C.key, L.id, TAG_THERMAL_HI, L.k);
  if constexpr (sizeof(R) == 4) {
    const float u0 = uni(h.x, 0u, 0.0f), u1 = uni(h.y, 0u, 0.0f), u2 = uni(h.z, 0u, 0.0f), u3 = uni(h.w, 0u, 0.0f);
    // -2 ln(1 - u) = -2 ln2 log2(1 - u); 1 - u is exact for a 24-bit uniform
    const float r01 = sqrt_(-2.0f * 0.693147180559945309f * __builtin_amdgcn_logf(1.0f - u0));
    const float r23 = sqrt_(-2.0f * 0.693147180559945309f * __builtin_amdgcn_logf(1.0f - u2));
    float s1, c1, s3, c3;
    sincos_rev(u1, &s1, &c1);
    sincos_rev(u3, &s3, &c3);
    const float sg = static_cast<float>(th.sigma), cM = static_cast<float>(th.cM);
    const float ux = cM * (vx - sg * r01 * c1), uy = cM * (vy - sg * r01 * s1), uz = cM * (vz - sg * r23 * c3);
    vcm[0] = static_cast<double>(vx - ux);
    vcm[1] = static_cast<double>(vy - uy);
    vcm[2] = static_cast<double>(vz - uz);
    const double dx = ux, dy = uy, dz = uz;
    *g2 = (dx * dx + dy * dy + dz * dz) - th.loss;
    return;
  }
  double u0, u1, u2, u3;
  {
    const W4 l = draw(C.key, L.id, TAG_THERMAL_LO, L.k);
    u0 = uni(h.x, l.x, 0.0); u1 = uni(h.y, l.y, 0.0); u2 = uni(h.z, l.z, 0.0); u3 = uni(h.w, l.w, 0.0);
  }
  const double r01 = sqrt(-2.0 * log(1.0 - u0));
  const double r23 = sqrt(-2.0 * log(1.0 - u2));
  double s1, c1, s3, c3;
  sincos_rev(u1, &s1, &c1);
  sincos_rev(u3, &s3, &c3);
  const double M = th.mass, inv = 1.0 / (kMe + M);
  const double ax = vx, ay = vy, az = vz;
  vcm[0] = (ax * kMe + th.sigma * r01 * c1 * M) * inv;
  vcm[1] = (ay * kMe + th.sigma * r01 * s1 * M) * inv;
  vcm[2] = (az * kMe + th.sigma * r23 * c3 * M) * inv;
  const double ux = ax - vcm[0], uy = ay - vcm[1], uz = az - vcm[2];
  *g2 = (ux * ux + uy * uy + uz * uz) - th.loss;
}

// The paper's equation for the electron after a collision with a moving target: V1' = Vcm +
// sqrt(g2) u, u the new direction in the centre-of-momentum frame (isotropic from the
// scattering block's first two uniforms, or theta about V1 - Vcm for the anisotropic
// models).  Gives the direction of V1' and the energy after (zero for attachment).
template <typename R>
__device__ __forceinline__ void moving_target_outcome(const ChannelDev& ch, const Consts<R>& C, R eps, R u_c, R u_p,
                                                      R vx, R vy, R vz, const double* vcm, double g2,
                                                      R* nx, R* ny, R* nz, R* epsp) {
  if constexpr (sizeof(R) == 4) {
    const float cx = static_cast<float>(vcm[0]), cy = static_cast<float>(vcm[1]), cz = static_cast<float>(vcm[2]);
    // (unit vectors through the hardware reciprocal square root)
    const float ux = vx - cx, uy = vy - cy, uz = vz - cz;
    const float gg = fmaf(uz, uz, fmaf(uy, uy, ux * ux));
    float hx, hy, hz;
    if (ch.scat == SWARM_SCATTER_ISOTROPIC || !(gg > 0.0f)) {
      iso_dir<float>(u_c, u_p, &hx, &hy, &hz);
    } else {
      const float ig = rsqrt_(gg);
      rotate_dir<float>(ux * ig, uy * ig, uz * ig, scatter_cos(ch.scat, ch.xi_f, eps, u_c), u_p, &hx, &hy, &hz);
    }
    const float sp = sqrt_(fmaxf(static_cast<float>(g2), 0.0f));
    const float px = cx + hx * sp, py = cy + hy * sp, pz = cz + hz * sp;
    const float p2 = fmaf(pz, pz, fmaf(py, py, px * px));
    if (p2 > 0.0f) {
      const float is = rsqrt_(p2);
      *nx = px * is; *ny = py * is; *nz = pz * is;
    } else {
      *nx = hx; *ny = hy; *nz = hz;
    }
    *epsp = ch.kind == SWARM_ATTACHMENT ? 0.0f : C.c_eps * p2;
    return;
  }
  const double ux = static_cast<double>(vx) - vcm[0], uy = static_cast<double>(vy) - vcm[1],
               uz = static_cast<double>(vz) - vcm[2];
  const double g = sqrt(ux * ux + uy * uy + uz * uz);
  double hx, hy, hz;
  if (ch.scat == SWARM_SCATTER_ISOTROPIC || !(g > 0.0)) {
    iso_dir<double>(u_c, u_p, &hx, &hy, &hz);
  } else {
    const double ig = 1.0 / g;
    rotate_dir<double>(ux * ig, uy * ig, uz * ig, scatter_cos(ch.scat, ch.xi, static_cast<double>(eps), static_cast<double>(u_c)), u_p,
                       &hx, &hy, &hz);
  }
  const double sp = sqrt(fmax(g2, 0.0));
  const double px = vcm[0] + hx * sp, py = vcm[1] + hy * sp, pz = vcm[2] + hz * sp;
  const double p2 = px * px + py * py + pz * pz;
  const double s1 = sqrt(p2);
  if (s1 > 0.0) {
    const double is = 1.0 / s1;
    *nx = static_cast<R>(px * is); *ny = static_cast<R>(py * is); *nz = static_cast<R>(pz * is);
  } else {
    *nx = static_cast<R>(hx); *ny = static_cast<R>(hy); *nz = static_cast<R>(hz);
  }
  *epsp = ch.kind == SWARM_ATTACHMENT ? R(0) : static_cast<R>(0.5 * kMe * p2 / kQe);
}

// Speed held by a lane after a collision to energy eps: sqrt(2 eps/m), or with the
// relativistic mover the proper speed sqrt(2 eps/m (1 + eps/(2 m c^2))).
template <typename R, int EXT>
__device__ __forceinline__ R speed_of_energy(const Consts<R>& C, R eps) {
  if constexpr (EXT == 2 && sizeof(R) == 8) {
    if (C.relativistic) return C.c_speed * sqrt(eps * (1.0 + eps * (kQe / (2.0 * kMe * kC * kC))));
  }
  return C.c_speed * sqrt_(eps);
}

// A forbidden channel pick: counted, traced and treated as a null trial.
template <typename R, bool TR, int EXT>
__device__ __forceinline__ int forbidden_pick(const InstanceDesc& d, Lane<R>& L, const Consts<R>& C, int lo, R eps,
                                              R nu_eps) {
  L.nforb += 1;
  trace_event<R, TR>(d, L, 2, lo, eps, eps, L.t + static_cast<double>(L.T), L.rx, L.ry, L.rz);
  if (EXT && C.variable && L.grace == 0u) renew_trial_frequency(L, C, nu_eps, L.p_gi - C.off1);   // as after a null
  L.state = ST_ACTIVE;
  return RC_CONTINUE;
}

// A pending candidate: channel selection (min c with x < C_c(eps)), the kinematic onset
// check, isotropic scattering with Fraser-Mathieson energy transfer, ionisation and
// attachment, then the anchor moves to the collision point.  Returns RC_STOP when the
// electron has reached its stop count or was removed.
template <typename R, bool HB, bool TR, bool REAL, int EXT>
__device__ __forceinline__ int real_collision(const InstanceDesc& d, Lane<R>& L, const Consts<R>& C,
                                              const typename Pair<R>::T* __restrict__ s_nu,
                                              bool* spawn) {
  *spawn = false;
  const R eps = L.p_eps;
  const R x = L.p_x;
  L.nfirst += L.p_sub == 0 ? 1u : 0u;
  R nu_eps = R(0);
  if (EXT && C.variable) {
    // the total rate the trial compared with (same table entry and weight)
    nu_eps = lerp_pair(s_nu[L.p_gi - C.off1], L.p_w);
    if (nu_eps > lane_nup(L)) {
      // Fail: nu(eps) <= nu' does not hold.  Back to the state of the last real collision
      // (the anchor: T = 0) with a new nu'; the grace count restarts.
      L.nfail += 1u;
      trace_event<R, TR>(d, L, 3, -1, eps, eps, L.t + static_cast<double>(L.T), L.rx, L.ry, L.rz);
      L.T = R(0);
      fail_trial_frequency<R, HB, EXT>(L, C, nu_eps);
      L.state = ST_ACTIVE;
      return RC_CONTINUE;
    }
  }
  // row and weight of the candidate: the running sums are padded as the total rate is (row 0
  // below the grid, row G at or above its top, both with zero differences), so the trial's
  // padded index and weight select them without clamps (the weight is zeroed above the grid
  // only because that keeps the magnetic adaptive kernels at 128 registers)
  const int gi = L.p_gi - C.off1;
  const bool over = gi >= C.G;
  const R w = over ? R(0) : L.p_w;
  const typename Pair<R>::T* row = C.cum + gi * C.nc;   // (G+1) nc < 2^31: a 32-bit offset
  int lo;
  if (C.nc == 1) {
    lo = 0;
  } else if (C.nc <= 5) {
    lo = first_channel_below<R, 4>(C, row, x, w);     // the argon-like gas: 5 channels
  } else if (C.nc <= kScanChannels) {
    lo = first_channel_below<R, kScanChannels - 1>(C, row, x, w);
  } else {
    // many channels: bisection on the running sums, which do not decrease with c
    lo = 0;
    int hi = C.nc - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (x < lerp_pair(row[mid], w)) hi = mid; else lo = mid + 1;
    }
  }
  const ChannelDev ch = C.chan[lo];     // channel descriptors are staged in LDS
  R vx, vy, vz;
  double rx, ry, rz;
  move_full<R, HB, EXT>(L, C, L.T, &vx, &vy, &vz, &rx, &ry, &rz);
  // Forbidden: with moving targets, below the threshold in the centre-of-momentum frame;
  // with targets at rest, an energy below the inelastic onset eps_k (m+M)/M (compared in
  // FP64).
  double vcm[3] = {0.0, 0.0, 0.0}, g2 = 0.0;
  if constexpr (EXT == 2) {
    if (C.thermal) {
      moving_target<R>(L, C, lo, vx, vy, vz, vcm, &g2);
      if (ch.kind != SWARM_ATTACHMENT && g2 < 0.0) return forbidden_pick<R, TR, EXT>(d, L, C, lo, eps, nu_eps);
    }
  }
  if (!(EXT == 2 && C.thermal) && (ch.kind == SWARM_EXCITATION || ch.kind == SWARM_IONIZATION)) {
    double e64;
    if constexpr (sizeof(R) == 8) {
      e64 = eps;
    } else {
      // the squares of binary32 components are exact in binary64, so the FMAs round as the
      // plain sum does
      const double dx = vx, dy = vy, dz = vz;
      e64 = d.c_eps * fma(dz, dz, fma(dy, dy, dx * dx));
    }
    if (e64 < ch.onset) return forbidden_pick<R, TR, EXT>(d, L, C, lo, eps, nu_eps);
  }
  if (over) L.nover += 1;
  draw_scattering<R>(L, C);   // scattering block k (kept in the lane for a secondary)
  const W4 h = L.sh;
  const W4 l = L.sl;
  R nx, ny, nz;
  const R u_c = uni(h.x, l.x, R(0)), u_p = uni(h.y, l.y, R(0));
  R epsp;
  if (EXT == 2 && C.thermal) {
    moving_target_outcome<R>(ch, C, eps, u_c, u_p, vx, vy, vz, vcm, g2, &nx, &ny, &nz, &epsp);
  } else {
    R v2;
    if constexpr (sizeof(R) == 8) v2 = vx * vx + vy * vy + vz * vz;
    else v2 = fmaf(vz, vz, fmaf(vy, vy, vx * vx));
    R cos_t;
    if (ch.scat == SWARM_SCATTER_ISOTROPIC || !(v2 > R(0))) {
      // isotropic in the lab frame; theta is the angle to the incoming velocity
      if constexpr (sizeof(R) == 4) iso_dir_u24(h.x, u_p, &nx, &ny, &nz);
      else iso_dir<R>(u_c, u_p, &nx, &ny, &nz);
      if constexpr (sizeof(R) == 8) cos_t = v2 > 0.0 ? (nx * vx + ny * vy + nz * vz) / sqrt(v2) : 0.0;
      else cos_t = v2 > 0.0f ? fmaf(nz, vz, fmaf(ny, vy, nx * vx)) * rsqrt_(v2) : 0.0f;
    } else {
      // anisotropic: theta about the incoming direction, azimuth 2 pi u'
      R xi;
      if constexpr (sizeof(R) == 8) xi = ch.xi;
      else xi = ch.xi_f;
      cos_t = scatter_cos(ch.scat, xi, eps, u_c);
      R inv;
      if constexpr (sizeof(R) == 8) inv = 1.0 / sqrt(v2);
      else inv = rsqrt_(v2);
      rotate_dir<R>(vx * inv, vy * inv, vz * inv, cos_t, u_p, &nx, &ny, &nz);
    }
    R c_ela, c_M, c_mM, thr;
    if constexpr (sizeof(R) == 8) { c_ela = ch.c_ela; c_M = ch.c_M; c_mM = ch.c_mM; thr = ch.thr; }
    else { c_ela = ch.c_ela_f; c_M = ch.c_M_f; c_mM = ch.c_mM_f; thr = ch.thr_f; }
    if constexpr (sizeof(R) == 4) {
      // FP32: one branch-free evaluation for every kind.  With the threshold taken as 0 for
      // an elastic channel, ratio = 0 and root = 1 make eq. delta_energy_ine round exactly as
      // eq. delta_energy_ela (1 + c (cos - 1) is 1 - c (1 - cos) negated twice); attachment
      // (plastic) selects 0.  Mixed-kind passes then run no divergent branches.  Same box,
      // interleaved, identical records: argon-sweep step 784-785 against 787-788 ms; variable
      // trial frequency 611 against 617 ms, binned 636-637 against 632-633 ms.
      const float th = ch.kind == SWARM_ELASTIC ? 0.0f : thr;
      const float ratio = th * __builtin_amdgcn_rcpf(eps);
      const float root = sqrt_(fmaxf(0.0f, 1.0f - c_mM * ratio));
      epsp = eps * (1.0f - c_M * ratio + c_ela * (root * cos_t - 1.0f));
      if (ch.kind == SWARM_ATTACHMENT) epsp = 0.0f;
    } else if (ch.kind == SWARM_ELASTIC) {
      epsp = eps * (R(1) - c_ela * (R(1) - cos_t));                       // eq. delta_energy_ela
    } else if (ch.kind == SWARM_ATTACHMENT) {
      epsp = R(0);                                                       // plastic collision
    } else {
      R ratio;
      if constexpr (sizeof(R) == 4) ratio = thr * __builtin_amdgcn_rcpf(eps);
      else ratio = thr / eps;
      const R root = sqrt_(fmax(R(0), R(1) - c_mM * ratio));
      epsp = eps * (R(1) - c_M * ratio + c_ela * (root * cos_t - R(1)));  // eq. delta_energy_ine
    }
  }
  epsp = fmax(epsp, R(0));
  L.se += static_cast<double>(eps);
  bool removed = false;
  if (ch.kind == SWARM_IONIZATION) {
    epsp = epsp * R(0.5);            // equal sharing with the ejected electron
    L.G += 1;
    if constexpr (REAL) {
      // The secondary is built after this collision from the lane (make_child): it starts at
      // the collision point and time with the parent's count after it, takes its direction
      // from words 3 and 4 of the scattering block (still in L.sh, L.sl) and this energy,
      // which is kept in the candidate field (unused until the next trial).
      L.p_eps = epsp;
      *spawn = true;
    }
  } else if (ch.kind == SWARM_ATTACHMENT) {
    L.D += 1;
    if constexpr (REAL) removed = true;
  }
  L.sep += static_cast<double>(epsp);
  const double tn = L.t + static_cast<double>(L.T);
  trace_event<R, TR>(d, L, 1, lo, eps, epsp, tn, rx, ry, rz);
  L.k += 1;
  L.rx = rx; L.ry = ry; L.rz = rz;
  L.t = tn;
  L.T = R(0);
  const R sp = speed_of_energy<R, EXT>(C, epsp);
  L.vx = sp * nx; L.vy = sp * ny; L.vz = sp * nz;
  if (EXT && C.variable) {
    L.flags &= ~kRetryFlag;     // a binned retry ends at the next real collision
    if (L.grace == 0u) {        // renewed after a real collision: from the energy after it
      int raw;
      R w;
      const R nu_n = lds_rate(s_nu, epsp, C, &raw, &w);
      renew_trial_frequency(L, C, nu_n, raw - C.off1);
    }
  }
  if (removed) {
    L.flags |= 2u;
    return RC_STOP;
  }
  if (L.k >= L.k_stop) return RC_STOP;
  set_anchor<R, HB>(L, C);
  L.state = ST_ACTIVE;
  return RC_CONTINUE;
}

// The secondary of an ionisation served by real_collision (see there): the lane holds the
// collision point, time and count after it, the scattering words and the shared energy.
template <typename R, int EXT>
__device__ __forceinline__ ChildState make_child(const Lane<R>& L, const Consts<R>& C) {
  const W4 cw = draw(C.key, L.id, TAG_CHILD, L.k - 1);
  R sx, sy, sz;
  iso_dir<R>(uni(L.sh.z, L.sl.z, R(0)), uni(L.sh.w, L.sl.w, R(0)), &sx, &sy, &sz);
  const R epsp = L.p_eps;
  const R sp = speed_of_energy<R, EXT>(C, epsp);
  ChildState child;
  child.r[0] = L.rx; child.r[1] = L.ry; child.r[2] = L.rz;
  child.t = L.t;
  child.v[0] = sp * sx; child.v[1] = sp * sy; child.v[2] = sp * sz;
  child.id = (static_cast<uint64_t>(cw.x) | (static_cast<uint64_t>(cw.y) << 32)) | (1ull << 63);
  child.k = L.k;
  child.pad = 0;
  child.eps_birth = static_cast<double>(epsp);
  return child;
}

// Table layout 1: the instance's running-sum pairs (G x nc, node major) staged in LDS at
// cum_off, so the channel search reads LDS instead of L2.
template <typename R>
__device__ __forceinline__ void stage_cum(const InstanceDesc& d, unsigned char* smem, int cum_off) {
  using PT = typename Pair<R>::T;
  if (cum_off < 0) return;
  const PT* src = reinterpret_cast<const PT*>(sizeof(R) == 8 ? static_cast<const void*>(d.cum64)
                                                             : static_cast<const void*>(d.cum32));
  PT* dst = reinterpret_cast<PT*>(smem + cum_off);
  const int n = (d.G + 1) * d.nc;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// ---------------------------------------------------------------------------------------
// Dummy-mode persistent kernel over work items (instance, electron range).  A work-group
// claims an item, stages the instance's total-rate pairs in LDS (if it changed), and its
// lanes take electrons of the item one after another.  Lanes that reach a real-collision
// candidate wait; the wave serves all waiting lanes together once `pend_trig` of them
// wait (or no lane can make progress otherwise), which keeps the costly collision code
// from running for one lane at a time.
// ---------------------------------------------------------------------------------------
template <typename R, bool HB, bool TR, int EXT>
__global__ void __launch_bounds__(512) k_swarm_dummy(const InstanceDesc* __restrict__ descs,
                                                     const WorkItem* __restrict__ items, int n_items,
                                                     int* __restrict__ item_ctr, int pend_trig,
                                                     int ch_off, int cum_off) {
  using PT = typename Pair<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  PT* s_nu = reinterpret_cast<PT*>(smem);
  __shared__ double s_logtab[sizeof(R) == 8 ? kUnitLogStride * kUnitLogEntries : 1];
  ChannelDev* s_ch = reinterpret_cast<ChannelDev*>(smem + ch_off);
  __shared__ int s_item;
  __shared__ int s_next;
  int cur_inst = -1;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(item_ctr, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= n_items) break;
    const WorkItem wi = items[it];
    const int inst = __builtin_amdgcn_readfirstlane(wi.inst);
    const InstanceDesc& d = descs[inst];
    if (inst != cur_inst) {
      const PT* src = reinterpret_cast<const PT*>(sizeof(R) == 8 ? static_cast<const void*>(d.nu64)
                                                                 : static_cast<const void*>(d.nu32));
      for (int g = threadIdx.x; g <= d.G; g += blockDim.x) {
        PT q = src[g > 0 ? g - 1 : 0];
        if (g == 0) q.y = 0;
        s_nu[g] = q;
      }
      for (int c = threadIdx.x; c < d.nc; c += blockDim.x) s_ch[c] = d.chan[c];
      if constexpr (sizeof(R) == 8)
        for (int j = threadIdx.x; j < kUnitLogStride * kUnitLogEntries; j += blockDim.x) s_logtab[j] = d.logtab[j];
      stage_cum<R>(d, smem, cum_off);
      cur_inst = inst;
    }
    if (threadIdx.x == 0) s_next = 0;
    __syncthreads();
    Consts<R> C = load_consts<R>(d);
    C.chan = s_ch;
    C.logtab = s_logtab;
    if (cum_off >= 0) {
      C.cum = reinterpret_cast<const PT*>(smem + cum_off);
      C.cum_lds = true;
    }
    const int64_t count = wi.count;
    Lane<R> L;
    L.state = ST_IDLE;
    L.trace_slot = -1;
    L.n_ev = 0;
    for (;;) {
      if (L.state == ST_IDLE) {
        const int e = atomicAdd(&s_next, 1);
        if (e < count) {
          const int64_t ei = wi.first + e;
          const uint32_t started = d.saved != nullptr ? d.saved[ei].started : 0u;
          if (started != 2u) {          // 2: finished in an earlier launch
            L.rec = ei;
            if (started == 1u) load_state<R, HB, EXT>(d, L, C, ei);
            else init_primary<R, HB, EXT>(L, C, s_nu, static_cast<uint64_t>(ei));
            L.k_stop = stop_count(L.k, C);
            if constexpr (TR) {
              L.trace_slot = find_trace<TR>(d, L.id);
              L.n_ev = L.trace_slot >= 0 ? d.trace_count[L.trace_slot] : 0;
            }
            L.state = ST_ACTIVE;
          }
        } else {
          L.state = ST_DONE;
        }
      }
      // Trial phase: random-number blocks until enough lanes of the wave wait on a
      // real-collision candidate (or none can go on), then serve them together.  (`drawing`
      // is carried to the next pass, so the test is made once per pass.)
      bool drawing = L.state == ST_ACTIVE;
      for (;;) {
        if (drawing) trial_block<R, HB, EXT>(L, C, s_nu);
        drawing = L.state == ST_ACTIVE;
        const uint64_t ready = __ballot(L.state == ST_READY);
        if (__ballot(drawing) == 0 || static_cast<int>(__popcll(ready)) >= pend_trig) break;
      }
      if (L.state == ST_READY) {
        bool spawn;
        if (real_collision<R, HB, TR, false, EXT>(d, L, C, s_nu, &spawn) == RC_STOP) L.state = ST_STOPPED;
      }
      // An electron that stopped leaves its final record (budget reached or block cap) or
      // its resumable state (end of the launch's quantum).
      if (L.state == ST_STOPPED) {
        if (L.k >= C.n_coll || (L.flags & 4u)) {
          if (L.k >= C.n_coll) L.flags |= 1u;
          write_record(d, L);
          atomicAdd(reinterpret_cast<unsigned long long*>(&d.ctr->n_done), 1ull);
          if (d.saved != nullptr) d.saved[L.rec].started = 2u;
        } else {
          save_state<R, EXT>(d, L, C, L.rec);
        }
        L.state = ST_IDLE;
      }
      if (__ballot(L.state != ST_DONE) == 0) break;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Pooled dummy-mode kernel.  The same per-electron work as k_swarm_dummy, scheduled so that
// collision code runs at full wave width.  A work-group has trial waves and service waves.
// A round has three barriers.  Before the first, the owning lanes take back the electrons
// served in the previous round (so no slot is reused before it has been read).  Between the
// first and the second each trial wave runs one random-number block on its electrons, and
// lanes that found a real-collision candidate copy their state into a pool in LDS (one slot
// per candidate, at most 64 per service wave; the others retry in the next round).  Between
// the second and the third the service waves draw the scattering words, serve the pool, one
// full wave per 64 candidates, and write the outcome back into the slots.  Only the schedule
// differs from k_swarm_dummy: the streams and the per-electron arithmetic are the same, so
// the results are identical.
// ---------------------------------------------------------------------------------------

// Pool layout: structure of arrays over `cap` slots (doubles, then working-precision
// values, then 32-bit words), so that consecutive lanes touch consecutive LDS words.
enum : int { PD_RX = 0, PD_RY, PD_RZ, PD_T, PD_SE, PD_SEP, kPoolD };
enum : int { PR_VX = 0, PR_VY, PR_VZ, PR_TT, PR_EPS, PR_X, PR_W, PR_NUP, kPoolR };
enum : int { PU_GI = 0, PU_SUB, PU_NFIRST, PU_NFORB, PU_NOVER, PU_G, PU_D, PU_K, PU_KSTOP, PU_FLAGS,
             PU_STATE, PU_GRACE, PU_NFAIL, PU_IDLO, PU_IDHI, kPoolU };

template <typename R>
struct Pool {
  double* d;
  R* r;
  uint32_t* u;
  int cap;
  __device__ double& D(int f, int s) const { return d[f * cap + s]; }
  __device__ R& V(int f, int s) const { return r[f * cap + s]; }
  __device__ uint32_t& U(int f, int s) const { return u[f * cap + s]; }
};

// Owner -> pool: the candidate and everything the collision code reads or updates.
template <typename R, int EXT>
__device__ __forceinline__ void pool_put(const Pool<R>& P, int s, const Lane<R>& L) {
  P.D(PD_RX, s) = L.rx; P.D(PD_RY, s) = L.ry; P.D(PD_RZ, s) = L.rz; P.D(PD_T, s) = L.t;
  P.D(PD_SE, s) = L.se; P.D(PD_SEP, s) = L.sep;
  P.V(PR_VX, s) = L.vx; P.V(PR_VY, s) = L.vy; P.V(PR_VZ, s) = L.vz; P.V(PR_TT, s) = L.T;
  P.V(PR_EPS, s) = L.p_eps; P.V(PR_X, s) = L.p_x; P.V(PR_W, s) = L.p_w;
  P.U(PU_GI, s) = static_cast<uint32_t>(L.p_gi); P.U(PU_SUB, s) = L.p_sub;
  P.U(PU_NFIRST, s) = L.nfirst; P.U(PU_NFORB, s) = L.nforb; P.U(PU_NOVER, s) = L.nover;
  P.U(PU_G, s) = L.G; P.U(PU_D, s) = L.D; P.U(PU_K, s) = L.k; P.U(PU_KSTOP, s) = L.k_stop;
  P.U(PU_FLAGS, s) = L.flags; P.U(PU_NFAIL, s) = L.nfail;
  P.U(PU_IDLO, s) = static_cast<uint32_t>(L.id); P.U(PU_IDHI, s) = static_cast<uint32_t>(L.id >> 32);
  if constexpr (EXT) {
    P.V(PR_NUP, s) = lane_nup(L);
    P.U(PU_GRACE, s) = L.grace;
  }
}

// Per-lane trial frequency from a stored nu' (at the cap: the constant strategy's values).
template <typename R, int EXT>
__device__ __forceinline__ void restore_trial_frequency(Lane<R>& L, const Consts<R>& C, R v) {
  if constexpr (EXT) {
    if (C.variable && v < C.nup) apply_trial_frequency(L, v);
    else constant_trial_frequency(L, C);
  }
}

// Service lane <- pool: a lane state complete enough for real_collision.
template <typename R, bool HB, int EXT>
__device__ __forceinline__ void pool_take(const Pool<R>& P, int s, Lane<R>& S, const Consts<R>& C) {
  S.rx = P.D(PD_RX, s); S.ry = P.D(PD_RY, s); S.rz = P.D(PD_RZ, s); S.t = P.D(PD_T, s);
  S.se = P.D(PD_SE, s); S.sep = P.D(PD_SEP, s);
  S.vx = P.V(PR_VX, s); S.vy = P.V(PR_VY, s); S.vz = P.V(PR_VZ, s); S.T = P.V(PR_TT, s);
  S.p_eps = P.V(PR_EPS, s); S.p_x = P.V(PR_X, s); S.p_w = P.V(PR_W, s);
  S.p_gi = static_cast<int>(P.U(PU_GI, s)); S.p_sub = P.U(PU_SUB, s);
  S.nfirst = P.U(PU_NFIRST, s); S.nforb = P.U(PU_NFORB, s); S.nover = P.U(PU_NOVER, s);
  S.G = P.U(PU_G, s); S.D = P.U(PU_D, s); S.k = P.U(PU_K, s); S.k_stop = P.U(PU_KSTOP, s);
  S.flags = P.U(PU_FLAGS, s); S.nfail = P.U(PU_NFAIL, s);
  set_id(S, C, static_cast<uint64_t>(P.U(PU_IDLO, s)) | (static_cast<uint64_t>(P.U(PU_IDHI, s)) << 32));
  if constexpr (EXT) {
    restore_trial_frequency<R, EXT>(S, C, P.V(PR_NUP, s));
    S.grace = P.U(PU_GRACE, s);
  }
  S.trace_slot = -1;
  S.n_ev = 0;
  set_anchor<R, HB>(S, C);
  // (the collision code draws the scattering block k from the first-round terms set_id made)
}

// Service lane -> pool: the outcome.
template <typename R, int EXT>
__device__ __forceinline__ void pool_give(const Pool<R>& P, int s, const Lane<R>& S) {
  P.D(PD_RX, s) = S.rx; P.D(PD_RY, s) = S.ry; P.D(PD_RZ, s) = S.rz; P.D(PD_T, s) = S.t;
  P.D(PD_SE, s) = S.se; P.D(PD_SEP, s) = S.sep;
  P.V(PR_VX, s) = S.vx; P.V(PR_VY, s) = S.vy; P.V(PR_VZ, s) = S.vz; P.V(PR_TT, s) = S.T;
  P.U(PU_NFIRST, s) = S.nfirst; P.U(PU_NFORB, s) = S.nforb; P.U(PU_NOVER, s) = S.nover;
  P.U(PU_G, s) = S.G; P.U(PU_D, s) = S.D; P.U(PU_K, s) = S.k; P.U(PU_FLAGS, s) = S.flags;
  P.U(PU_STATE, s) = static_cast<uint32_t>(S.state); P.U(PU_NFAIL, s) = S.nfail;
  if constexpr (EXT) {
    P.V(PR_NUP, s) = lane_nup(S);
    P.U(PU_GRACE, s) = S.grace;
  }
}

// Owner <- pool: take the served electron back.
template <typename R, bool HB, int EXT>
__device__ __forceinline__ void pool_back(const Pool<R>& P, int s, Lane<R>& L, const Consts<R>& C) {
  L.rx = P.D(PD_RX, s); L.ry = P.D(PD_RY, s); L.rz = P.D(PD_RZ, s); L.t = P.D(PD_T, s);
  L.se = P.D(PD_SE, s); L.sep = P.D(PD_SEP, s);
  L.vx = P.V(PR_VX, s); L.vy = P.V(PR_VY, s); L.vz = P.V(PR_VZ, s); L.T = P.V(PR_TT, s);
  L.nfirst = P.U(PU_NFIRST, s); L.nforb = P.U(PU_NFORB, s); L.nover = P.U(PU_NOVER, s);
  L.G = P.U(PU_G, s); L.D = P.U(PU_D, s); L.k = P.U(PU_K, s); L.flags = P.U(PU_FLAGS, s);
  L.state = static_cast<int>(P.U(PU_STATE, s)); L.nfail = P.U(PU_NFAIL, s);
  if constexpr (EXT) {
    restore_trial_frequency<R, EXT>(L, C, P.V(PR_NUP, s));
    L.grace = P.U(PU_GRACE, s);
  }
  set_anchor<R, HB>(L, C);
}

// One random-number block of an ACTIVE lane in the pooled schedule: a real candidate
// leaves the lane in CAND (the scattering words are drawn by the service wave).
template <typename R, bool HB, int EXT>
__device__ __forceinline__ void trial_block_pooled(Lane<R>& L, const Consts<R>& C,
                                                   const typename Pair<R>::T* __restrict__ s_nu) {
  if (L.block >= kMaxBlocks) {
    L.flags |= 4u;
    L.state = ST_STOPPED;
    return;
  }
  const W4 h = draw_trial(C.key, L.pre_hi, L.block);
  W4 l = {0, 0, 0, 0};
  if constexpr (sizeof(R) == 8) l = draw_trial(C.key, L.pre_lo, L.block);
  L.block += 1;
  bool hit = one_trial<R, HB, EXT>(L, C, s_nu, h.x, h.y, l.x, l.y);
  L.p_sub = 0;
  if (!hit) {
    hit = one_trial<R, HB, EXT>(L, C, s_nu, h.z, h.w, l.z, l.w);
    L.p_sub = 1;
  }
  if (hit) L.state = ST_CAND;
}

template <typename R, bool HB, int EXT>
__global__ void __launch_bounds__(512) k_swarm_pooled(const InstanceDesc* __restrict__ descs,
                                                      const WorkItem* __restrict__ items, int n_items,
                                                      int* __restrict__ item_ctr, int n_service,
                                                      int ch_off, int pool_off, int cum_off) {
  using PT = typename Pair<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  PT* s_nu = reinterpret_cast<PT*>(smem);
  __shared__ double s_logtab[sizeof(R) == 8 ? kUnitLogStride * kUnitLogEntries : 1];
  ChannelDev* s_ch = reinterpret_cast<ChannelDev*>(smem + ch_off);
  __shared__ int s_item;
  __shared__ int s_next;
  __shared__ int s_ncand[2];   // pool slots asked for, by round parity
  __shared__ int s_live[3];    // some electron of the item is not done, by round mod 3
  const int wave = static_cast<int>(threadIdx.x) >> 6;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int n_trial = static_cast<int>(blockDim.x >> 6) - n_service;
  const bool server = wave >= n_trial;
  Pool<R> P;
  P.cap = 64 * n_service;
  P.d = reinterpret_cast<double*>(smem + pool_off);
  P.r = reinterpret_cast<R*>(P.d + kPoolD * P.cap);
  P.u = reinterpret_cast<uint32_t*>(P.r + kPoolR * P.cap);
  const uint64_t lane_lt = (1ull << lane) - 1ull;
  int cur_inst = -1;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(item_ctr, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= n_items) break;
    const WorkItem wi = items[it];
    const int inst = __builtin_amdgcn_readfirstlane(wi.inst);
    const InstanceDesc& d = descs[inst];
    if (inst != cur_inst) {
      const PT* src = reinterpret_cast<const PT*>(sizeof(R) == 8 ? static_cast<const void*>(d.nu64)
                                                                 : static_cast<const void*>(d.nu32));
      for (int g = threadIdx.x; g <= d.G; g += blockDim.x) {
        PT q = src[g > 0 ? g - 1 : 0];
        if (g == 0) q.y = 0;
        s_nu[g] = q;
      }
      for (int c = threadIdx.x; c < d.nc; c += blockDim.x) s_ch[c] = d.chan[c];
      if constexpr (sizeof(R) == 8)
        for (int j = threadIdx.x; j < kUnitLogStride * kUnitLogEntries; j += blockDim.x) s_logtab[j] = d.logtab[j];
      stage_cum<R>(d, smem, cum_off);
      cur_inst = inst;
    }
    if (threadIdx.x == 0) {
      s_next = 0;
      s_ncand[0] = s_ncand[1] = 0;
      s_live[0] = s_live[1] = s_live[2] = 0;
    }
    __syncthreads();
    Consts<R> C = load_consts<R>(d);
    C.chan = s_ch;
    C.logtab = s_logtab;
    if (cum_off >= 0) {
      C.cum = reinterpret_cast<const PT*>(smem + cum_off);
      C.cum_lds = true;
    }
    if (server) {
      // ---- service waves: the same three barriers per round as the trial waves ----
      for (int round = 0;; ++round) {
        __syncthreads();
        __syncthreads();
        const int n = min(s_ncand[round & 1], P.cap);
        if (static_cast<int>(threadIdx.x) == n_trial * 64) {
          s_ncand[(round + 1) & 1] = 0;
          s_live[(round + 1) % 3] = 0;
        }
        const int s = (wave - n_trial) * 64 + lane;
        if (s < n) {
          Lane<R> S;
          pool_take<R, HB, EXT>(P, s, S, C);
          bool spawn;
          S.state = ST_ACTIVE;
          if (real_collision<R, HB, false, false, EXT>(d, S, C, s_nu, &spawn) == RC_STOP)
            S.state = ST_STOPPED;
          pool_give<R, EXT>(P, s, S);
        }
        __syncthreads();
        if (s_live[round % 3] == 0) break;
      }
    } else {
      // ---- trial waves ----
      const int64_t count = wi.count;
      Lane<R> L;
      L.state = ST_IDLE;
      L.trace_slot = -1;
      L.n_ev = 0;
      int slot = 0;
      for (int round = 0;; ++round) {
        if (L.state == ST_WAIT) pool_back<R, HB, EXT>(P, slot, L, C);   // served last round
        if (L.state == ST_STOPPED) {
          if (L.k >= C.n_coll || (L.flags & 4u)) {
            if (L.k >= C.n_coll) L.flags |= 1u;
            write_record(d, L);
            atomicAdd(reinterpret_cast<unsigned long long*>(&d.ctr->n_done), 1ull);
            if (d.saved != nullptr) d.saved[L.rec].started = 2u;
          } else {
            save_state<R, EXT>(d, L, C, L.rec);
          }
          L.state = ST_IDLE;
        }
        if (L.state == ST_IDLE) {
          const int e = atomicAdd(&s_next, 1);
          if (e < count) {
            const int64_t ei = wi.first + e;
            const uint32_t started = d.saved != nullptr ? d.saved[ei].started : 0u;
            if (started != 2u) {
              L.rec = ei;
              if (started == 1u) load_state<R, HB, EXT>(d, L, C, ei);
              else init_primary<R, HB, EXT>(L, C, s_nu, static_cast<uint64_t>(ei));
              L.k_stop = stop_count(L.k, C);
              L.state = ST_ACTIVE;
            }
          } else {
            L.state = ST_DONE;
          }
        }
        __syncthreads();      // every served electron is back: the pool slots are free
        if (L.state == ST_ACTIVE) trial_block_pooled<R, HB, EXT>(L, C, s_nu);
        // candidates into the pool: one LDS reservation per wave, ranks from the lane mask
        const uint64_t m = __ballot(L.state == ST_CAND);
        if (m != 0) {
          const int leader = __ffsll(static_cast<long long>(m)) - 1;
          int base = 0;
          if (lane == leader) base = atomicAdd(&s_ncand[round & 1], __popcll(m));
          base = __shfl(base, leader);
          if (L.state == ST_CAND) {
            const int s = base + static_cast<int>(__popcll(m & lane_lt));
            if (s < P.cap) {
              pool_put<R, EXT>(P, s, L);
              slot = s;
              L.state = ST_WAIT;
            }
          }
        }
        if (__ballot(L.state != ST_DONE) != 0 && lane == 0) s_live[round % 3] = 1;
        __syncthreads();
        __syncthreads();
        if (s_live[round % 3] == 0) break;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Real-secondaries kernel (one instance, one generation per launch).  Generation 0 is the
// primaries; generation g + 1 is the secondaries that generation g created.  Lanes take
// the electrons of their generation from a global counter and run each to the end of its
// lineage budget.  A secondary is appended to the queue with one atomic per wave (ballot
// of the ionising lanes, prefix rank from the lane mask) and is not touched again in this
// launch: the next launch runs it, so the kernel boundary publishes it and no lane ever
// waits on another.  `first` < 0 selects the primaries [0, count); otherwise the queue
// slots [first, first + count).  A wave takes its electrons in chunks of 64 with one
// atomic and hands them to its idle lanes by ballot rank, and it reads the overflow
// counter once every 64 passes, so no pass waits on device-coherent memory.  With `flush`
// set (the launch after an overflow) every electron is recorded as it was created.
// A launch also resumes the electrons the launch before it parked (park_in, taken first).
// Once all of its electrons are claimed, a wave that is down to park_lanes running lanes or
// fewer, in a launch that has created at least park_min secondaries so far, parks them: each lane
// stops at its next real collision and writes its resumable state to park_out, and the
// next launch runs them together with those secondaries instead of this launch idling
// through their tail.  Parking moves no electron to another stream position, so the
// results do not depend on it.
// ---------------------------------------------------------------------------------------
constexpr uint32_t kClaimChunk = 64;      // electrons a wave takes per claim
constexpr uint32_t kAbortPoll = 64;       // passes between reads of the overflow counter
constexpr uint32_t kParkPoll = 8;         // passes between a parking candidate's reads of the queue tail

// A value the whole wave holds, kept in scalar registers.
__device__ __forceinline__ int64_t wave_uniform(int64_t x) {
  const uint64_t u = static_cast<uint64_t>(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

template <typename R, bool HB, bool TR, int EXT>
__global__ void __launch_bounds__(512) k_swarm_real(const InstanceDesc* __restrict__ desc, int pend_trig,
                                                    int ch_off, int cum_off, int64_t first, int64_t count,
                                                    int flush, const ParkedState* __restrict__ park_in,
                                                    int64_t n_park_in, ParkedState* __restrict__ park_out,
                                                    int64_t park_min, int park_lanes, int64_t tail0) {
  using PT = typename Pair<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  PT* s_nu = reinterpret_cast<PT*>(smem);
  __shared__ double s_logtab[sizeof(R) == 8 ? kUnitLogStride * kUnitLogEntries : 1];
  ChannelDev* s_ch = reinterpret_cast<ChannelDev*>(smem + ch_off);
  const InstanceDesc& d = *desc;
  {
    const PT* src = reinterpret_cast<const PT*>(sizeof(R) == 8 ? static_cast<const void*>(d.nu64)
                                                               : static_cast<const void*>(d.nu32));
    for (int g = threadIdx.x; g <= d.G; g += blockDim.x) {
      PT q = src[g > 0 ? g - 1 : 0];
      if (g == 0) q.y = 0;
      s_nu[g] = q;
    }
    for (int c = threadIdx.x; c < d.nc; c += blockDim.x) s_ch[c] = d.chan[c];
    if constexpr (sizeof(R) == 8)
      for (int j = threadIdx.x; j < kUnitLogStride * kUnitLogEntries; j += blockDim.x) s_logtab[j] = d.logtab[j];
    stage_cum<R>(d, smem, cum_off);
  }
  __syncthreads();
  Consts<R> C = load_consts<R>(d);
  C.chan = s_ch;
  C.logtab = s_logtab;
  if (cum_off >= 0) {
      C.cum = reinterpret_cast<const PT*>(smem + cum_off);
      C.cum_lds = true;
    }
  RunCounters* ctr = d.ctr;
  const int64_t N = d.n_electrons;
  const int64_t child_cap = d.capacity - N;
  Lane<R> L;
  L.state = ST_IDLE;
  L.trace_slot = -1;
  L.n_ev = 0;
  const uint64_t lane_lt = (1ull << __lane_id()) - 1ull;
  // wave-uniform: the wave's chunk [w_next, w_end), whether the generation is exhausted,
  // whether the run is stopping after an overflow, and the pass count
  const int64_t total = n_park_in + count;   // parked electrons first, then the generation's
  int64_t w_next = 0, w_end = 0;
  bool exhausted = false, aborting = flush != 0, parking = false;
  uint32_t pass = 0;
  for (;;) {
    const uint64_t idle = __ballot(L.state == ST_IDLE);
    if (idle != 0) {
      if (w_next >= w_end && !exhausted) {
        const int leader = __ffsll(static_cast<long long>(idle)) - 1;
        unsigned long long base = 0;
        if (static_cast<int>(__lane_id()) == leader)
          base = atomicAdd(reinterpret_cast<unsigned long long*>(&ctr->gen_next),
                           static_cast<unsigned long long>(kClaimChunk));
        w_next = wave_uniform(static_cast<int64_t>(__shfl(base, leader)));
        w_end = min(w_next + static_cast<int64_t>(kClaimChunk), total);
        exhausted = w_next >= total;
      }
      const int64_t avail = max(w_end - w_next, int64_t{0});
      const int64_t rank = static_cast<int64_t>(__popcll(idle & lane_lt));
      const int64_t e = w_next + rank;
      w_next = wave_uniform(min(w_end, w_next + static_cast<int64_t>(__popcll(idle))));
      if (L.state == ST_IDLE && exhausted && avail == 0) L.state = ST_DONE;
      if (L.state == ST_IDLE && rank < avail) {
        if (e < n_park_in) {
          // parked by the launch before, at a real-collision boundary
          const ParkedState ps = park_in[e];
          load_saved<R, HB, EXT>(ps.s, L, C);
          L.rec = ps.rec;
          L.k_stop = C.n_coll;
          L.state = ST_ACTIVE;
        } else if (first < 0) {
          init_primary<R, HB, EXT>(L, C, s_nu, e - n_park_in);
          L.rec = static_cast<int64_t>(e - n_park_in);
          L.k_stop = C.n_coll;
          L.state = ST_ACTIVE;
        } else {
          const int64_t slot = first + static_cast<int64_t>(e - n_park_in);
          const ChildState cs = d.children[slot];
          L.rx = cs.r[0]; L.ry = cs.r[1]; L.rz = cs.r[2];
          L.t = cs.t;
          L.vx = static_cast<R>(cs.v[0]); L.vy = static_cast<R>(cs.v[1]); L.vz = static_cast<R>(cs.v[2]);
          set_id(L, C, cs.id);
          L.k = L.k_start = cs.k;
          L.k_stop = C.n_coll;
          L.block = 0;
          L.G = L.D = L.nforb = L.nover = L.nfirst = L.flags = 0;
          L.se = L.sep = 0.0;
          L.T = R(0);
          L.rec = N + slot;
          set_anchor<R, HB>(L, C);
          start_trial_frequency<R, EXT>(L, C, s_nu, static_cast<R>(cs.eps_birth));
          // a secondary born at its lineage's last collision has nothing left to do
          L.state = L.k >= L.k_stop ? ST_STOPPED : ST_ACTIVE;
        }
        // after an overflow, electrons not yet started are recorded as they are (flag 8)
        if (L.state == ST_ACTIVE && aborting) {
          L.flags |= 8u;
          L.state = ST_STOPPED;
        }
        if constexpr (TR) {
          // a resumed electron goes on with the events it recorded before it was parked
          L.trace_slot = find_trace<TR>(d, L.id);
          L.n_ev = L.trace_slot >= 0 ? d.trace_count[L.trace_slot] : 0;
        }
      }
    }
    // Parking: all of the launch's electrons are claimed, few lanes of the wave still run,
    // and this launch has created enough secondaries for the next one.  The running lanes
    // stop at their next real collision (a ready lane at the one it is about to make).
    if (park_min > 0 && exhausted && !parking && !aborting && pass % kParkPoll == 0) {
      const int running = static_cast<int>(__popcll(__ballot(L.state == ST_ACTIVE || L.state == ST_READY)));
      if (running > 0 && running <= park_lanes) {
        const int64_t made = wave_uniform(static_cast<int64_t>(__hip_atomic_load(
                                              &ctr->child_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) - tail0;
        if (made >= park_min) {
          parking = true;
          if (L.state == ST_ACTIVE || L.state == ST_READY) L.k_stop = min(L.k_stop, L.k + 1u);
        }
      }
    }
    uint64_t ready;
    bool drawing = L.state == ST_ACTIVE;
    for (;;) {
      if (drawing) trial_block<R, HB, EXT>(L, C, s_nu);
      drawing = L.state == ST_ACTIVE;
      ready = __ballot(L.state == ST_READY);
      if (__ballot(drawing) == 0 || static_cast<int>(__popcll(ready)) >= pend_trig) break;
    }
    if (ready != 0) {
      bool spawn = false;
      if (L.state == ST_READY) {
        if (real_collision<R, HB, TR, true, EXT>(d, L, C, s_nu, &spawn) == RC_STOP) L.state = ST_STOPPED;
      }
      // append the secondaries of this wave: one reservation, ranks from the lane mask
      const uint64_t sm = __ballot(spawn);
      if (sm != 0) {
        const int leader = __ffsll(static_cast<long long>(sm)) - 1;
        unsigned long long base = 0;
        if (static_cast<int>(__lane_id()) == leader)
          base = atomicAdd(reinterpret_cast<unsigned long long*>(&ctr->child_tail),
                           static_cast<unsigned long long>(__popcll(sm)));
        base = __shfl(base, leader);
        if (spawn) {
          const int64_t s = static_cast<int64_t>(base + __popcll(sm & lane_lt));
          if (s < child_cap) d.children[s] = make_child<R, EXT>(L, C);
          else atomicAdd(reinterpret_cast<unsigned long long*>(&ctr->dropped), 1ull);
        }
      }
    }
    // Once the queue has overflowed the run's result is an error: stop every electron at
    // its current anchor (flag 8), so the launch ends promptly.  The electrons this
    // generation has not started yet are then recorded unstarted.
    if (!aborting && ++pass % kAbortPoll == 0)
      aborting = __builtin_amdgcn_readfirstlane(static_cast<int>(
                     __hip_atomic_load(&ctr->dropped, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) != 0;
    if (aborting && (L.state == ST_ACTIVE || L.state == ST_READY)) {
      L.flags |= 8u;
      L.state = ST_STOPPED;
    }
    if (L.state == ST_STOPPED) {
      if (parking && L.k < C.n_coll && !(L.flags & 14u)) {
        // parked (not attached, capped or aborted): resumed by the next launch.  The slots
        // stay below parked_capacity of the launch's threads, which the host's buffers hold;
        // past that a lane would run on.
        const uint64_t ps = atomicAdd(reinterpret_cast<unsigned long long*>(&ctr->parked), 1ull);
        if (ps < static_cast<uint64_t>(parked_capacity(static_cast<int64_t>(gridDim.x) * blockDim.x, park_lanes))) {
          ParkedState p;
          p.s = saved_of<R, EXT>(L, C);
          p.rec = L.rec;
          park_out[ps] = p;
          L.state = ST_DONE;
        } else {
          L.k_stop = C.n_coll;
          set_anchor<R, HB>(L, C);
          L.state = ST_ACTIVE;
        }
      } else {
        if (L.k >= C.n_coll && !(L.flags & 10u)) L.flags |= 1u;   // attached or aborted: not finished
        write_record(d, L);
        L.state = ST_IDLE;
      }
    }
    if (__ballot(L.state != ST_DONE) == 0) break;
  }
}

// =======================================================================================
// Tallies: two passes of fixed-tile, fixed-tree FP64 reductions (bitwise reproducible for
// a given record order), then a finishing kernel per instance.
// =======================================================================================

__device__ __forceinline__ void block_sum(double* vals, int nq, double* s_red) {
  // s_red: nq x kTallyThreads doubles.  Fixed pairwise tree over threads.
  for (int q = 0; q < nq; ++q) s_red[q * kTallyThreads + threadIdx.x] = vals[q];
  __syncthreads();
  for (int s = kTallyThreads / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s)
      for (int q = 0; q < nq; ++q)
        s_red[q * kTallyThreads + threadIdx.x] += s_red[q * kTallyThreads + threadIdx.x + s];
    __syncthreads();
  }
}

// pass-1 accumulator indices
enum {
  T1_NF = 0, T1_VX, T1_VY, T1_VZ, T1_AG, T1_AD, T1_ZH, T1_GF, T1_DF,
  T1_KREAL, T1_KNULL, T1_KFORB, T1_KOVER, T1_NATT, T1_NSTUCK, T1_NCREATED, T1_GALL, T1_DALL,
  T1_SE, T1_SEP, T1_NK, T1_PE, T1_PEP, T1_NREC, T1_KFAIL, T1_NRETRY
};
// pass-2 accumulator indices
enum {
  T2_VX = 0, T2_VY, T2_VZ, T2_AG, T2_AD, T2_PE, T2_PEP,
  T2_Q = 7   // then 12 diffusion quantities (paper form 6, vector form 6), value and square
};

__global__ void __launch_bounds__(kTallyThreads) k_tally1(const InstanceDesc* __restrict__ descs,
                                                         const TallyTile* __restrict__ tiles,
                                                         const int32_t* __restrict__ tile_base,
                                                         double* __restrict__ part1) {
  __shared__ double s_red[kTally1 * kTallyThreads];
  const TallyTile tt = tiles[blockIdx.x];
  const InstanceDesc& d = descs[tt.inst];
  double a[kTally1];
  for (int q = 0; q < kTally1; ++q) a[q] = 0.0;
  for (int64_t j = threadIdx.x; j < tt.count; j += kTallyThreads) {
    const swarm_record r = d.records[tt.first + j];
    if (r.id == ~0ull) continue;   // empty slot
    const double kr = static_cast<double>(r.k_end) - static_cast<double>(r.k_start);
    a[T1_NREC] += 1.0;
    a[T1_KREAL] += kr;
    a[T1_KNULL] += static_cast<double>(r.n_null);
    a[T1_KFORB] += static_cast<double>(r.n_forbidden);
    a[T1_KFAIL] += static_cast<double>(r.n_fail);
    a[T1_KOVER] += static_cast<double>(r.n_over);
    a[T1_NATT] += (r.flags & 2u) ? 1.0 : 0.0;
    a[T1_NSTUCK] += (r.flags & 4u) ? 1.0 : 0.0;
    a[T1_NRETRY] += (r.flags & 16u) ? 1.0 : 0.0;
    a[T1_NCREATED] += (r.id >> 63) ? 1.0 : 0.0;
    a[T1_GALL] += static_cast<double>(r.G);
    a[T1_DALL] += static_cast<double>(r.D);
    a[T1_SE] += r.sum_eps;
    a[T1_SEP] += r.sum_epsp;
    if (kr > 0.0) {
      a[T1_NK] += 1.0;
      a[T1_PE] += r.sum_eps / kr;
      a[T1_PEP] += r.sum_epsp / kr;
    }
    if (r.flags & 1u) {
      const double zh = -r.r[2];
      a[T1_NF] += 1.0;
      a[T1_VX] += r.r[0] / r.t;
      a[T1_VY] += r.r[1] / r.t;
      a[T1_VZ] += r.r[2] / r.t;
      a[T1_AG] += static_cast<double>(r.G) / zh;
      a[T1_AD] += static_cast<double>(r.D) / zh;
      a[T1_ZH] += zh;
      a[T1_GF] += static_cast<double>(r.G);
      a[T1_DF] += static_cast<double>(r.D);
    }
  }
  block_sum(a, kTally1, s_red);
  if (threadIdx.x < kTally1)
    part1[(static_cast<int64_t>(tile_base[tt.inst]) + tt.tile) * kTally1 + threadIdx.x] =
        s_red[threadIdx.x * kTallyThreads];
}

// Sum the tiles of each instance in tile order.
__global__ void k_tally_sum(const int32_t* __restrict__ tile_base, const int64_t* __restrict__ nrec,
                            const double* __restrict__ part, int nq, double* __restrict__ tot) {
  const int inst = blockIdx.x;
  const int q = threadIdx.x;
  if (q >= nq) return;
  const int ntiles = static_cast<int>((nrec[inst] + kTallyTile - 1) / kTallyTile);
  double s = 0.0;
  for (int t = 0; t < ntiles; ++t) s += part[(static_cast<int64_t>(tile_base[inst]) + t) * nq + q];
  tot[static_cast<int64_t>(inst) * nq + q] = s;
}

__device__ __forceinline__ void diff6(double dx, double dy, double dz, double t, double* q) {
  const double dz2 = dz * dz, dp2 = dx * dx + dy * dy;
  q[0] = (dz2 + dp2) / t;
  q[1] = dz2 / (2.0 * t);
  q[2] = dp2 / (4.0 * t);
  q[3] = 2.0 * sqrt(dz2 + dp2);
  q[4] = 2.0 * fabs(dz);
  q[5] = 2.0 * sqrt(dp2);
}

__global__ void __launch_bounds__(kTallyThreads) k_tally2(const InstanceDesc* __restrict__ descs,
                                                         const TallyTile* __restrict__ tiles,
                                                         const int32_t* __restrict__ tile_base,
                                                         const double* __restrict__ tot1,
                                                         double* __restrict__ part2) {
  __shared__ double s_red[kTally2 * kTallyThreads];
  const TallyTile tt = tiles[blockIdx.x];
  const InstanceDesc& d = descs[tt.inst];
  const double* t1 = tot1 + static_cast<int64_t>(tt.inst) * kTally1;
  const double nf = t1[T1_NF];
  const double mvx = t1[T1_VX] / nf, mvy = t1[T1_VY] / nf, mvz = t1[T1_VZ] / nf;
  const double mag = t1[T1_AG] / nf, mad = t1[T1_AD] / nf;
  const double mpe = t1[T1_PE] / t1[T1_NK], mpep = t1[T1_PEP] / t1[T1_NK];
  double a[kTally2];
  for (int q = 0; q < kTally2; ++q) a[q] = 0.0;
  for (int64_t j = threadIdx.x; j < tt.count; j += kTallyThreads) {
    const swarm_record r = d.records[tt.first + j];
    if (r.id == ~0ull) continue;   // empty slot
    const double kr = static_cast<double>(r.k_end) - static_cast<double>(r.k_start);
    if (kr > 0.0) {
      const double pe = r.sum_eps / kr - mpe, pep = r.sum_epsp / kr - mpep;
      a[T2_PE] += pe * pe;
      a[T2_PEP] += pep * pep;
    }
    if (r.flags & 1u) {
      const double t = r.t;
      const double vx = r.r[0] / t - mvx, vy = r.r[1] / t - mvy, vz = r.r[2] / t - mvz;
      const double zh = -r.r[2];
      const double ag = static_cast<double>(r.G) / zh - mag, ad = static_cast<double>(r.D) / zh - mad;
      a[T2_VX] += vx * vx;
      a[T2_VY] += vy * vy;
      a[T2_VZ] += vz * vz;
      a[T2_AG] += ag * ag;
      a[T2_AD] += ad * ad;
      double q[6];
      diff6(r.r[0], r.r[1], r.r[2] - t * mvz, t, q);          // paper form: d = x - t W_z z^
      for (int i = 0; i < 6; ++i) { a[T2_Q + i] += q[i]; a[T2_Q + 12 + i] += q[i] * q[i]; }
      diff6(r.r[0] - t * mvx, r.r[1] - t * mvy, r.r[2] - t * mvz, t, q);   // vector form
      for (int i = 0; i < 6; ++i) { a[T2_Q + 6 + i] += q[i]; a[T2_Q + 18 + i] += q[i] * q[i]; }
    }
  }
  block_sum(a, kTally2 - 1, s_red);   // kTally2 - 1 = 31 accumulators used
  if (threadIdx.x < kTally2 - 1)
    part2[(static_cast<int64_t>(tile_base[tt.inst]) + tt.tile) * kTally2 + threadIdx.x] =
        s_red[threadIdx.x * kTallyThreads];
}

__device__ __forceinline__ swarm_stat mk_stat(double mean, double ss_dev, double n) {
  swarm_stat s;
  s.value = mean;
  const double sd = n > 1.0 ? sqrt(ss_dev / (n - 1.0)) : 0.0;
  s.spread = sd;
  s.stat_sigma = n > 0.0 ? sd / sqrt(n) : 0.0;
  return s;
}

__device__ __forceinline__ swarm_stat mk_stat_sq(double sum, double sumsq, double n) {
  const double mean = sum / n;
  double ss = sumsq - sum * mean;
  if (ss < 0.0) ss = 0.0;
  return mk_stat(mean, ss, n);
}

__global__ void k_tally_final(const InstanceDesc* __restrict__ descs, const double* __restrict__ tot1,
                              const double* __restrict__ tot2, swarm_tallies_t* __restrict__ out) {
  const int inst = blockIdx.x;
  if (threadIdx.x != 0) return;
  const InstanceDesc& d = descs[inst];
  const double* a = tot1 + static_cast<int64_t>(inst) * kTally1;
  const double* b = tot2 + static_cast<int64_t>(inst) * kTally2;
  swarm_tallies_t T;
  const double nf = a[T1_NF];
  T.Wx = mk_stat(a[T1_VX] / nf, b[T2_VX], nf);
  T.Wy = mk_stat(a[T1_VY] / nf, b[T2_VY], nf);
  T.Wz = mk_stat(a[T1_VZ] / nf, b[T2_VZ], nf);
  T.W = T.Wz;
  T.W.value = -T.Wz.value;
  const double kreal = a[T1_KREAL];
  T.mean_energy = mk_stat(a[T1_PE] / a[T1_NK], b[T2_PE], a[T1_NK]);
  T.mean_energy_after = mk_stat(a[T1_PEP] / a[T1_NK], b[T2_PEP], a[T1_NK]);
  T.mean_energy.value = a[T1_SE] / kreal;
  T.mean_energy_after.value = a[T1_SEP] / kreal;
  swarm_stat* dst[12] = {&T.D, &T.DL, &T.DT, &T.sigma, &T.sigmaL, &T.sigmaT,
                         &T.D_vec, &T.DL_vec, &T.DT_vec, &T.sigma_vec, &T.sigmaL_vec, &T.sigmaT_vec};
  for (int i = 0; i < 12; ++i) *dst[i] = mk_stat_sq(b[T2_Q + i], b[T2_Q + 12 + i], nf);
  T.alpha = mk_stat(a[T1_AG] / nf, b[T2_AG], nf);
  T.eta = mk_stat(a[T1_AD] / nf, b[T2_AD], nf);
  T.alpha_rate = a[T1_GF] / a[T1_ZH];
  T.eta_rate = a[T1_DF] / a[T1_ZH];
  // efficiency (section "Trial frequency strategies"): real / (real + null + fail), with
  // forbidden picks counted as null trials
  const double trials = kreal + a[T1_KNULL] + a[T1_KFORB] + a[T1_KFAIL];
  T.efficiency = kreal / trials;
  T.majorant = d.majorant;
  T.n_real = static_cast<int64_t>(kreal);
  T.n_null = static_cast<int64_t>(a[T1_KNULL]);
  T.n_forbidden = static_cast<int64_t>(a[T1_KFORB]);
  T.n_fail = static_cast<int64_t>(a[T1_KFAIL]);
  T.n_over = static_cast<int64_t>(a[T1_KOVER]);
  T.n_electrons = static_cast<int64_t>(a[T1_NREC]);
  T.n_finished = static_cast<int64_t>(nf);
  T.n_attached = static_cast<int64_t>(a[T1_NATT]);
  T.n_stuck = static_cast<int64_t>(a[T1_NSTUCK]);
  T.n_created = static_cast<int64_t>(a[T1_NCREATED]);
  T.n_ionizations = static_cast<int64_t>(a[T1_GALL]);
  T.n_attachments = static_cast<int64_t>(a[T1_DALL]);
  T.n_dropped = d.ctr ? static_cast<int64_t>(d.ctr->dropped) : 0;
  T.n_retry_failed = static_cast<int64_t>(a[T1_NRETRY]);
  T.exact = d.trial_strategy == SWARM_TRIAL_CONSTANT ? 1 : 0;
  T.trial_strategy = d.trial_strategy;
  out[inst] = T;
}

template <typename R, bool HB, bool TR>
void* dummy_fn(int ext) {
  return ext == 2 ? reinterpret_cast<void*>(&k_swarm_dummy<R, HB, TR, 2>)
       : ext == 1 ? reinterpret_cast<void*>(&k_swarm_dummy<R, HB, TR, 1>)
                  : reinterpret_cast<void*>(&k_swarm_dummy<R, HB, TR, 0>);
}
template <typename R, bool HB, bool TR>
void* real_fn(int ext) {
  return ext == 2 ? reinterpret_cast<void*>(&k_swarm_real<R, HB, TR, 2>)
       : ext == 1 ? reinterpret_cast<void*>(&k_swarm_real<R, HB, TR, 1>)
                  : reinterpret_cast<void*>(&k_swarm_real<R, HB, TR, 0>);
}

template <typename R, bool HB>
void* pooled_fn(int ext) {
  return ext == 2 ? reinterpret_cast<void*>(&k_swarm_pooled<R, HB, 2>)
       : ext == 1 ? reinterpret_cast<void*>(&k_swarm_pooled<R, HB, 1>)
                  : reinterpret_cast<void*>(&k_swarm_pooled<R, HB, 0>);
}

void* pick_pooled(int precision, bool has_b, int ext) {
  if (precision == SWARM_FP32_MIXED) return has_b ? pooled_fn<float, true>(ext) : pooled_fn<float, false>(ext);
  return has_b ? pooled_fn<double, true>(ext) : pooled_fn<double, false>(ext);
}

void* pick_kernel(int precision, bool has_b, bool trace, bool real, int ext) {
  const bool f32 = precision == SWARM_FP32_MIXED;
#define SW_PICK(R)                                                                            \
  if (real) {                                                                                 \
    if (has_b) return trace ? real_fn<R, true, true>(ext) : real_fn<R, true, false>(ext);     \
    return trace ? real_fn<R, false, true>(ext) : real_fn<R, false, false>(ext);              \
  }                                                                                           \
  if (has_b) return trace ? dummy_fn<R, true, true>(ext) : dummy_fn<R, true, false>(ext);     \
  return trace ? dummy_fn<R, false, true>(ext) : dummy_fn<R, false, false>(ext);
  if (f32) { SW_PICK(float) }
  SW_PICK(double)
#undef SW_PICK
}

}  // namespace

// =======================================================================================
// Host-side launchers.
// =======================================================================================
hipError_t launch_build(InstanceDesc* d_desc, const InstanceDesc& h, hipStream_t s) {
  hipLaunchKernelGGL(k_build_rates, dim3((h.G + 127) / 128), dim3(128), 0, s, d_desc);
  const int64_t n = static_cast<int64_t>(h.G) * h.nc;
  hipLaunchKernelGGL(k_build_pairs, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, d_desc);
  hipLaunchKernelGGL(k_build_constants, dim3(1), dim3(256), 0, s, d_desc);
  if (h.n_bins > 0) hipLaunchKernelGGL(k_build_bins, dim3((h.n_bins + 63) / 64), dim3(64), 0, s, d_desc);
  return hipGetLastError();
}

hipError_t launch_mark_empty(swarm_record* r, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_mark_empty, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, r, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u64, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

size_t swarm_pool_slot_bytes(int precision) {
  const size_t r = precision == SWARM_FP32_MIXED ? sizeof(float) : sizeof(double);
  return kPoolD * sizeof(double) + kPoolR * r + kPoolU * sizeof(uint32_t);
}

hipError_t launch_swarm_dummy(const InstanceDesc* d_desc, const WorkItem* d_items, int32_t n_items,
                              int32_t* d_item_counter, int precision, bool has_b, bool trace,
                              int ext, int service_waves, int block_size, int grid, int pending_trigger,
                              size_t lds_bytes, int ch_off, int pool_off, int cum_off, hipStream_t s) {
  if (service_waves > 0 && !trace) {
    if (service_waves >= block_size / 64) return hipErrorInvalidValue;
    void* fn = pick_pooled(precision, has_b, ext);
    void* args[] = {const_cast<InstanceDesc**>(&d_desc), const_cast<WorkItem**>(&d_items), &n_items,
                    &d_item_counter, &service_waves, &ch_off, &pool_off, &cum_off};
    return hipLaunchKernel(fn, dim3(grid), dim3(block_size), args, lds_bytes, s);
  }
  void* fn = pick_kernel(precision, has_b, trace, false, ext);
  void* args[] = {const_cast<InstanceDesc**>(&d_desc), const_cast<WorkItem**>(&d_items), &n_items,
                  &d_item_counter, &pending_trigger, &ch_off, &cum_off};
  return hipLaunchKernel(fn, dim3(grid), dim3(block_size), args, lds_bytes, s);
}

hipError_t launch_swarm_real(const InstanceDesc* d_desc, int precision, bool has_b, bool trace,
                             int ext, int block_size, int grid, int pending_trigger, size_t lds_bytes,
                             int ch_off, int cum_off, int64_t first, int64_t count, int flush,
                             const ParkedState* park_in, int64_t n_park_in, ParkedState* park_out,
                             int64_t park_min, int park_lanes, int64_t tail0, hipStream_t s) {
  void* fn = pick_kernel(precision, has_b, trace, true, ext);
  void* args[] = {const_cast<InstanceDesc**>(&d_desc), &pending_trigger, &ch_off, &cum_off, &first, &count, &flush,
                  const_cast<ParkedState**>(&park_in), &n_park_in, &park_out, &park_min, &park_lanes, &tail0};
  return hipLaunchKernel(fn, dim3(grid), dim3(block_size), args, lds_bytes, s);
}

hipError_t launch_tallies(const InstanceDesc* d_desc, const TallyTile* d_tiles, int32_t n_tiles,
                          const int32_t* d_tile_base, const int64_t* d_nrec, int32_t n_inst,
                          double* d_part1, double* d_part2, double* d_tot1,
                          swarm_tallies_t* d_out, hipStream_t s) {
  double* d_tot2 = d_tot1 + static_cast<int64_t>(n_inst) * kTally1;
  hipLaunchKernelGGL(k_tally1, dim3(n_tiles), dim3(kTallyThreads), 0, s, d_desc, d_tiles, d_tile_base, d_part1);
  hipLaunchKernelGGL(k_tally_sum, dim3(n_inst), dim3(64), 0, s, d_tile_base, d_nrec, d_part1, kTally1, d_tot1);
  hipLaunchKernelGGL(k_tally2, dim3(n_tiles), dim3(kTallyThreads), 0, s, d_desc, d_tiles, d_tile_base, d_tot1, d_part2);
  hipLaunchKernelGGL(k_tally_sum, dim3(n_inst), dim3(64), 0, s, d_tile_base, d_nrec, d_part2, kTally2, d_tot2);
  hipLaunchKernelGGL(k_tally_final, dim3(n_inst), dim3(64), 0, s, d_desc, d_tot1, d_tot2, d_out);
  return hipGetLastError();
}

int swarm_kernel_max_blocks_per_cu(int precision, bool has_b, bool trace, bool real, int ext,
                                   int service_waves, int block_size, size_t lds_bytes) {
  int n = 0;
  void* fn = service_waves > 0 && !trace && !real ? pick_pooled(precision, has_b, ext)
                                                  : pick_kernel(precision, has_b, trace, real, ext);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn,
                                                   block_size, lds_bytes) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

}  // namespace swarm_impl
