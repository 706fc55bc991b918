// FP64 CPU oracle of the null-collision electron-swarm method of
// "Betaboltz: a Monte-Carlo simulation tool for gas scattering processes"
// (Renda, Ciubotaru, Banu; arXiv 1901.08140).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the HIP path is
// checked against.  Only tests, the smoke check and the benchmark's CPU-baseline leg load
// it; the product library never includes, links or calls it, and it shares no source with
// the HIP path (its own Philox, table extension, grid, mover, kinematics and bookkeeping).
//
// Everything is IEEE binary64, built with -ffp-contract=off, one electron at a time, in
// the order the paper describes the steps.  Where the paper is silent the reading used is
// stated next to the code (the same readings are listed in the design notes).
//
// Parity pins (see tests/test_oracle_*.py): Philox known-answer vectors; closed-form
// free-flight motion (E, E x B, cyclotron); energy conservation in free flight; the
// elastic/inelastic energy formulas against exact two-body kinematics; the table
// extension on power laws; the Maxwell-gas drift velocity eE/(m nu) and mean energy;
// Drude drift with crossed B; diffusion and alpha/eta closed forms for constant rates;
// channel-selection frequencies; the worked example's report identities; the variable trial
// frequency's special cases (cap = constant method, constant rate, no field); anisotropic
// scattering: quadrature of the sampled cos(theta) against sigma_mt/sigma_el and the
// screened-Coulomb closed form, rotation geometry, the Maxwell drift eE/(m nu (1-<cos>)).
// The diffusion magnitudes (sigma, sigma_L, sigma_T) are pinned against an independent
// random walk of the field-free process and its Gaussian limit.  The fail sequences of the
// variable and binned trial frequencies are pinned by plain-Python runs of the strategies'
// steps on the oracle's primitives.  Parity unpinned by a closed form: tallies for the
// synthetic argon/CO2 tables at non-trivial fields; those rest on GPU-vs-oracle parity.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

namespace {

// CODATA 2018 exact/recommended values.
constexpr double kQe = 1.602176634e-19;     // C
constexpr double kMe = 9.1093837015e-31;    // kg
constexpr double kAmu = 1.66053906660e-27;  // kg
constexpr double kPi = 3.14159265358979323846;
constexpr double kHartreeEV = 27.211386245988;   // Hartree energy in eV (CODATA 2018)
constexpr double kKb = 1.380649e-23;         // J/K
constexpr double kC = 299792458.0;           // m/s

enum Kind { ELASTIC = 0, EXCITATION = 1, IONIZATION = 2, ATTACHMENT = 3 };

// ---------------------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).  A round maps
// the counter (c0,c1,c2,c3) with key (k0,k1) to
//   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)),
// with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is advanced by the Weyl constants
// (0x9E3779B9, 0xBB67AE85) between rounds.  Ten rounds.
// ---------------------------------------------------------------------------------------
struct Words { uint32_t w[4]; };

Words philox4x32_10(const uint32_t ctr[4], const uint32_t key[2]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
  Words out;
  for (int i = 0; i < 4; ++i) out.w[i] = c[i];
  return out;
}

// Stream layout: key = (lo32(seed), hi32(seed)); counter = (block, tag, lo32(id), hi32(id)).
enum Tag : uint32_t { TRIAL_HI = 0, TRIAL_LO = 1, SCAT_HI = 2, SCAT_LO = 3, INIT_HI = 4,
                      INIT_LO = 5, CHILD_ID = 6, THERMAL_HI = 7, THERMAL_LO = 8 };

Words stream_block(uint64_t seed, uint64_t id, uint32_t tag, uint32_t block) {
  const uint32_t ctr[4] = {block, tag, static_cast<uint32_t>(id), static_cast<uint32_t>(id >> 32)};
  const uint32_t key[2] = {static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
  return philox4x32_10(ctr, key);
}

// A uniform in [0,1) with 53 random bits: the 32 bits of the HI word on top of the upper
// 21 bits of the LO word.  (Its top 24 bits are the single-precision uniform hi >> 8.)
double uniform53(uint32_t hi, uint32_t lo) {
  const uint64_t m = (static_cast<uint64_t>(hi) << 21) | static_cast<uint64_t>(lo >> 11);
  return static_cast<double>(m) * 0x1.0p-53;
}

struct Vec3 { double x, y, z; };
Vec3 add(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
Vec3 sub(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
Vec3 scale(Vec3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
Vec3 cross(Vec3 a, Vec3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// Isotropic unit vector from two uniforms: cos(Theta) = 1 - 2u, Phi = 2 pi u'.
Vec3 iso_direction(double u_cos, double u_phi) {
  const double ct = 1.0 - 2.0 * u_cos;
  const double st = std::sqrt(std::max(0.0, (1.0 - ct) * (1.0 + ct)));
  const double ph = 2.0 * kPi * u_phi;
  return {st * std::cos(ph), st * std::sin(ph), ct};
}

// Unit vector at angle theta (cos given) and azimuth phi about the unit vector d = (a, b, c),
// by the usual rotation of direction cosines with s = sqrt(a^2 + b^2):
//   (a cos + sin (a c cos phi - b sin phi)/s, b cos + sin (b c cos phi + a sin phi)/s,
//    c cos - s sin cos phi);  for s = 0 (d along z): (sin cos phi, sin sin phi, c cos).
Vec3 rotate_direction(Vec3 d, double cos_t, double phi) {
  const double sin_t = std::sqrt(std::max(0.0, (1.0 - cos_t) * (1.0 + cos_t)));
  const double cp = std::cos(phi), sp = std::sin(phi);
  const double s = std::sqrt(d.x * d.x + d.y * d.y);
  if (s > 0.0) {
    return {d.x * cos_t + sin_t * (d.x * d.z * cp - d.y * sp) / s,
            d.y * cos_t + sin_t * (d.y * d.z * cp + d.x * sp) / s,
            d.z * cos_t - s * sin_t * cp};
  }
  return {sin_t * cp, sin_t * sp, d.z * cos_t};
}

// ---------------------------------------------------------------------------------------
// Gas model.
// ---------------------------------------------------------------------------------------
struct Channel {
  int kind;
  double threshold_eV;
  std::vector<double> e, s;   // raw table points (eV, m^2)
  int component;
  double mass_kg;             // target mass M
  double density;             // n_k = fraction_k * N
  int scattering;             // of its component: 0 isotropic, 1 screened Coulomb, 2 constant xi
  double xi;                  // scattering 2: the anisotropy parameter
  double thermal_sigma;       // moving targets: sqrt(k T / M), each velocity component's spread
};

// Okhrimovskyy anisotropic scattering (section "Theoretical framework", eqs. collision_angle
// and collision_angle_xi).  For molecular gases xi solves
//   sigma_mt / sigma_el = (1 - xi)/(2 xi^2) ((1 + xi) ln((1 + xi)/(1 - xi)) - 2 xi),
// whose right side falls from 1 (xi -> 0, isotropic) to 0 (xi -> 1, forward); the ratio of
// the two cross-sections is taken constant per component (the tables here carry only the
// momentum-transfer cross-section).  Bisection on (0, 1) in binary64.
double mt_over_el_of_xi(double xi) {
  if (xi <= 0.0) return 1.0;
  return (1.0 - xi) / (2.0 * xi * xi) * ((1.0 + xi) * std::log((1.0 + xi) / (1.0 - xi)) - 2.0 * xi);
}
double xi_from_ratio(double r) {
  if (r >= 1.0) return 0.0;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (mt_over_el_of_xi(mid) > r) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// cos(theta) of a scattering from a uniform u in [0,1): isotropic 1 - 2u; screened Coulomb
// for atoms with eps in atomic units (eq. collision_angle); the xi form for molecules
// (eq. collision_angle_xi).
double scatter_cos(int scattering, double xi, double eps_eV, double u) {
  if (scattering == 1) {
    const double e = eps_eV / kHartreeEV;
    return 1.0 - 2.0 * u / (1.0 + 8.0 * e * (1.0 - u));
  }
  if (scattering == 2) return 1.0 - 2.0 * u * (1.0 - xi) / (1.0 + xi * (1.0 - 2.0 * u));
  return 1.0 - 2.0 * u;
}

// Raw cross-section with the paper's table extension (section "Extension of the
// cross-section tables"):
//  * elastic, left of the first point: the first point's value (constant);
//  * inelastic: zero below the threshold; if the table starts above the threshold, the
//    point (threshold, 0) is put in front of it (reading of the truncation rule);
//  * right of the last point: the power law A eps^K through the last two points,
//    K = ln(s2/s1)/ln(e2/e1), A = s2/e2^K (zero if either value is zero);
//  * inside the table: linear interpolation in (eps, sigma).
double sigma_raw(const Channel& ch, double eps) {
  std::vector<double> e = ch.e, s = ch.s;
  if (ch.kind != ELASTIC) {
    if (eps < ch.threshold_eV) return 0.0;
    if (e.front() > ch.threshold_eV) {
      e.insert(e.begin(), ch.threshold_eV);
      s.insert(s.begin(), 0.0);
    }
  }
  const size_t n = e.size();
  if (eps <= e[0]) return s[0];
  if (eps > e[n - 1]) {
    const double e1 = e[n - 2], e2 = e[n - 1], s1 = s[n - 2], s2 = s[n - 1];
    if (!(s1 > 0.0) || !(s2 > 0.0)) return 0.0;
    const double K = std::log(s2 / s1) / std::log(e2 / e1);
    const double A = s2 / std::pow(e2, K);
    return A * std::pow(eps, K);
  }
  // first index i with e[i] >= eps; the segment is [i-1, i]
  size_t i = 1;
  while (e[i] < eps) ++i;
  const double t = (eps - e[i - 1]) / (e[i] - e[i - 1]);
  return s[i - 1] + (s[i] - s[i - 1]) * t;
}

// Speed of an electron of kinetic energy eps (eV; joule inside).  Classically sqrt(2 eps/m),
// the factor of eq. (frequency).  Relativistically |u|/gamma with gamma = 1 + eps/(m c^2)
// and the proper speed |u| = gamma |v| = sqrt(2 eps/m (1 + eps/(2 m c^2))) (from
// gamma^2 - 1 = |u|^2/c^2); this equals c sqrt(1 - 1/gamma^2) without its cancellation.
double proper_speed(double eps, bool rel) {
  const double e = eps * kQe;
  return rel ? std::sqrt(2.0 * e / kMe * (1.0 + e / (2.0 * kMe * kC * kC))) : std::sqrt(2.0 * e / kMe);
}
double speed_of(double eps, bool rel) {
  return rel ? proper_speed(eps, true) / (1.0 + eps * kQe / (kMe * kC * kC)) : proper_speed(eps, false);
}

// Rate of one channel, the summand of the paper's eq. (frequency):
// nu_c(eps) = n_k sigma_c(eps) v(eps), eps converted from eV to joule, v = sqrt(2 eps/m)
// (the relativistic mover takes the electron's true speed).
double rate_raw(const Channel& ch, double eps, bool rel) {
  return ch.density * sigma_raw(ch, eps) * speed_of(eps, rel);
}

struct Params {
  double E, B, B_angle, N, T, eps0;
  int secondaries;  // 0 dummy (counted only), 1 real (children created / electrons removed)
  int grid_P, grid_emin, grid_emax;
  double user_majorant;
  int trial_strategy;   // 0 constant nu' (lazy maximum or fixed), 1 variable (zeta, grace),
                        // 2 binned (bins per decade, grace)
  double zeta;          // variable: nu' = (1 + zeta) nu(eps)
  int64_t grace;        // variable and binned: trials between updates of nu'
  int bins;             // binned: bins per decade of energy
  int thermal;          // 1: targets move (Maxwell-Boltzmann at temperature T), 0: at rest
  int relativistic;     // 1: relativistic motion (B = 0), velocities held as u = gamma v
};

struct Model {
  Params p;
  std::vector<Channel> ch;
  int G;
  std::vector<double> nodes;   // G node energies (eV)
  std::vector<double> C;       // cumulative rate, channel-major: C[c*G + g]
  double majorant;
  std::vector<int> node_bin;   // binned strategy: bin of every node (0 = the bin of node 0)
  std::vector<double> bin_nup; // binned strategy: nu' of every bin
  double node_min, node_max;   // 2^emin, 2^emax
  // field frame
  double omega;                // e B / m
  Vec3 a, bhat, vD;
};

// Octave grid node g = o*P + i has energy 2^(emin+o) * (1 + i/P); node G-1 = 2^emax.
double node_energy(const Params& p, int g) {
  const int o = g / p.grid_P, i = g % p.grid_P;
  return std::ldexp(1.0 + static_cast<double>(i) / p.grid_P, p.grid_emin + o);
}

// Linear interpolation of a node array at eps (the reading of the paper's per-collision
// "linear interpolation" after resampling on the octave grid).  Split eps = 2^(ex-1) (1+f)
// exactly with frexp; i = floor(f P), w = f P - i, g = (ex-1-emin) P + i.
// Below the grid: F[0].  At or above the top node: F[G-1] (counted as over the cap).
// locate() gives the lower node g of the cell holding eps and the weight w (energies below
// the grid: node 0; at or above its top: node G-1; both with w = 0); interp() the value.
int locate(const Model& m, double eps, double* w) {
  *w = 0.0;
  if (eps < m.node_min) return 0;
  if (eps >= m.node_max) return m.G - 1;
  int ex = 0;
  const double mant = std::frexp(eps, &ex);        // eps = mant * 2^ex, mant in [0.5, 1)
  const double f = 2.0 * mant - 1.0;               // in [0, 1), exact
  const double fP = f * m.p.grid_P;                // exact (P is a power of two)
  const double fi = std::floor(fP);
  *w = fP - fi;                                    // exact
  return (ex - 1 - m.p.grid_emin) * m.p.grid_P + static_cast<int>(fi);
}

double interp(const Model& m, const double* F, double eps, bool* over) {
  if (over) *over = eps >= m.node_max;
  double w;
  const int g = locate(m, eps, &w);
  if (eps < m.node_min || eps >= m.node_max) return F[g];
  return F[g] + w * (F[g + 1] - F[g]);
}

double nu_total(const Model& m, double eps, bool* over = nullptr) {
  const int nc = static_cast<int>(m.ch.size());
  return interp(m, &m.C[static_cast<size_t>(nc - 1) * m.G], eps, over);
}

// Free flight in uniform static E and B (classical motion; the paper's
// UniformFieldClassic).  E-frame: z along E, B = |B| (sin th, 0, cos th).  The electron
// charge is -e, so a = -(e/m) E z^ and the velocity rotates as dv/dt = a + omega b^ x v.
//   v(T) = v_par0 + a_par T + vD + u0 cos(wT) + (b^ x u0) sin(wT)
//   r(T) = r0 + (v_par0 + vD) T + a_par T^2/2 + [u0 sin(wT) + (b^ x u0)(1 - cos wT)]/w
// with vD = E x B / B^2 and u0 = v0 - v_par0 - vD;  1 - cos(wT) is taken as 2 sin^2(wT/2).
void move(const Model& m, Vec3 r0, Vec3 v0, double T, Vec3* r, Vec3* v) {
  if (m.p.B == 0.0) {
    if (v) *v = add(v0, scale(m.a, T));
    if (r) *r = add(add(r0, scale(v0, T)), scale(m.a, 0.5 * T * T));
    return;
  }
  const Vec3 b = m.bhat;
  const Vec3 vpar0 = scale(b, dot(v0, b));
  const Vec3 apar = scale(b, dot(m.a, b));
  const Vec3 u0 = sub(sub(v0, vpar0), m.vD);
  const Vec3 bxu = cross(b, u0);
  const double wt = m.omega * T;
  const double c = std::cos(wt), s = std::sin(wt);
  if (v) *v = add(add(add(vpar0, scale(apar, T)), m.vD), add(scale(u0, c), scale(bxu, s)));
  if (r) {
    const double sh = std::sin(0.5 * wt);
    const double one_minus_c = 2.0 * sh * sh;
    Vec3 rr = add(r0, scale(add(vpar0, m.vD), T));
    rr = add(rr, scale(apar, 0.5 * T * T));
    rr = add(rr, scale(add(scale(u0, s), scale(bxu, one_minus_c)), 1.0 / m.omega));
    *r = rr;
  }
}

double energy_eV(Vec3 v) { return 0.5 * kMe * dot(v, v) / kQe; }

// Relativistic motion in a uniform static E (the paper's UniformFieldRelativisticChin with
// B = 0), in the proper velocity u = gamma v: u(T) = u0 + a T with a = -(e/m) E z^ (from dp/dt
// = -e E), and the position is the time integral of u/gamma, gamma = sqrt(1 + |u|^2/c^2):
//   z(T) = z0 + c^2 (gamma(T) - gamma0) / a        (the work of the field)
//        = z0 + (u_z0 + u_z(T)) T / (gamma0 + gamma(T))
//   (gamma(T)^2 - gamma0^2 = (u_z(T)^2 - u_z0^2)/c^2 and u_z(T) - u_z0 = a T), and across E,
//   with gamma = sqrt(A^2 + u_z^2)/c, A^2 = c^2 + u_x^2 + u_y^2,
//   x(T) = x0 + u_x (c/a) (asinh(u_z(T)/A) - asinh(u_z0/A))   (likewise y);
// without a field the motion is straight, r0 + u0 T / gamma0.
void move_rel(const Model& m, Vec3 r0, Vec3 u0, double T, Vec3* r, Vec3* u) {
  const double a = m.a.z;
  const Vec3 uT{u0.x, u0.y, u0.z + a * T};
  if (u) *u = uT;
  if (!r) return;
  const double c2 = kC * kC;
  const double g0 = std::sqrt(1.0 + dot(u0, u0) / c2), g1 = std::sqrt(1.0 + dot(uT, uT) / c2);
  if (a == 0.0) {
    *r = add(r0, scale(u0, T / g0));
    return;
  }
  const double A = std::sqrt(c2 + u0.x * u0.x + u0.y * u0.y);
  const double s = kC / a * (std::asinh(uT.z / A) - std::asinh(u0.z / A));
  *r = {r0.x + u0.x * s, r0.y + u0.y * s, r0.z + (u0.z + uT.z) * T / (g0 + g1)};
}

// Relativistic motion in uniform static E and B (the paper's UniformFieldRelativisticChin):
// in proper time tau the 4-velocity Y = (w, u) = (gamma c, gamma v) obeys the linear system
// dY/dtau = M Y, with (charge -e)
//   M (w, u) = k (E.u / c, E w / c + u x B),  k = -e/m,
// so Y(tau) = exp(M tau) Y0 and the 4-position X(tau) = X0 + (integral of exp(M s) ds from
// 0 to tau) Y0, X = (c t, r).  Both come from one exponential of the 8x8 block matrix
// [[M tau, I tau], [0, 0]] (Van Loan), whose upper blocks are exp(M tau) and the integral.
// The exponential is the Taylor series after scaling by 2^-s (squared back s times).  The
// proper time of a flight of laboratory duration T solves c t(tau) = c T, by Newton's method
// (d(c t)/dtau = w > 0).
void expm8(const double A[8][8], double E8[8][8]) {
  double nrm = 0.0;
  for (int i = 0; i < 8; ++i) {
    double row = 0.0;
    for (int j = 0; j < 8; ++j) row += std::fabs(A[i][j]);
    nrm = std::max(nrm, row);
  }
  int s = 0;
  while (nrm > 0.25) { nrm *= 0.5; ++s; }
  const double scale_ = std::ldexp(1.0, -s);
  double B[8][8], term[8][8], sum[8][8], tmp[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      B[i][j] = A[i][j] * scale_;
      term[i][j] = (i == j) ? 1.0 : 0.0;
      sum[i][j] = term[i][j];
    }
  for (int n = 1; n <= 24; ++n) {
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        double acc = 0.0;
        for (int l = 0; l < 8; ++l) acc += term[i][l] * B[l][j];
        tmp[i][j] = acc / n;
      }
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        term[i][j] = tmp[i][j];
        sum[i][j] += term[i][j];
      }
  }
  for (int q = 0; q < s; ++q) {
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        double acc = 0.0;
        for (int l = 0; l < 8; ++l) acc += sum[i][l] * sum[l][j];
        tmp[i][j] = acc;
      }
    std::memcpy(sum, tmp, sizeof(sum));
  }
  std::memcpy(E8, sum, sizeof(sum));
}

void move_rel_eb(const Model& m, Vec3 r0, Vec3 u0, double T, Vec3* r, Vec3* u) {
  const double k = -kQe / kMe;
  const Vec3 E{0.0, 0.0, m.p.E};
  const Vec3 B = scale(m.bhat, m.p.B);
  // the generator M on (w, u_x, u_y, u_z)
  double M[4][4] = {{0.0, k * E.x / kC, k * E.y / kC, k * E.z / kC},
                    {k * E.x / kC, 0.0, k * B.z, -k * B.y},
                    {k * E.y / kC, -k * B.z, 0.0, k * B.x},
                    {k * E.z / kC, k * B.y, -k * B.x, 0.0}};
  const double Y0[4] = {kC * std::sqrt(1.0 + dot(u0, u0) / (kC * kC)), u0.x, u0.y, u0.z};
  double E8[8][8];
  auto eval = [&](double tau) {
    double A[8][8] = {};
    for (int i = 0; i < 4; ++i) {
      for (int j = 0; j < 4; ++j) A[i][j] = M[i][j] * tau;
      A[i][4 + i] = tau;
    }
    expm8(A, E8);
  };
  // The proper time of the flight solves f(tau) = c t(tau) - c T = 0 with tau in [0, T] (dt/dtau
  // = gamma >= 1), f increasing (f' = w > 0).  Newton's method from T/gamma0, safeguarded: a
  // bisection step of the bracket whenever the Newton step would leave it or would not halve
  // the step before (in a strong E, gamma grows like exp(l tau) and Newton alone crawls down
  // from a far guess), or the exponential overflows.
  double lo = 0.0, hi = T, tau = std::min(T * kC / Y0[0], T), step_old = T, step = T;
  auto f_w = [&](double t, double* f, double* w) {
    eval(t);
    double ct = 0.0, ww = 0.0;
    for (int j = 0; j < 4; ++j) {
      ct += E8[0][4 + j] * Y0[j];
      ww += E8[0][j] * Y0[j];
    }
    *f = ct - kC * T;
    *w = ww;
    return std::isfinite(*f) && std::isfinite(*w) && *w > 0.0;
  };
  double f, w;
  bool ok = f_w(tau, &f, &w);
  for (int it = 0; it < 400 && T > 0.0; ++it) {
    if (!ok || f > 0.0) hi = tau; else lo = tau;
    const double newton = ok ? tau - f / w : -1.0;
    if (!ok || !(newton >= lo && newton <= hi) || std::fabs(2.0 * f) > std::fabs(step_old * w)) {
      step_old = step;
      step = 0.5 * (hi - lo);
      tau = lo + step;
    } else {
      step_old = step;
      step = tau - newton;
      tau = newton;
    }
    if (std::fabs(step) <= 1e-12 * tau || hi - lo <= 1e-15 * hi) break;
    ok = f_w(tau, &f, &w);
  }
  eval(tau);
  double Y[4] = {}, X[4] = {};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      Y[i] += E8[i][j] * Y0[j];
      X[i] += E8[i][4 + j] * Y0[j];
    }
  if (u) *u = {Y[1], Y[2], Y[3]};
  if (r) *r = {r0.x + X[1], r0.y + X[2], r0.z + X[3]};
}

// Kinetic energy (eV) of the velocity held: classically m |v|^2 / 2; relativistically
// (gamma - 1) m c^2 = m |u|^2 / (gamma + 1), gamma = sqrt(1 + |u|^2/c^2).
double kinetic_eV(Vec3 u, bool rel) {
  if (!rel) return energy_eV(u);
  const double u2 = dot(u, u);
  return kMe * u2 / (std::sqrt(1.0 + u2 / (kC * kC)) + 1.0) / kQe;
}

// Motion of either mover.
void advance(const Model& m, Vec3 r0, Vec3 v0, double T, Vec3* r, Vec3* v) {
  if (m.p.relativistic && m.p.B > 0.0) move_rel_eb(m, r0, v0, T, r, v);
  else if (m.p.relativistic) move_rel(m, r0, v0, T, r, v);
  else move(m, r0, v0, T, r, v);
}

// Energy after an elastic collision (Fraser-Mathieson, the paper's eq. delta_energy_ela).
double energy_after_elastic(double eps, double cos_t, double M) {
  const double m = kMe;
  return eps * (1.0 - 2.0 * m * M * (1.0 - cos_t) / ((m + M) * (m + M)));
}

// Energy after an inelastic collision with threshold eps_k (eq. delta_energy_ine).
// The square-root argument is clamped at zero; the caller has already rejected events
// below the kinematic onset eps_k (m+M)/M.
double energy_after_inelastic(double eps, double eps_k, double cos_t, double M) {
  const double m = kMe;
  const double ratio = eps_k / eps;
  const double root = std::sqrt(std::max(0.0, 1.0 - (m + M) / M * ratio));
  return eps * (1.0 - M / (m + M) * ratio + 2.0 * m * M / ((m + M) * (m + M)) * (root * cos_t - 1.0));
}

// Velocity of the target in a collision with moving targets (section "Effect of gas
// temperature"): the gas molecules have the Maxwell-Boltzmann distribution of temperature T,
// so each Cartesian component is normal with standard deviation sigma = sqrt(k T / M).  The
// three normals come from four uniforms by the Box-Muller transform.
Vec3 target_velocity(double sigma, double u0, double u1, double u2, double u3) {
  const double r01 = std::sqrt(-2.0 * std::log(1.0 - u0));
  const double r23 = std::sqrt(-2.0 * std::log(1.0 - u2));
  return {sigma * r01 * std::cos(2.0 * kPi * u1), sigma * r01 * std::sin(2.0 * kPi * u1),
          sigma * r23 * std::cos(2.0 * kPi * u3)};
}

// The paper's equation for the electron (V1') in a collision with a target moving at V2:
// with Vcm = (m V1 + M V2)/(m + M), the electron's speed in the centre-of-momentum frame
// |V1 - Vcm| becomes sqrt(|V1 - Vcm|^2 - 2 eps_k M / ((m + M) m)), in the direction u_hat
// there.  cm_speed2() is the argument of that root: negative when the energy in that frame is
// below the threshold eps_k (joule), and the process cannot happen.
double cm_speed2(Vec3 V1, Vec3 Vcm, double M, double eps_k_J) {
  const Vec3 u1 = sub(V1, Vcm);
  return dot(u1, u1) - 2.0 * eps_k_J / (kMe + M) * (M / kMe);
}
Vec3 centre_of_momentum(Vec3 V1, Vec3 V2, double M) {
  return scale(add(scale(V1, kMe), scale(V2, M)), 1.0 / (kMe + M));
}

// ---------------------------------------------------------------------------------------
// Per-electron simulation.
// ---------------------------------------------------------------------------------------
// FLAG_RETRY_FAILED: a binned-strategy retry failed again before its next real collision or
// renewal, where the paper throws.  The electron goes on with the constant nu' instead.
constexpr uint32_t FLAG_FINISHED = 1, FLAG_ATTACHED = 2, FLAG_STUCK = 4, FLAG_RETRY_FAILED = 16;
constexpr uint64_t kMaxBlocks = 0x7fffffffull;   // per-electron cap on trial blocks
constexpr int EV_REAL = 1, EV_FORBIDDEN = 2, EV_FAIL = 3;

struct Record {
  uint64_t id;
  uint32_t flags, k_start, k_end, G, D, n_forbidden, n_over, n_fail;
  uint64_t n_null, blocks;
  double r[3], t, sum_eps, sum_epsp;
};

struct Event {
  uint64_t id;
  int32_t type, channel;
  uint32_t k, block, sub, pad;
  double eps, epsp, t, r[3];
};

struct Electron {
  uint64_t id;
  Vec3 r, v;
  double t;
  uint32_t k;
  double eps_birth;   // energy it was created with (eV): the initial energy or eps'/2
};

struct RunCtx {
  const Model* m;
  uint64_t seed;
  uint32_t n_coll;
  std::vector<uint64_t> trace_ids;
  int max_events;
  std::atomic<int64_t>* created;
  int64_t capacity;
  std::atomic<int>* capacity_error;
};

// The paper's VariableTrialFrequency (section "Trial frequency strategies"): a new trial
// frequency nu' = (1 + zeta) nu(eps) from the total rate at the current energy.  It is
// capped at the constant (lazy) maximum, which can never fail, so repeated fails end.
double variable_nup(const Model& m, double nu) { return std::min((1.0 + m.p.zeta) * nu, m.majorant); }

// The paper's BinnedTrialFrequency: the energy axis is cut into bins, b per decade, bin k
// holding [10^(k/b), 10^((k+1)/b)) eV.  A grid cell belongs to the bin of its lower node, so
// each bin is a run of whole cells, and its nu' is the largest total rate on those cells
// (the rate is linear on a cell: the larger of its two end nodes), raised by 2^-20 as for
// the constant strategy and capped at the constant value.
int decade_bin(double eps, int b) { return static_cast<int>(std::floor(b * std::log10(eps))); }

int bin_of(const Model& m, double eps) {
  double w;
  return m.node_bin[locate(m, eps, &w)];
}

double binned_nup(const Model& m, double eps) { return m.bin_nup[bin_of(m, eps)]; }

// After a fail the electron retries from its last real collision with the largest nu' of
// the bins from the one of that collision's energy to the one where the trial failed.
double binned_retry_nup(const Model& m, double eps_anchor, double eps_fail) {
  const int a = bin_of(m, eps_anchor), f = bin_of(m, eps_fail);
  double v = 0.0;
  for (int k = std::min(a, f); k <= std::max(a, f); ++k) v = std::max(v, m.bin_nup[k]);
  return v;
}

bool traced(const RunCtx& cx, uint64_t id) {
  return std::find(cx.trace_ids.begin(), cx.trace_ids.end(), id) != cx.trace_ids.end();
}

// One electron from its birth state until it has made n_coll real collisions (counting
// the ones inherited from its lineage), is attached (real secondaries mode) or exceeds the
// block cap.  Children (real secondaries mode) are appended to `children`.
Record simulate(const RunCtx& cx, const Electron& e0, std::vector<Electron>& children,
                std::vector<Event>& events) {
  const Model& m = *cx.m;
  const int nc = static_cast<int>(m.ch.size());
  // Trial frequency: constant (lazy maximum or the user's fixed value), or the variable or
  // binned strategy: the first value from the birth energy, then updated after every
  // `grace` trials (from the energy after the trial that used up the grace) and after every
  // fail.
  const bool variable = m.p.trial_strategy == 1;
  const bool binned = m.p.trial_strategy == 2;
  const bool adaptive = variable || binned;
  double nup = variable ? variable_nup(m, nu_total(m, e0.eps_birth))
             : binned ? binned_nup(m, e0.eps_birth) : m.majorant;
  int64_t grace = m.p.grace;
  bool retry = false;        // binned: nu' set by a fail, no real collision or renewal since
  auto renew = [&](double eps_now, double nu_now) {
    nup = binned ? binned_nup(m, eps_now) : variable_nup(m, nu_now);
    grace = m.p.grace;
    retry = false;
  };
  Record rec{};
  rec.id = e0.id;
  rec.k_start = e0.k;
  Vec3 r = e0.r, v = e0.v;   // anchor: state right after the last real collision
  double t = e0.t;
  double T = 0.0;            // flight time since the anchor
  uint32_t k = e0.k;
  uint64_t block = 0;
  const bool tr = !cx.trace_ids.empty() && traced(cx, e0.id);
  int n_ev = 0;
  bool alive = true;

  while (alive && k < cx.n_coll) {
    if (block >= kMaxBlocks) { rec.flags |= FLAG_STUCK; break; }
    const uint32_t blk = static_cast<uint32_t>(block);
    const Words hi = stream_block(cx.seed, e0.id, TRIAL_HI, blk);
    const Words lo = stream_block(cx.seed, e0.id, TRIAL_LO, blk);
    ++block;
    ++rec.blocks;
    // A block holds two candidate trials; a non-null outcome (real or forbidden) of the
    // first ends the block and its second trial is not used.
    for (int sub = 0; sub < 2; ++sub) {
      const double u_f = uniform53(hi.w[2 * sub], lo.w[2 * sub]);
      const double u_r = uniform53(hi.w[2 * sub + 1], lo.w[2 * sub + 1]);
      // Flight time against the trial frequency nu' (eq. random_time).
      T += -std::log(1.0 - u_f) / nup;
      Vec3 vT;
      advance(m, r, v, T, nullptr, &vT);
      const double eps = kinetic_eV(vT, m.p.relativistic);
      bool over = false;
      const double nu = nu_total(m, eps, &over);
      if (adaptive && nu > nup) {
        // Fail: nu(eps) <= nu' does not hold just before the candidate.  The electron goes
        // back to the state of its last real collision (the anchor: T = 0), a new nu' comes
        // from the rate that failed (variable) or from the bins between the anchor and the
        // failing energy (binned), and the grace count restarts.  The fail uses up its trial
        // and ends the block.
        ++rec.n_fail;
        if (tr && n_ev < cx.max_events) {
          Event ev{};
          ev.id = e0.id; ev.type = EV_FAIL; ev.channel = -1; ev.k = k;
          ev.block = blk; ev.sub = sub; ev.eps = eps; ev.epsp = eps;
          ev.t = t + T; ev.r[0] = r.x; ev.r[1] = r.y; ev.r[2] = r.z;
          events.push_back(ev);
          ++n_ev;
        }
        T = 0.0;
        if (binned) {
          if (retry) {
            rec.flags |= FLAG_RETRY_FAILED;
            nup = m.majorant;
          } else {
            nup = binned_retry_nup(m, kinetic_eV(v, m.p.relativistic), eps);
          }
          retry = true;
        } else {
          nup = variable_nup(m, nu);
        }
        grace = m.p.grace;
        break;
      }
      // Null test (eq. null_fraction): null when R > nu(eps)/nu'; here real iff
      // R nu' < nu(eps) (strict), with the same R choosing the channel below.
      const double x = u_r * nup;
      if (!(x < nu)) {
        ++rec.n_null;
        if (adaptive && --grace == 0) renew(eps, nu);
        continue;
      }
      int c = 0;
      while (c < nc - 1 && !(x < interp(m, &m.C[static_cast<size_t>(c) * m.G], eps, nullptr))) ++c;
      const Channel& chn = m.ch[c];
      const double M = chn.mass_kg;
      const double eps_k_J = (chn.kind == EXCITATION || chn.kind == IONIZATION) ? chn.threshold_eV * kQe : 0.0;
      // Moving targets: the target velocity of this collision (THERMAL block k) and the
      // electron's squared speed in the centre-of-momentum frame after the threshold loss.
      Vec3 Vcm{0.0, 0.0, 0.0};
      double g2 = 0.0;
      if (m.p.thermal) {
        const Words th = stream_block(cx.seed, e0.id, THERMAL_HI, k);
        const Words tl = stream_block(cx.seed, e0.id, THERMAL_LO, k);
        const Vec3 V2 = target_velocity(chn.thermal_sigma, uniform53(th.w[0], tl.w[0]), uniform53(th.w[1], tl.w[1]),
                                        uniform53(th.w[2], tl.w[2]), uniform53(th.w[3], tl.w[3]));
        Vcm = centre_of_momentum(vT, V2, M);
        g2 = cm_speed2(vT, Vcm, M, eps_k_J);
      }
      const bool forbidden =
          m.p.thermal ? (chn.kind != ATTACHMENT && g2 < 0.0)
                      : ((chn.kind == EXCITATION || chn.kind == IONIZATION) &&
                         eps < chn.threshold_eV * ((kMe + M) / M));
      if (forbidden) {
        // Kinematically forbidden: just above threshold (grid smearing), or with moving
        // targets below the threshold in the centre-of-momentum frame.  Treated as null.
        ++rec.n_forbidden;
        if (adaptive && --grace == 0) renew(eps, nu);
        if (tr && n_ev < cx.max_events) {
          Event ev{};
          ev.id = e0.id; ev.type = EV_FORBIDDEN; ev.channel = c; ev.k = k;
          ev.block = blk; ev.sub = sub; ev.eps = eps; ev.epsp = eps;
          ev.t = t + T; ev.r[0] = r.x; ev.r[1] = r.y; ev.r[2] = r.z;
          events.push_back(ev);
          ++n_ev;
        }
        break;
      }
      // Real collision.
      if (over) ++rec.n_over;
      Vec3 rT;
      advance(m, r, v, T, &rT, nullptr);
      const Words sh = stream_block(cx.seed, e0.id, SCAT_HI, k);
      const Words sl = stream_block(cx.seed, e0.id, SCAT_LO, k);
      const double v2 = dot(vT, vT);
      Vec3 n;
      double cos_t = 0.0;
      double epsp;
      if (m.p.thermal) {
        // Moving target: the new direction in the centre-of-momentum frame (isotropic, or
        // theta about the incoming relative direction), then back to the laboratory.
        const Vec3 u1 = ::sub(vT, Vcm);   // (the block loop's `sub` hides the function)
        const double g = std::sqrt(dot(u1, u1));
        Vec3 uh;
        if (chn.scattering == 0 || !(g > 0.0)) {
          uh = iso_direction(uniform53(sh.w[0], sl.w[0]), uniform53(sh.w[1], sl.w[1]));
        } else {
          cos_t = scatter_cos(chn.scattering, chn.xi, eps, uniform53(sh.w[0], sl.w[0]));
          uh = rotate_direction(scale(u1, 1.0 / g), cos_t, 2.0 * kPi * uniform53(sh.w[1], sl.w[1]));
        }
        const Vec3 V1p = add(Vcm, scale(uh, std::sqrt(std::max(g2, 0.0))));
        const double s1 = std::sqrt(dot(V1p, V1p));
        n = s1 > 0.0 ? scale(V1p, 1.0 / s1) : uh;
        epsp = chn.kind == ATTACHMENT ? 0.0 : energy_eV(V1p);
      } else if (chn.scattering == 0 || !(v2 > 0.0)) {
        // isotropic in the lab frame; theta is the angle to the incoming velocity
        n = iso_direction(uniform53(sh.w[0], sl.w[0]), uniform53(sh.w[1], sl.w[1]));
        cos_t = v2 > 0.0 ? dot(n, vT) / std::sqrt(v2) : 0.0;
      } else {
        // anisotropic: theta about the incoming direction, azimuth 2 pi u'
        cos_t = scatter_cos(chn.scattering, chn.xi, eps, uniform53(sh.w[0], sl.w[0]));
        n = rotate_direction(scale(vT, 1.0 / std::sqrt(v2)), cos_t, 2.0 * kPi * uniform53(sh.w[1], sl.w[1]));
      }
      if (m.p.thermal) {
        // (epsp set above)
      } else if (chn.kind == ELASTIC) {
        epsp = energy_after_elastic(eps, cos_t, M);
      } else if (chn.kind == ATTACHMENT) {
        epsp = 0.0;   // plastic collision: all the energy is transferred
      } else {
        epsp = energy_after_inelastic(eps, chn.threshold_eV, cos_t, M);
      }
      epsp = std::max(epsp, 0.0);
      rec.sum_eps += eps;
      if (chn.kind == IONIZATION) {
        epsp *= 0.5;   // equal sharing with the ejected electron
        ++rec.G;
        if (m.p.secondaries == 1) {
          const Words cw = stream_block(cx.seed, e0.id, CHILD_ID, k);
          Electron child;
          child.id = (static_cast<uint64_t>(cw.w[0]) | (static_cast<uint64_t>(cw.w[1]) << 32)) |
                     (1ull << 63);
          child.r = rT;
          child.t = t + T;
          child.k = k + 1;
          child.v = scale(iso_direction(uniform53(sh.w[2], sl.w[2]), uniform53(sh.w[3], sl.w[3])),
                          proper_speed(epsp, m.p.relativistic));
          child.eps_birth = epsp;
          const int64_t n_created = cx.created->fetch_add(1) + 1;
          if (n_created > cx.capacity) {
            cx.capacity_error->store(1);
          } else {
            children.push_back(child);
          }
        }
      } else if (chn.kind == ATTACHMENT) {
        ++rec.D;
        if (m.p.secondaries == 1) alive = false;
      }
      rec.sum_epsp += epsp;
      if (tr && n_ev < cx.max_events) {
        Event ev{};
        ev.id = e0.id; ev.type = EV_REAL; ev.channel = c; ev.k = k;
        ev.block = blk; ev.sub = sub; ev.eps = eps; ev.epsp = epsp;
        ev.t = t + T; ev.r[0] = rT.x; ev.r[1] = rT.y; ev.r[2] = rT.z;
        events.push_back(ev);
        ++n_ev;
      }
      ++k;
      r = rT;
      t += T;
      T = 0.0;
      v = scale(n, proper_speed(epsp, m.p.relativistic));
      retry = false;
      if (adaptive && --grace == 0) renew(epsp, nu_total(m, epsp));
      break;
    }
  }
  rec.k_end = k;
  if (!alive) rec.flags |= FLAG_ATTACHED;
  else if (k >= cx.n_coll) rec.flags |= FLAG_FINISHED;
  rec.r[0] = r.x; rec.r[1] = r.y; rec.r[2] = r.z;
  rec.t = t;
  return rec;
}

Electron primary(const Model& m, uint64_t seed, uint64_t id) {
  const Words hi = stream_block(seed, id, INIT_HI, 0);
  const Words lo = stream_block(seed, id, INIT_LO, 0);
  Electron e;
  e.id = id;
  e.r = {0.0, 0.0, 0.0};
  e.t = 0.0;
  e.k = 0;
  e.v = scale(iso_direction(uniform53(hi.w[0], lo.w[0]), uniform53(hi.w[1], lo.w[1])),
              proper_speed(m.p.eps0, m.p.relativistic));
  e.eps_birth = m.p.eps0;
  return e;
}

struct RunResult {
  std::vector<Record> records;
  std::vector<Event> events;
  int status;
};

}  // namespace

// =======================================================================================
// C ABI used by the Python wrapper (oracle/__init__.py).
// =======================================================================================
extern "C" {

struct or_channel { int32_t kind; double threshold_eV; int32_t n_points; const double* energy_eV;
                    const double* sigma_m2; };
struct or_component { double mass_amu; double fraction; int32_t n_channels; const or_channel* channels;
                      int32_t scattering; double mt_over_el; };
struct or_params { double E_V_per_m, B_T, B_angle_rad, N_per_m3, T_K, init_energy_eV;
                   int32_t secondaries, grid_P, grid_emin, grid_emax; double user_majorant;
                   int32_t trial_strategy; double trial_zeta; int64_t trial_grace;
                   int32_t trial_bins; int32_t thermal_targets; int32_t relativistic; };

enum { OR_OK = 0, OR_INVALID = -1, OR_CAPACITY = -3 };

void or_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  const Words w = philox4x32_10(ctr, key);
  for (int i = 0; i < 4; ++i) out[i] = w.w[i];
}

void or_stream_block(uint64_t seed, uint64_t id, uint32_t tag, uint32_t block, uint32_t* out) {
  const Words w = stream_block(seed, id, tag, block);
  for (int i = 0; i < 4; ++i) out[i] = w.w[i];
}

double or_uniform53(uint32_t hi, uint32_t lo) { return uniform53(hi, lo); }

void* or_create(const or_component* comps, int32_t n_comps, const or_params* p, int32_t* status) {
  *status = OR_INVALID;
  if (!comps || n_comps <= 0 || !p) return nullptr;
  if (!(p->N_per_m3 > 0.0) || !(p->E_V_per_m >= 0.0) || !(p->B_T >= 0.0) || !(p->init_energy_eV >= 0.0))
    return nullptr;
  if (p->grid_P <= 0 || (p->grid_P & (p->grid_P - 1)) != 0 || p->grid_emax <= p->grid_emin) return nullptr;
  if (p->trial_strategy < 0 || p->trial_strategy > 2) return nullptr;
  if (p->trial_strategy == 1 && (!(p->trial_zeta > 0.0) || !std::isfinite(p->trial_zeta) || p->trial_grace < 1))
    return nullptr;
  if (p->trial_strategy == 2 && (p->trial_bins < 1 || p->trial_bins > 100 || p->trial_grace < 1)) return nullptr;
  if (p->thermal_targets < 0 || p->thermal_targets > 1 || !(p->T_K >= 0.0) || !std::isfinite(p->T_K)) return nullptr;
  // the relativistic mover, not with moving targets (whose kinematics take laboratory
  // velocities)
  if (p->relativistic < 0 || p->relativistic > 1) return nullptr;
  if (p->relativistic && p->thermal_targets) return nullptr;
  double fsum = 0.0;
  auto* m = new Model();
  m->p = {p->E_V_per_m, p->B_T, p->B_angle_rad, p->N_per_m3, p->T_K, p->init_energy_eV,
          p->secondaries, p->grid_P, p->grid_emin, p->grid_emax, p->user_majorant,
          p->trial_strategy, p->trial_zeta, p->trial_grace, p->trial_bins, p->thermal_targets,
          p->relativistic};
  for (int k = 0; k < n_comps; ++k) {
    const or_component& c = comps[k];
    if (!(c.mass_amu > 0.0) || !(c.fraction >= 0.0) || c.n_channels <= 0) { delete m; return nullptr; }
    if (c.scattering < 0 || c.scattering > 2) { delete m; return nullptr; }
    if (c.scattering == 2 && !(c.mt_over_el > 0.0 && c.mt_over_el <= 1.0)) { delete m; return nullptr; }
    const double xi = c.scattering == 2 ? xi_from_ratio(c.mt_over_el) : 0.0;
    fsum += c.fraction;
    for (int j = 0; j < c.n_channels; ++j) {
      const or_channel& q = c.channels[j];
      if (q.n_points < 2 || q.kind < 0 || q.kind > 3 || !(q.threshold_eV >= 0.0)) { delete m; return nullptr; }
      Channel ch;
      ch.kind = q.kind;
      ch.threshold_eV = q.threshold_eV;
      ch.e.assign(q.energy_eV, q.energy_eV + q.n_points);
      ch.s.assign(q.sigma_m2, q.sigma_m2 + q.n_points);
      for (int i = 0; i < q.n_points; ++i) {
        if (!(ch.e[i] > 0.0) || !std::isfinite(ch.e[i]) || !(ch.s[i] >= 0.0) || !std::isfinite(ch.s[i])) {
          delete m; return nullptr;
        }
        if (i > 0 && !(ch.e[i] > ch.e[i - 1])) { delete m; return nullptr; }
      }
      ch.component = k;
      ch.scattering = c.scattering;
      ch.xi = xi;
      ch.mass_kg = c.mass_amu * kAmu;
      ch.density = c.fraction * p->N_per_m3;
      ch.thermal_sigma = std::sqrt(kKb * p->T_K / ch.mass_kg);
      m->ch.push_back(std::move(ch));
    }
  }
  if (std::fabs(fsum - 1.0) > 1e-9) { delete m; return nullptr; }
  const int nc = static_cast<int>(m->ch.size());
  m->G = (p->grid_emax - p->grid_emin) * p->grid_P + 1;
  m->nodes.resize(m->G);
  m->C.assign(static_cast<size_t>(nc) * m->G, 0.0);
  double numax = 0.0;
  for (int g = 0; g < m->G; ++g) {
    const double eps = node_energy(m->p, g);
    m->nodes[g] = eps;
    double acc = 0.0;
    for (int c = 0; c < nc; ++c) {
      acc += rate_raw(m->ch[c], eps, p->relativistic);   // running sum in channel order (eq. frequency)
      m->C[static_cast<size_t>(c) * m->G + g] = acc;
    }
    if (!(acc > 0.0)) { delete m; return nullptr; }   // every electron must be able to collide
    numax = std::max(numax, acc);
  }
  // Constant trial frequency (the paper's LazyTrialFrequency: the table maximum) raised by
  // 2^-20 so that nu(eps) <= nu' holds after interpolation; a user value must not be below
  // the maximum (the paper's FixedTrialFrequency refuses such a value).
  if (p->user_majorant > 0.0) {
    if (p->user_majorant < numax) { delete m; return nullptr; }
    m->majorant = p->user_majorant;
  } else {
    m->majorant = (1.0 + 0x1.0p-20) * numax;
  }
  m->node_min = std::ldexp(1.0, p->grid_emin);
  m->node_max = std::ldexp(1.0, p->grid_emax);
  if (p->trial_strategy == 2) {
    // bins of the nodes, counted from the bin of node 0, and the nu' of every bin
    const int k0 = decade_bin(m->nodes[0], p->trial_bins);
    m->node_bin.resize(m->G);
    for (int g = 0; g < m->G; ++g) m->node_bin[g] = decade_bin(m->nodes[g], p->trial_bins) - k0;
    std::vector<double> top(m->node_bin[m->G - 1] + 1, 0.0);
    const double* F = &m->C[static_cast<size_t>(nc - 1) * m->G];
    for (int g = 0; g < m->G; ++g) {
      const double cell = g + 1 < m->G ? std::max(F[g], F[g + 1]) : F[g];
      top[m->node_bin[g]] = std::max(top[m->node_bin[g]], cell);
    }
    m->bin_nup.resize(top.size());
    for (size_t k = 0; k < top.size(); ++k) m->bin_nup[k] = std::min((1.0 + 0x1.0p-20) * top[k], m->majorant);
  }
  m->omega = kQe * p->B_T / kMe;
  m->a = {0.0, 0.0, -kQe * p->E_V_per_m / kMe};
  m->bhat = {std::sin(p->B_angle_rad), 0.0, std::cos(p->B_angle_rad)};
  if (p->B_T > 0.0) {
    const Vec3 Evec{0.0, 0.0, p->E_V_per_m};
    const Vec3 Bvec = scale(m->bhat, p->B_T);
    m->vD = scale(cross(Evec, Bvec), 1.0 / (p->B_T * p->B_T));
  } else {
    m->vD = {0.0, 0.0, 0.0};
  }
  *status = OR_OK;
  return m;
}

void or_destroy(void* h) { delete static_cast<Model*>(h); }

int32_t or_n_channels(void* h) { return static_cast<int32_t>(static_cast<Model*>(h)->ch.size()); }
int32_t or_grid_size(void* h) { return static_cast<Model*>(h)->G; }
double or_majorant(void* h) { return static_cast<Model*>(h)->majorant; }

// Binned strategy: the bin of every node (G entries) and the nu' of every bin; returns the
// number of bins (0 for the other strategies).  Either pointer may be NULL.
int32_t or_bins(void* h, int32_t* node_bin, double* bin_nup) {
  const Model& m = *static_cast<Model*>(h);
  if (node_bin) std::copy(m.node_bin.begin(), m.node_bin.end(), node_bin);
  if (bin_nup) std::copy(m.bin_nup.begin(), m.bin_nup.end(), bin_nup);
  return static_cast<int32_t>(m.bin_nup.size());
}

void or_tables(void* h, double* nodes, double* C) {
  const Model& m = *static_cast<Model*>(h);
  std::copy(m.nodes.begin(), m.nodes.end(), nodes);
  std::copy(m.C.begin(), m.C.end(), C);
}

double or_sigma_raw(void* h, int32_t c, double eps) { return sigma_raw(static_cast<Model*>(h)->ch[c], eps); }
double or_rate_raw_total(void* h, double eps) {
  const Model& m = *static_cast<Model*>(h);
  double acc = 0.0;
  for (const auto& ch : m.ch) acc += rate_raw(ch, eps, m.p.relativistic);
  return acc;
}
double or_nu_grid(void* h, double eps, int32_t* over) {
  bool ov = false;
  const double v = nu_total(*static_cast<Model*>(h), eps, &ov);
  if (over) *over = ov ? 1 : 0;
  return v;
}
double or_channel_cum(void* h, int32_t c, double eps) {
  const Model& m = *static_cast<Model*>(h);
  return interp(m, &m.C[static_cast<size_t>(c) * m.G], eps, nullptr);
}
// Real/null decision and channel for a given energy and x = R nu'; -1 means null.
int32_t or_select(void* h, double eps, double x) {
  const Model& m = *static_cast<Model*>(h);
  const int nc = static_cast<int>(m.ch.size());
  if (!(x < nu_total(m, eps))) return -1;
  int c = 0;
  while (c < nc - 1 && !(x < interp(m, &m.C[static_cast<size_t>(c) * m.G], eps, nullptr))) ++c;
  return c;
}

void or_move(void* h, const double* r0, const double* v0, double T, double* r, double* v) {
  const Model& m = *static_cast<Model*>(h);
  Vec3 rr, vv;
  advance(m, {r0[0], r0[1], r0[2]}, {v0[0], v0[1], v0[2]}, T, &rr, &vv);
  r[0] = rr.x; r[1] = rr.y; r[2] = rr.z;
  v[0] = vv.x; v[1] = vv.y; v[2] = vv.z;
}

// Kinetic energy (eV) of a held velocity, and speed / proper speed at an energy, for the
// model's mover.
double or_kinetic(void* h, const double* u) {
  return kinetic_eV({u[0], u[1], u[2]}, static_cast<Model*>(h)->p.relativistic);
}
double or_speed(void* h, double eps, int32_t proper) {
  const bool rel = static_cast<Model*>(h)->p.relativistic;
  return proper ? proper_speed(eps, rel) : speed_of(eps, rel);
}

double or_energy_after(int32_t kind, double eps, double eps_k, double cos_t, double mass_amu) {
  const double M = mass_amu * kAmu;
  if (kind == ELASTIC) return energy_after_elastic(eps, cos_t, M);
  if (kind == ATTACHMENT) return 0.0;
  return energy_after_inelastic(eps, eps_k, cos_t, M);
}

double or_xi_from_ratio(double r) { return xi_from_ratio(r); }

// Moving-target kinematics: the target velocity from four uniforms, and the electron's
// velocity after a collision with a target of mass_amu moving at V2 (direction u_hat in the
// centre-of-momentum frame, threshold eps_k_eV); returns 0 when the process cannot happen.
void or_target_velocity(double sigma, const double* u, double* out) {
  const Vec3 v = target_velocity(sigma, u[0], u[1], u[2], u[3]);
  out[0] = v.x; out[1] = v.y; out[2] = v.z;
}
int32_t or_moving_target(const double* V1, const double* V2, double mass_amu, double eps_k_eV,
                         const double* u_hat, double* V1p) {
  const double M = mass_amu * kAmu;
  const Vec3 a{V1[0], V1[1], V1[2]}, b{V2[0], V2[1], V2[2]}, uh{u_hat[0], u_hat[1], u_hat[2]};
  const Vec3 Vcm = centre_of_momentum(a, b, M);
  const double g2 = cm_speed2(a, Vcm, M, eps_k_eV * kQe);
  if (g2 < 0.0) return 0;
  const Vec3 r = add(Vcm, scale(uh, std::sqrt(g2)));
  V1p[0] = r.x; V1p[1] = r.y; V1p[2] = r.z;
  return 1;
}
double or_mt_over_el_of_xi(double xi) { return mt_over_el_of_xi(xi); }
double or_scatter_cos(int32_t scattering, double xi, double eps_eV, double u) {
  return scatter_cos(scattering, xi, eps_eV, u);
}
void or_rotate(const double* d, double cos_t, double phi, double* out) {
  const Vec3 n = rotate_direction({d[0], d[1], d[2]}, cos_t, phi);
  out[0] = n.x; out[1] = n.y; out[2] = n.z;
}

double or_const(int32_t which) {
  switch (which) {
    case 0: return kQe;
    case 1: return kMe;
    case 2: return kAmu;
    case 3: return kHartreeEV;
    case 4: return kKb;
    case 5: return kC;
    default: return 0.0;
  }
}

// Run n_electrons primaries (ids 0..n-1) for n_collisions real collisions each, on
// n_threads host threads.  Returns a result handle (records sorted by id).
void* or_run(void* h, int64_t n_electrons, int64_t n_collisions, uint64_t seed, int32_t n_threads,
             int64_t capacity, const uint64_t* trace_ids, int32_t n_trace, int32_t max_events,
             int64_t first_id) {
  const Model& m = *static_cast<Model*>(h);
  auto* res = new RunResult();
  res->status = OR_OK;
  if (n_electrons < 0 || n_collisions < 0 || n_collisions > 0xffffffffLL) {
    res->status = OR_INVALID;
    return res;
  }
  std::atomic<int64_t> created(n_electrons);
  std::atomic<int> cap_err(0);
  RunCtx cx;
  cx.m = &m;
  cx.seed = seed;
  cx.n_coll = static_cast<uint32_t>(n_collisions);
  if (trace_ids && n_trace > 0) cx.trace_ids.assign(trace_ids, trace_ids + n_trace);
  cx.max_events = max_events;
  cx.created = &created;
  cx.capacity = capacity > 0 ? capacity : (int64_t{1} << 62);
  cx.capacity_error = &cap_err;
  if (n_threads <= 0) n_threads = 1;
  std::atomic<int64_t> next(0);
  std::mutex mu;
  auto worker = [&]() {
    std::vector<Record> recs;
    std::vector<Event> evs;
    std::vector<Electron> stack;
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= n_electrons) break;
      stack.push_back(primary(m, seed, static_cast<uint64_t>(first_id + i)));
      while (!stack.empty()) {
        const Electron e = stack.back();
        stack.pop_back();
        recs.push_back(simulate(cx, e, stack, evs));
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    res->records.insert(res->records.end(), recs.begin(), recs.end());
    res->events.insert(res->events.end(), evs.begin(), evs.end());
  };
  std::vector<std::thread> th;
  for (int i = 0; i < n_threads; ++i) th.emplace_back(worker);
  for (auto& t : th) t.join();
  std::sort(res->records.begin(), res->records.end(),
            [](const Record& a, const Record& b) { return a.id < b.id; });
  std::stable_sort(res->events.begin(), res->events.end(), [](const Event& a, const Event& b) {
    if (a.id != b.id) return a.id < b.id;
    if (a.k != b.k) return a.k < b.k;
    return a.block < b.block;
  });
  if (cap_err.load()) res->status = OR_CAPACITY;
  return res;
}

int32_t or_run_status(void* r) { return static_cast<RunResult*>(r)->status; }
int64_t or_run_count(void* r) { return static_cast<int64_t>(static_cast<RunResult*>(r)->records.size()); }
int64_t or_run_event_count(void* r) { return static_cast<int64_t>(static_cast<RunResult*>(r)->events.size()); }
int32_t or_record_size() { return static_cast<int32_t>(sizeof(Record)); }
int32_t or_event_size() { return static_cast<int32_t>(sizeof(Event)); }
void or_run_copy(void* r, void* out) {
  const auto& v = static_cast<RunResult*>(r)->records;
  if (!v.empty()) std::memcpy(out, v.data(), v.size() * sizeof(Record));
}
void or_run_copy_events(void* r, void* out) {
  const auto& v = static_cast<RunResult*>(r)->events;
  if (!v.empty()) std::memcpy(out, v.data(), v.size() * sizeof(Event));
}
void or_run_free(void* r) { delete static_cast<RunResult*>(r); }

}  // extern "C"
