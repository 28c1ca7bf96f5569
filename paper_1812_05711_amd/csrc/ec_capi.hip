// Host side of the library: parameter mapping, reference rows, transform
// plans, workspace layout, the time loop and the C ABI of include/lbm_ec.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm_ec.h"
#include "ec_internal.hpp"

// Scratch of lbm_ec_poisson_static (see there): one copy per GPU.
constexpr size_t kStaticScratchBytes = (size_t)LBM_EC_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define EC_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(LBM_EC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

constexpr double kCs2 = 1.0 / 3.0;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Widest grid: a row pair's x transform is held in LDS (at most 160 KiB per
// workgroup); collide tiles are at most ec::kTileW columns wide whatever nx.
constexpr int kMaxNx = 8192;

// v rounded to `bits` significant bits, ties to even.
double round_bits(double v, int bits) {
  if (v == 0.0 || !std::isfinite(v)) return v;
  int e;
  const double m = std::frexp(v, &e);
  return std::ldexp(std::nearbyint(std::ldexp(m, bits)), e - bits);
}

// Field at the injector of the closed-form hydrostatic state (Eq. 27-28):
// the root E0 of [(E0^2 + 2 C E0)^(3/2) - E0^3] / (3 C E0) = 1, by bisection.
double field_at_injector(double C) {
  if (C == 0.0) return 1.0;
  auto drop = [C](double e0) { return (std::pow(e0 * e0 + 2.0 * C * e0, 1.5) - std::pow(e0, 3.0)) / (3.0 * C * e0) - 1.0; };
  double lo = 0.0, hi = 1.0;
  for (;;) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (drop(mid) < 0.0)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

ec::FftPlan make_plan(int n) {
  ec::FftPlan p{};
  p.n = n;
  p.nr = 0;
  int m = n;
  const int pref[5] = {8, 4, 2, 3, 5};
  for (int r : pref)
    while (m % r == 0 && p.nr < ec::kMaxRadices) {
      p.r[p.nr++] = r;
      m /= r;
    }
  for (int q = 7; m > 1 && p.nr < ec::kMaxRadices; q += 2)
    while (m % q == 0) {
      p.r[p.nr++] = q;
      m /= q;
    }
  return p;
}

// Launch shapes of a new instance: whole rows of collide threads (up to
// 1024) and about eight transform elements per thread (64 .. 512).
ec::Tuning default_tuning(int nx) {
  ec::Tuning tu;
  const int r64 = (nx + 63) / 64 * 64;
  tu.cbx = std::min(1024, std::max(64, r64));
  tu.cby = 1;
  const int f = ((nx + 7) / 8 + 63) / 64 * 64;
  tu.fft_threads = f <= 64 ? 64 : (f <= 128 ? 128 : (f <= 256 ? 256 : 512));
  return tu;
}

struct Layout {
  int P, M, MP, NC, KP;
  size_t tsize;
  size_t off_f[2], off_g[2], off_phi, off_rq, off_eu, off_ed, off_spec, off_tt, off_ends, off_gh, off_rf, off_iface,
      off_tw, off_twy, off_rows,
      off_rowsd, off_dmean, off_mom, off_stats, off_spart, total;
};

// poisson_only: the buffers of the Poisson chain alone (no populations, no
// charge sums of the collide tiles), for lbm_ec_poisson_static.
Layout make_layout(const lbm_ec_params& p, bool poisson_only = false) {
  Layout L{};
  L.tsize = p.precision == LBM_EC_FP64 ? 8 : 4;
  const int elems = (int)(256 / L.tsize);  // pitch multiple of 256 bytes
  L.P = (p.nx + elems - 1) / elems * elems;
  // a row pitch that is a multiple of 4 KiB is padded by 256 bytes, so that
  // the rows and the population planes a block streams from together do not
  // sit at power-of-two distances (which map them onto the same channels)
  if ((L.P * L.tsize) % 4096 == 0) L.P += elems;
  L.M = p.nx / 2 + 1;
  L.MP = (L.M + elems - 1) / elems * elems;
  L.NC = (p.ny + ec::kChunk - 1) / ec::kChunk;
  L.KP = L.NC >= 2 ? (L.NC - 1 + 7) / 8 * 8 : 0;
  const size_t ny = (size_t)p.ny, nx = (size_t)p.nx, nc = (size_t)L.NC;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t pop = poisson_only ? 0 : 9 * ny * L.P * L.tsize;
  L.off_f[0] = take(pop);
  L.off_f[1] = take(pop);
  L.off_g[0] = take(pop);
  L.off_g[1] = take(pop);
  L.off_phi = take(ny * L.P * L.tsize);
  const size_t tiles = poisson_only ? 0 : (ny + ec::tile_rows(p.ny) - 1) / ec::tile_rows(p.ny);
  L.off_rq = take(poisson_only ? 0 : ny * L.P * L.tsize);
  L.off_eu = take(tiles * L.P * L.tsize);
  L.off_ed = take(tiles * L.P * L.tsize);
  L.off_spec = take(ny * L.MP * 2 * L.tsize);
  L.off_tt = take(4 * 3 * (size_t)ec::kChunk * L.MP * L.tsize);
  L.off_ends = take(nc * 2 * L.MP * 2 * L.tsize);
  L.off_gh = take(nc * 6 * L.MP * L.tsize);
  L.off_rf = take((size_t)L.MP * ec::RF_COUNT * L.KP * L.tsize);
  L.off_iface = take(nc * 2 * L.MP * 2 * L.tsize);
  L.off_tw = take(nx * 4 * L.tsize);
  L.off_twy = take(ny * 8 * L.tsize);
  L.off_rows = take(ec::ROW_COUNT * ny * L.tsize);
  L.off_rowsd = take(ec::ROWD_COUNT * ny * 8);
  L.off_dmean = take((ny + 1) * 8);
  L.off_mom = take(4 * ny * nx * 8);
  L.off_stats = take(16 * 8);
  L.off_spart = take((size_t)ec::kStatsBands * 8 * 8);
  L.total = o;
  return L;
}

// LDS of one x-transform block of `threads` threads for rows of nx.
size_t transform_lds(int nx, int precision, int threads) {
  const ec::FftPlan pl = make_plan(nx);
  return precision == LBM_EC_FP64 ? ec::fft_lds_bytes<double>(pl, threads) : ec::fft_lds_bytes<float>(pl, threads);
}

int validate(const lbm_ec_params* p) {
  if (!p) return fail(LBM_EC_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 3) return fail(LBM_EC_EINVAL, "grid must have nx >= 1 and ny >= 3");
  if (p->precision != LBM_EC_FP64 && p->precision != LBM_EC_FP32_DEV && p->precision != LBM_EC_FP32_DEV_F64MATH)
    return fail(LBM_EC_EINVAL, "unknown precision");
  if (p->nx > kMaxNx) return fail(LBM_EC_EINVAL, "nx exceeds " + std::to_string(kMaxNx));
  if (transform_lds(p->nx, p->precision, 512) > ec::kMaxLds)
    return fail(LBM_EC_EINVAL, "the x transform of this nx does not fit LDS in this precision");
  if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return fail(LBM_EC_EINVAL, "grid too large");
  if (!(p->tau_plus > 0.5) || !std::isfinite(p->tau_plus)) return fail(LBM_EC_EINVAL, "tau_plus must exceed 1/2");
  if (!(p->Lambda > 0) || !(p->Lambda_g > 0) || !std::isfinite(p->Lambda) || !std::isfinite(p->Lambda_g))
    return fail(LBM_EC_EINVAL, "Lambda and Lambda_g must be positive and finite");
  if (!(p->T > 0) || !(p->M > 0) || !(p->Fe > 0) || !(p->C >= 0) || !std::isfinite(p->T) ||
      !std::isfinite(p->C) || !std::isfinite(p->M) || !std::isfinite(p->Fe))
    return fail(LBM_EC_EINVAL, "T, M, Fe must be positive and finite, C non-negative");
  if (p->init_mode < 0 || p->init_mode > 2) return fail(LBM_EC_EINVAL, "unknown init_mode");
  if (p->charge_rates != LBM_EC_RATES_ANTISYMMETRIC && p->charge_rates != LBM_EC_RATES_SYMMETRIC)
    return fail(LBM_EC_EINVAL, "unknown charge_rates");
  if (!std::isfinite(p->noise_amp) || !std::isfinite(p->body_force_x))
    return fail(LBM_EC_EINVAL, "noise_amp and body_force_x must be finite");
  // the lattice constants of Eq. 16 and 26 (as setup forms them) must be
  // finite and positive: extreme T, M or C overflow eps = (M K)^2 or rho0
  const double nu = kCs2 * (p->tau_plus - 0.5);
  const double K = nu * p->T / (p->M * p->M);
  const double eps = (p->M * K) * (p->M * K);
  const double rho0 = p->C * eps / ((double)p->ny * (double)p->ny);
  const double Dc = K / p->Fe;
  if (!(K > 0) || !(eps > 0) || !(Dc > 0) || !std::isfinite(K) || !std::isfinite(eps) || !std::isfinite(rho0) ||
      !std::isfinite(Dc) || !std::isfinite(0.5 + Dc / kCs2))
    return fail(LBM_EC_EINVAL, "the lattice constants (K, eps, rho0, D_c) of these parameters are not finite and positive");
  return LBM_EC_OK;
}

}  // namespace

// Kernel classes timed by the profiling hooks.
enum { KC_FORWARD = 0, KC_TRIDIAG, KC_INVERSE, KC_COLLIDE, KC_COUNT };

struct Profiler {
  bool on = false;
  uint32_t mask = 0;           // kernel classes timed in the current window
  std::vector<hipEvent_t> ev;  // pool, reused across profiling windows
  std::vector<int> cls;        // class of each recorded pair
  size_t used = 0;             // events used in the current window
};

struct lbm_ec {
  lbm_ec_params p;
  ec::Tuning tu;
  Profiler prof;
  Layout L;
  ec::Consts c;
  ec::Bufs b;
  ec::FftPlan plan;
  ec::FftPlan plan_y;  // length 2 ny (spectral y solve)
  int ysolver;         // LBM_EC_Y_TRIDIAGONAL or LBM_EC_Y_SPECTRAL
  hipStream_t s;
  int cur;  // buffer holding the latest post-collision populations
  int64_t steps;
  bool fp32;
};

namespace {

// Reference rows: the closed-form hydrostatic charge profile r(j) and the
// linear density profile balancing its uniform force; rounded to `bits`
// significant bits so that w_i times them, and their differences between
// rows, are exact in the storage type.
struct RefRows {
  std::vector<double> rc_closed, q, rho_ref;  // q = r / 36
  double s_ref = 0.0, s_init = 0.0;
};

RefRows reference_rows(const lbm_ec_params& p, double eps, int bits) {
  const int ny = p.ny;
  const double H = (double)ny;
  RefRows R;
  R.rc_closed.assign(ny, 0.0);
  R.q.resize(ny);
  R.rho_ref.resize(ny);
  double s_ref = 0.0;
  if (p.init_mode != LBM_EC_INIT_REST) {
    const double e0 = field_at_injector(p.C);
    for (int j = 0; j < ny; ++j) {
      const double y = ((double)j + 0.5) / (double)ny;
      double rc_nd = 0.0;
      if (p.C != 0.0) {
        const double e2 = e0 * e0 + 2.0 * p.C * e0 * y;
        rc_nd = p.C * e0 / std::sqrt(e2);
      }
      R.rc_closed[j] = eps / (H * H) * rc_nd;
    }
    const double F0 = eps * p.C * e0 / std::pow(H, 3.0);
    s_ref = 3.0 * F0;
  }
  R.s_init = 36.0 * round_bits(s_ref / 36.0, 40);
  R.s_ref = 36.0 * round_bits(s_ref / 36.0, bits);
  for (int j = 0; j < ny; ++j) {
    R.q[j] = round_bits(R.rc_closed[j] / 36.0, bits);
    R.rho_ref[j] = 1.0 + R.s_ref * (((double)j + 0.5) - 0.5 * H);
  }
  return R;
}

double lattice_eps(const lbm_ec_params& p) {
  const double nu = kCs2 * (p.tau_plus - 0.5);
  const double K = nu * p.T / (p.M * p.M);
  return (p.M * K) * (p.M * K);
}

// Twiddles of a transform plan: [n] complex exp(-2 pi i k / n), then for
// each pass of a register radix (2, 3, 4, 5, 8) and each k < Ns its R - 1
// factors exp(-2 pi i r k / (Ns R)) side by side (at most n more).
template <typename T>
std::vector<T> twiddle_table(const ec::FftPlan& pl) {
  const int n = pl.n;
  std::vector<T> tw(4 * (size_t)n, T(0));
  const long double twopi = 2.0L * 3.14159265358979323846264338327950288L;
  for (int k = 0; k < n; ++k) {
    const long double a = twopi * (long double)k / (long double)n;
    tw[2 * k] = (T)cosl(a);
    tw[2 * k + 1] = (T)(-sinl(a));
  }
  size_t o = 2 * (size_t)n;
  long long Ns = 1;
  for (int p = 0; p < pl.nr; ++p) {
    const int R = pl.r[p];
    if (R == 2 || R == 3 || R == 4 || R == 5 || R == 8) {
      for (long long k = 0; k < Ns; ++k)
        for (int r = 1; r < R; ++r) {
          const long double a = twopi * (long double)(r * k) / (long double)(Ns * R);
          tw[o++] = (T)cosl(a);
          tw[o++] = (T)(-sinl(a));
        }
    }
    Ns *= R;
  }
  return tw;
}

// Lattice constants (Eq. 16-17, Eq. 26 with rho = 1, dphi0 = 1, H = ny) and
// all tables, written into host vectors then copied to the device.  fresh:
// a new instance (the potential, the spectrum and the moments are cleared);
// otherwise only what the parameters fix is rewritten, and the state, the
// potential and the rows each step writes are left as they are.
template <typename T>
int setup(lbm_ec* h, unsigned char* ws, bool fresh = true) {
  const lbm_ec_params& p = h->p;
  const Layout& L = h->L;
  const int nx = p.nx, ny = p.ny;
  const double H = (double)ny;
  const double nu = kCs2 * (p.tau_plus - 0.5);
  const double K = nu * p.T / (p.M * p.M);
  const double eps = (p.M * K) * (p.M * K);
  const double rho0 = p.C * eps / (H * H);
  const double Dc = K / p.Fe;
  const double tau_m = 0.5 + p.Lambda / (p.tau_plus - 0.5);
  const double tau_gd = 0.5 + Dc / kCs2;
  const double tau_go = 0.5 + p.Lambda_g / (tau_gd - 0.5);
  double tau_gp, tau_gm;
  if (p.charge_rates == LBM_EC_RATES_ANTISYMMETRIC) {
    tau_gp = tau_go;
    tau_gm = tau_gd;
  } else {
    tau_gp = tau_gd;
    tau_gm = tau_go;
  }
  ec::Consts& c = h->c;
  c.nx = nx;
  c.ny = ny;
  c.P = L.P;
  c.M = L.M;
  c.MP = L.MP;
  c.NC = L.NC;
  c.KP = L.KP;
  c.TH = ec::tile_rows(ny);
  c.TW = ec::tile_width(nx, h->tu.ctw, (int)sizeof(T));
  c.wp = 1.0 / p.tau_plus;
  c.wm = 1.0 / tau_m;
  c.wgp = 1.0 / tau_gp;
  c.wgm = 1.0 / tau_gm;
  c.K = K;
  c.eps = eps;
  c.bx = p.body_force_x;
  c.H = H;
  c.u0 = K / H;
  c.init_mode = p.init_mode;
  c.noise_amp = p.noise_amp;
  c.seed = p.seed + (uint64_t)(int64_t)p.instance_id;

  const RefRows ref = reference_rows(p, eps, sizeof(T) == 8 ? 40 : 18);
  const std::vector<double>& rc_closed = ref.rc_closed;
  const std::vector<double>& q = ref.q;
  const std::vector<double>& rho_ref = ref.rho_ref;
  const double s_ref = ref.s_ref;
  c.s_init = ref.s_init;
  const double wa = 1.0 / 9.0, wd = 1.0 / 36.0;
  c.s_ref = s_ref;
  // R_axis = 4 q, R_diag = q (36 w_i is exactly 4 and 1)
  c.g_abb_axis = 2.0 * (wa * rho0 - 4.0 * q[0]);
  c.g_abb_diag = 2.0 * (wd * rho0 - 1.0 * q[0]);

  std::vector<T> rows((size_t)ec::ROW_COUNT * ny, T(0));
  std::vector<double> rowsd((size_t)ec::ROWD_COUNT * ny, 0.0);
  for (int j = 0; j < ny; ++j) {
    rows[ec::ROW_RHO_REF * ny + j] = (T)rho_ref[j];
    rows[ec::ROW_R * ny + j] = (T)(36.0 * q[j]);
    if (j > 0) {
      rows[ec::ROW_DG_UP_AXIS * ny + j] = (T)(4.0 * q[j - 1] - 4.0 * q[j]);
      rows[ec::ROW_DG_UP_DIAG * ny + j] = (T)(q[j - 1] - q[j]);
    }
    if (j < ny - 1) {
      rows[ec::ROW_DG_DN_AXIS * ny + j] = (T)(4.0 * q[j + 1] - 4.0 * q[j]);
      rows[ec::ROW_DG_DN_DIAG * ny + j] = (T)(q[j + 1] - q[j]);
    }
    // the pull adds, to the charge populations of row j, ua + 2 ud from
    // below (or the injector constants) and da + 2 dd from above (none at
    // the collector)
    const double below = j > 0 ? 6.0 * (q[j - 1] - q[j]) : c.g_abb_axis + 2.0 * c.g_abb_diag;
    const double above = j < ny - 1 ? 6.0 * (q[j + 1] - q[j]) : 0.0;
    rows[ec::ROW_KQ * ny + j] = (T)(below + above);
    rowsd[ec::ROWD_RHO_REF * ny + j] = rho_ref[j];
    rowsd[ec::ROWD_R * ny + j] = 36.0 * q[j];
    rowsd[ec::ROWD_RC_CLOSED * ny + j] = rc_closed[j];
  }

  // chunk tables of the per-wavenumber y systems (m >= 1): for each chunk
  // type the elimination factors of its own system and its responses v, w
  // to unit values just below / just above it (FP64, then rounded to T)
  const int M = L.M, MP = L.MP, NC = L.NC;
  const int KC = ec::kChunk;
  std::vector<T> tt((size_t)4 * 3 * KC * MP, T(0));
  auto tidx = [&](int type, int q, int i, int m) { return ((size_t)(type * 3 + q) * KC + i) * MP + m; };
  // end entries of the responses that couple neighbouring chunks (FP64)
  std::vector<double> ve_in(M, 0.0), we_in(M, 0.0), vs_in(M, 0.0), ws_in(M, 0.0), we_first(M, 0.0),
      vs_last(M, 0.0);
  for (int type = 0; type < 4; ++type) {
    int len;
    if (type == ec::CH_SINGLE) {
      if (NC != 1) continue;
      len = ny;
    } else {
      if (NC == 1) continue;
      if (type == ec::CH_INTERIOR && NC < 3) continue;
      len = type == ec::CH_LAST ? ny - (NC - 1) * KC : KC;
    }
    const bool wall_lo = type == ec::CH_SINGLE || type == ec::CH_FIRST;
    const bool wall_hi = type == ec::CH_SINGLE || type == ec::CH_LAST;
    std::vector<double> cpv(len), rhs(len), dp(len), x(len);
    for (int m = 1; m < M; ++m) {
      const int mf = std::min(m, nx - m);
      const double kap = 2.0 * M_PI * (double)mf / (double)nx;
      const double b = -(2.0 + kap * kap);
      for (int i = 0; i < len; ++i) {
        const double diag = b - ((i == 0 && wall_lo) ? 1.0 : 0.0) - ((i == len - 1 && wall_hi) ? 1.0 : 0.0);
        cpv[i] = i == 0 ? 1.0 / diag : 1.0 / (diag - cpv[i - 1]);
        tt[tidx(type, 0, i, m)] = (T)cpv[i];
      }
      // responses: A v = -e_0 (value just below), A w = -e_{len-1} (just above)
      for (int q = 1; q <= 2; ++q) {
        if (q == 1 && wall_lo) continue;
        if (q == 2 && wall_hi) continue;
        for (int i = 0; i < len; ++i) rhs[i] = 0.0;
        rhs[q == 1 ? 0 : len - 1] = -1.0;
        for (int i = 0; i < len; ++i) dp[i] = (rhs[i] - (i ? dp[i - 1] : 0.0)) * cpv[i];
        x[len - 1] = dp[len - 1];
        for (int i = len - 2; i >= 0; --i) x[i] = dp[i] - cpv[i] * x[i + 1];
        for (int i = 0; i < len; ++i) tt[tidx(type, q, i, m)] = (T)x[i];
        if (type == ec::CH_INTERIOR) {
          (q == 1 ? ve_in : we_in)[m] = x[len - 1];
          (q == 1 ? vs_in : ws_in)[m] = x[0];
        }
        if (type == ec::CH_FIRST && q == 2) we_first[m] = x[len - 1];
        if (type == ec::CH_LAST && q == 1) vs_last[m] = x[0];
      }
    }
  }
  // factors of the interface system (its matrix is fixed): the block
  // elimination over interfaces k = 0 .. NC-2 with 2x2 pivots, in FP64, as
  // the per-(m, k) coefficients of the two recurrences the device runs
  std::vector<T> rf((size_t)MP * ec::RF_COUNT * L.KP, T(0));
  if (NC >= 2) {
    const int K = NC - 1, KP = L.KP;
    for (int m = 1; m < M; ++m) {
      double g01_prev = 0.0;
      T* f = rf.data() + (size_t)m * ec::RF_COUNT * KP;
      for (int k = 0; k < K; ++k) {
        const double ve = k == 0 ? 0.0 : ve_in[m];
        const double we = k == 0 ? we_first[m] : we_in[m];
        const double vs = k + 1 == K ? vs_last[m] : vs_in[m];
        const double wsk = k + 1 == K ? 0.0 : ws_in[m];
        const double beta = -we + ve * g01_prev;
        const double gamma = -vs;
        const double inv = 1.0 / (1.0 - beta * gamma);
        const double g01 = beta * wsk * inv;
        f[ec::RF_INV * KP + k] = (T)inv;
        f[ec::RF_IB * KP + k] = (T)(inv * beta);
        f[ec::RF_A * KP + k] = (T)(inv * ve);
        f[ec::RF_P * KP + k] = (T)(inv * vs);
        f[ec::RF_Q * KP + k] = (T)(inv * vs * ve);
        f[ec::RF_C * KP + k] = (T)(wsk * inv);
        f[ec::RF_G * KP + k] = (T)g01;
        g01_prev = g01;
      }
    }
  }
  // twiddles exp(-2 pi i k / nx), then the same factors pass-major: for each
  // pass of radix R in {2, 3, 4, 5, 8} (Ns the product of the earlier
  // radices) and each k < Ns the R - 1 factors exp(-2 pi i r k / (Ns R)),
  // r = 1 .. R-1, next to each other (a butterfly reads them contiguously)
  const std::vector<T> tw = twiddle_table<T>(h->plan);
  EC_HIP(hipMemcpyAsync(h->b.rows, rows.data(), rows.size() * sizeof(T), hipMemcpyHostToDevice, h->s));
  // rows 0 .. ROWD_RC_CLOSED are fixed by the parameters, the others are
  // written by the steps
  EC_HIP(hipMemcpyAsync(h->b.rowsd, rowsd.data(),
                        (fresh ? rowsd.size() : (size_t)(ec::ROWD_RC_CLOSED + 1) * ny) * sizeof(double),
                        hipMemcpyHostToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.tt, tt.data(), tt.size() * sizeof(T), hipMemcpyHostToDevice, h->s));
  if (!rf.empty())
    EC_HIP(hipMemcpyAsync(h->b.rf, rf.data(), rf.size() * sizeof(T), hipMemcpyHostToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.tw, tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice, h->s));
  if (fresh) {
    EC_HIP(hipMemsetAsync(h->b.iface, 0, (size_t)NC * 2 * MP * 2 * sizeof(T), h->s));
    EC_HIP(hipMemsetAsync(ws + L.off_spec, 0, (size_t)ny * MP * 2 * sizeof(T), h->s));
    EC_HIP(hipMemsetAsync(ws + L.off_phi, 0, (size_t)ny * L.P * sizeof(T), h->s));
    EC_HIP(hipMemsetAsync(ws + L.off_mom, 0, 4 * (size_t)ny * nx * 8, h->s));
  }
  EC_HIP(hipStreamSynchronize(h->s));  // the host vectors go out of scope
  return LBM_EC_OK;
}

// Records an event on the handle's stream when class `cls` is being timed
// (start of a pair when `end` is false, its end otherwise).
int prof_mark(lbm_ec* h, int cls, bool end) {
  Profiler& P = h->prof;
  if (!P.on || !(P.mask & (1u << cls))) return LBM_EC_OK;
  if (P.used == P.ev.size()) {
    // timing only: no system-scope fence (cache writeback and invalidation)
    // around the kernels being timed; profile_end waits for the stream
    // before it reads the times
    hipEvent_t e;
    EC_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    P.ev.push_back(e);
  }
  if (!end) P.cls.push_back(cls);
  EC_HIP(hipEventRecord(P.ev[P.used++], h->s));
  return LBM_EC_OK;
}

#define EC_TIMED(h, cls, launch)           \
  do {                                     \
    int rc_ = prof_mark((h), (cls), false); \
    if (rc_) return rc_;                   \
    EC_HIP(launch);                        \
    rc_ = prof_mark((h), (cls), true);     \
    if (rc_) return rc_;                   \
  } while (0)

template <typename T>
int poisson_chain(lbm_ec* h, int mode, int src) {
  EC_TIMED(h, KC_FORWARD, (ec::launch_forward<T>(h->c, h->b, h->plan, mode, src, h->tu, h->s)));
  if (h->ysolver == LBM_EC_Y_SPECTRAL)
    EC_TIMED(h, KC_TRIDIAG, (ec::launch_yspec<T>(h->c, h->b, h->plan_y, h->s)));
  else
    EC_TIMED(h, KC_TRIDIAG, (ec::launch_tridiag<T>(h->c, h->b, h->s)));
  EC_TIMED(h, KC_INVERSE, (ec::launch_inverse<T>(h->c, h->b, h->plan, h->tu, h->s)));
  return LBM_EC_OK;
}

template <typename T, typename C>
int init_state(lbm_ec* h) {
  int rc;
  // initial charge, its potential, the equilibria into buffer 1
  EC_HIP(ec::launch_init_charge<T>(h->c, h->b, h->s));
  if ((rc = poisson_chain<T>(h, 2, 0))) return rc;
  EC_HIP(ec::launch_init_populations<T>(h->c, h->b, 1, h->s));
  // step 0: charge of the initial populations, Poisson, first collision
  // (no streaming) into buffer 0, with the moments of state 0
  if ((rc = poisson_chain<T>(h, 1, 1))) return rc;
  EC_HIP((ec::launch_collide<T, C>(h->c, h->b, false, true, 1, 0, h->tu, h->s)));
  h->cur = 0;
  h->steps = 0;
  return LBM_EC_OK;
}

template <typename T, typename C>
int run_steps(lbm_ec* h, int64_t n) {
  int rc;
  for (int64_t k = 0; k < n; ++k) {
    const int src = h->cur, dst = 1 - h->cur;
    if ((rc = poisson_chain<T>(h, 0, src))) return rc;
    EC_TIMED(h, KC_COLLIDE, (ec::launch_collide<T, C>(h->c, h->b, true, k == n - 1, src, dst, h->tu, h->s)));
    h->cur = dst;
    h->steps += 1;
  }
  return LBM_EC_OK;
}

// Points the handle at the buffers of layout L inside the device region ws.
void bind_buffers(lbm_ec* h, const lbm_ec_params* p, const Layout& L, unsigned char* ws, hipStream_t s) {
  h->p = *p;
  h->L = L;
  h->s = s;
  h->fp32 = p->precision != LBM_EC_FP64;
  h->plan = make_plan(p->nx);
  h->plan_y = make_plan(2 * p->ny);
  h->ysolver = LBM_EC_Y_TRIDIAGONAL;
  h->tu = default_tuning(p->nx);
  h->b.f[0] = ws + L.off_f[0];
  h->b.f[1] = ws + L.off_f[1];
  h->b.g[0] = ws + L.off_g[0];
  h->b.g[1] = ws + L.off_g[1];
  h->b.phi = ws + L.off_phi;
  h->b.rq = ws + L.off_rq;
  h->b.eu = ws + L.off_eu;
  h->b.ed = ws + L.off_ed;
  h->b.spec = ws + L.off_spec;
  h->b.tt = ws + L.off_tt;
  h->b.ends = ws + L.off_ends;
  h->b.gh = ws + L.off_gh;
  h->b.rf = ws + L.off_rf;
  h->b.iface = ws + L.off_iface;
  h->b.tw = ws + L.off_tw;
  h->b.twy = ws + L.off_twy;
  h->b.rows = ws + L.off_rows;
  h->b.rowsd = (double*)(ws + L.off_rowsd);
  h->b.dmean = (double*)(ws + L.off_dmean);
  h->b.mom = (double*)(ws + L.off_mom);
  h->b.stats = (double*)(ws + L.off_stats);
  h->b.spart = (double*)(ws + L.off_spart);
}

// Builds an instance in the device region ws (L.total bytes) on stream s and
// enqueues its initial state; waits for the stream.
int build_instance(lbm_ec* h, const lbm_ec_params* p, unsigned char* ws, hipStream_t s) {
  bind_buffers(h, p, make_layout(*p), ws, s);
  int rc = h->fp32 ? setup<float>(h, ws) : setup<double>(h, ws);
  if (!rc) {
    if (p->precision == LBM_EC_FP64)
      rc = init_state<double, double>(h);
    else if (p->precision == LBM_EC_FP32_DEV)
      rc = init_state<float, float>(h);
    else
      rc = init_state<float, double>(h);
  }
  if (!rc) {
    hipError_t e = hipStreamSynchronize(h->s);
    if (e != hipSuccess) rc = fail(LBM_EC_EHIP, std::string("initial state: ") + hipGetErrorString(e));
  }
  return rc;
}

// Continuation at another electric Rayleigh number (the state is that of
// lbm_ec_set_T): the charge populations are rescaled and re-referenced, the
// constants and tables of the new T written, and the density rows of the
// next step formed from the rescaled populations.  Waits for the stream.
template <typename T>
int continue_at_T(lbm_ec* h, double T_new) {
  lbm_ec_params p = h->p;
  p.T = T_new;
  int rc = validate(&p);
  if (rc) return rc;
  unsigned char* ws = (unsigned char*)h->b.f[0] - h->L.off_f[0];
  const double eps_new = lattice_eps(p);
  const double scale = eps_new / h->c.eps;
  const RefRows ref = reference_rows(p, eps_new, sizeof(T) == 8 ? 40 : 18);
  std::vector<double> r_new(p.ny);
  for (int j = 0; j < p.ny; ++j) r_new[j] = 36.0 * ref.q[j];
  EC_HIP(hipMemcpyAsync(h->b.rowsd + (size_t)ec::ROWD_RNEXT * p.ny, r_new.data(), sizeof(double) * p.ny,
                        hipMemcpyHostToDevice, h->s));
  // the reference rows use the force slope rounded for the storage type;
  // the state is defined by the slope the FP64 rows use (s_init)
  const double ddelta = (ref.s_ref - ref.s_init) - (h->c.s_ref - h->c.s_init);
  EC_HIP(ec::launch_continue<T>(h->c, h->b, h->cur, scale, ddelta, h->s));
  EC_HIP(hipStreamSynchronize(h->s));  // r_new goes out of scope
  h->p = p;
  if ((rc = setup<T>(h, ws, false))) return rc;
  EC_HIP(ec::launch_density<T>(h->c, h->b, h->cur, h->tu, h->s));
  hipError_t e = hipStreamSynchronize(h->s);
  if (e != hipSuccess) return fail(LBM_EC_EHIP, std::string("continuation: ") + hipGetErrorString(e));
  return LBM_EC_OK;
}

int continue_at(lbm_ec* h, double T_new) {
  return h->fp32 ? continue_at_T<float>(h, T_new) : continue_at_T<double>(h, T_new);
}

}  // namespace

// ------------------------------------------------------------------ batches
namespace {

constexpr int kGraphSteps = 16;  // steps per captured graph

struct Slot {
  bool used = false;
  bool reported = false;
  lbm_ec inst;
  size_t off = 0, bytes = 0;  // region in the batch workspace
  int64_t target = 0;
  int hist_cap = 0;
  double* hist = nullptr;
};

struct Range {
  size_t off, bytes;
};

}  // namespace

struct lbm_ec_batch {
  int max_slots;
  int precision;
  int emit_every;
  unsigned char* ws;
  size_t ws_bytes;
  hipStream_t s;
  bool own_stream;
  std::vector<Slot> slots;
  std::vector<Range> free_list;  // sorted by offset
  // device tables at the start of the workspace
  ec::SlotDesc* d_desc;
  int* d_off;
  double* d_hist;
  int hist_rows;  // history rows per slot
  size_t heap_off;
  // current launch tables
  std::vector<int> order;  // slot index of each descriptor entry
  int totals[ec::BK_COUNT];
  size_t lds;
  size_t collide_lds;
  bool fft8;
  bool dirty;
  hipGraphExec_t g_many, g_one;
  bool have_graphs;
  ec::Tuning tu;
};

namespace {

size_t batch_header_bytes(int max_slots, int hist_rows) {
  size_t o = align_up(sizeof(ec::SlotDesc) * (size_t)max_slots);
  o += align_up(sizeof(int) * (size_t)ec::BK_COUNT * (max_slots + 1));
  o += align_up(sizeof(double) * ec::kHistCols * (size_t)hist_rows * max_slots);
  return o;
}

bool heap_alloc(lbm_ec_batch* B, size_t bytes, size_t* off) {
  bytes = align_up(bytes);
  for (size_t i = 0; i < B->free_list.size(); ++i) {
    Range& r = B->free_list[i];
    if (r.bytes >= bytes) {
      *off = r.off;
      r.off += bytes;
      r.bytes -= bytes;
      if (r.bytes == 0) B->free_list.erase(B->free_list.begin() + i);
      return true;
    }
  }
  return false;
}

void heap_free(lbm_ec_batch* B, size_t off, size_t bytes) {
  bytes = align_up(bytes);
  std::vector<Range>& F = B->free_list;
  size_t i = 0;
  while (i < F.size() && F[i].off < off) ++i;
  F.insert(F.begin() + i, Range{off, bytes});
  // coalesce with the neighbours
  if (i + 1 < F.size() && F[i].off + F[i].bytes == F[i + 1].off) {
    F[i].bytes += F[i + 1].bytes;
    F.erase(F.begin() + i + 1);
  }
  if (i > 0 && F[i - 1].off + F[i - 1].bytes == F[i].off) {
    F[i - 1].bytes += F[i].bytes;
    F.erase(F.begin() + i);
  }
}

void drop_graphs(lbm_ec_batch* B) {
  if (B->have_graphs) {
    (void)hipGraphExecDestroy(B->g_many);
    (void)hipGraphExecDestroy(B->g_one);
    B->have_graphs = false;
  }
}

template <typename T, typename C>
int capture(lbm_ec_batch* B, int steps, hipGraphExec_t* out) {
  hipGraph_t g;
  EC_HIP(hipStreamBeginCapture(B->s, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int k = 0; k < steps && le == hipSuccess; ++k)
    le = ec::launch_batch_step<T, C>(B->d_desc, B->d_off, B->totals, (int)B->order.size(), B->lds, B->collide_lds,
                                     B->fft8, B->tu, B->s);
  hipError_t ee = hipStreamEndCapture(B->s, &g);
  if (le != hipSuccess) return fail(LBM_EC_EHIP, std::string("batch capture launch: ") + hipGetErrorString(le));
  if (ee != hipSuccess) return fail(LBM_EC_EHIP, std::string("batch capture: ") + hipGetErrorString(ee));
  hipError_t ie = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return fail(LBM_EC_EHIP, std::string("batch graph: ") + hipGetErrorString(ie));
  return LBM_EC_OK;
}

// Reads the device step state back into the slots.
int pull_state(lbm_ec_batch* B) {
  const int ns = (int)B->order.size();
  if (ns == 0) return LBM_EC_OK;
  std::vector<ec::SlotDesc> D(ns);
  EC_HIP(hipMemcpyAsync(D.data(), B->d_desc, sizeof(ec::SlotDesc) * ns, hipMemcpyDeviceToHost, B->s));
  EC_HIP(hipStreamSynchronize(B->s));
  for (int q = 0; q < ns; ++q) {
    if (B->order[q] < 0) continue;  // released since the tables were built
    Slot& sl = B->slots[B->order[q]];
    sl.inst.cur = D[q].cur;
    sl.inst.steps = D[q].steps_done;
  }
  return LBM_EC_OK;
}

// New descriptor and offset tables for the slots with steps left, and their graphs.
int rebuild(lbm_ec_batch* B) {
  int rc = pull_state(B);
  if (rc) return rc;
  drop_graphs(B);
  B->order.clear();
  for (int i = 0; i < B->max_slots; ++i) {
    const Slot& sl = B->slots[i];
    if (sl.used && sl.inst.steps < sl.target) B->order.push_back(i);
  }
  const int ns = (int)B->order.size();
  std::vector<ec::SlotDesc> D(ns);
  std::vector<int> off((size_t)ec::BK_COUNT * (ns + 1), 0);
  B->lds = 0;
  B->collide_lds = 0;
  B->fft8 = true;
  for (int k = 0; k < ec::BK_COUNT; ++k) B->totals[k] = 0;
  for (int q = 0; q < ns; ++q) {
    Slot& sl = B->slots[B->order[q]];
    ec::SlotDesc& d = D[q];
    d.c = sl.inst.c;
    d.c.TW = ec::tile_width(d.c.nx, B->tu.ctw, sl.inst.fp32 ? 4 : 8);
    d.b = sl.inst.b;
    d.plan = sl.inst.plan;
    d.cur = sl.inst.cur;
    d.active = 1;
    d.emit_every = B->emit_every;
    d.hist_cap = sl.hist_cap;
    d.steps_done = sl.inst.steps;
    d.steps_target = sl.target;
    d.hist = sl.hist;
    const size_t lds = sl.inst.fp32 ? ec::fft_lds_bytes<float>(sl.inst.plan, B->tu.fft_threads)
                                    : ec::fft_lds_bytes<double>(sl.inst.plan, B->tu.fft_threads);
    B->lds = std::max(B->lds, lds);
    const size_t clds = sl.inst.fp32 ? ec::collide_lds_bytes<float>(d.c.TW, d.c.nx)
                                     : ec::collide_lds_bytes<double>(d.c.TW, d.c.nx);
    B->collide_lds = std::max(B->collide_lds, clds);
    B->fft8 = B->fft8 && ec::fft_in_place(sl.inst.plan, B->tu.fft_threads, 8);
    for (int k = 0; k < ec::BK_COUNT; ++k) {
      off[(size_t)k * (ns + 1) + q] = B->totals[k];
      B->totals[k] += ec::batch_blocks(d.c, k);
    }
  }
  for (int k = 0; k < ec::BK_COUNT; ++k) off[(size_t)k * (ns + 1) + ns] = B->totals[k];
  if (B->lds > ec::kMaxLds || B->collide_lds > ec::kMaxLds)
    return fail(LBM_EC_EINVAL, "launch shapes too small for the widest slot (LDS of a block beyond 160 KiB)");
  if (ns) {
    EC_HIP(hipMemcpyAsync(B->d_desc, D.data(), sizeof(ec::SlotDesc) * ns, hipMemcpyHostToDevice, B->s));
    EC_HIP(hipMemcpyAsync(B->d_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, B->s));
    EC_HIP(hipStreamSynchronize(B->s));
    if (B->precision == LBM_EC_FP64) {
      if ((rc = capture<double, double>(B, kGraphSteps, &B->g_many))) return rc;
      if ((rc = capture<double, double>(B, 1, &B->g_one))) return rc;
    } else if (B->precision == LBM_EC_FP32_DEV) {
      if ((rc = capture<float, float>(B, kGraphSteps, &B->g_many))) return rc;
      if ((rc = capture<float, float>(B, 1, &B->g_one))) return rc;
    } else {
      if ((rc = capture<float, double>(B, kGraphSteps, &B->g_many))) return rc;
      if ((rc = capture<float, double>(B, 1, &B->g_one))) return rc;
    }
    B->have_graphs = true;
  }
  B->dirty = false;
  return LBM_EC_OK;
}

}  // namespace

extern "C" {

size_t lbm_ec_batch_workspace_bytes(const lbm_ec_params* ps, int32_t n, int32_t max_slots, int32_t hist_rows) {
  if (max_slots < 1 || hist_rows < 1 || n < 0 || (n > 0 && !ps)) return 0;
  size_t total = batch_header_bytes(max_slots, hist_rows);
  for (int i = 0; i < n; ++i) {
    if (validate(&ps[i]) != LBM_EC_OK) return 0;
    total += align_up(make_layout(ps[i]).total);
  }
  return total;
}

int lbm_ec_batch_create(int32_t max_slots, int32_t precision, int32_t emit_every, int32_t hist_rows, void* d_ws,
                        size_t ws_bytes, void* hip_stream, lbm_ec_batch_t** out) {
  g_err.clear();
  if (!out) return fail(LBM_EC_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096) return fail(LBM_EC_EINVAL, "max_slots must be in 1..4096");
  if (precision != LBM_EC_FP64 && precision != LBM_EC_FP32_DEV && precision != LBM_EC_FP32_DEV_F64MATH)
    return fail(LBM_EC_EINVAL, "unknown precision");
  if (emit_every < 0 || hist_rows < 1) return fail(LBM_EC_EINVAL, "emit_every >= 0 and hist_rows >= 1 required");
  if (!d_ws) return fail(LBM_EC_EINVAL, "workspace is NULL");
  if (((uintptr_t)d_ws) % kAlign) return fail(LBM_EC_ENOMEM, "workspace must be 256-byte aligned");
  const size_t head = batch_header_bytes(max_slots, hist_rows);
  if (ws_bytes < head) return fail(LBM_EC_ENOMEM, "workspace smaller than the batch tables");
  lbm_ec_batch* B = new lbm_ec_batch();
  B->max_slots = max_slots;
  B->precision = precision;
  B->emit_every = emit_every;
  B->ws = (unsigned char*)d_ws;
  B->ws_bytes = ws_bytes;
  B->own_stream = hip_stream == nullptr;
  if (B->own_stream) {
    hipError_t e = hipStreamCreateWithFlags(&B->s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete B;
      return fail(LBM_EC_EHIP, std::string("stream: ") + hipGetErrorString(e));
    }
  } else {
    B->s = (hipStream_t)hip_stream;
  }
  B->slots.resize(max_slots);
  size_t o = 0;
  B->d_desc = (ec::SlotDesc*)(B->ws + o);
  o += align_up(sizeof(ec::SlotDesc) * (size_t)max_slots);
  B->d_off = (int*)(B->ws + o);
  o += align_up(sizeof(int) * (size_t)ec::BK_COUNT * (max_slots + 1));
  B->d_hist = (double*)(B->ws + o);
  B->hist_rows = hist_rows;
  o += align_up(sizeof(double) * ec::kHistCols * (size_t)hist_rows * max_slots);
  B->heap_off = o;
  B->free_list.push_back(Range{o, ws_bytes - o});
  B->dirty = true;
  B->have_graphs = false;
  *out = B;
  return LBM_EC_OK;
}

int lbm_ec_batch_admit(lbm_ec_batch_t* B, const lbm_ec_params* p, int64_t n_steps, int32_t* slot) {
  if (!B || !p || !slot) return fail(LBM_EC_EINVAL, "NULL argument");
  int rc = validate(p);
  if (rc) return rc;
  if (p->precision != B->precision) return fail(LBM_EC_EINVAL, "precision differs from the batch's");
  if (n_steps < 1) return fail(LBM_EC_EINVAL, "n_steps must be positive");
  int idx = -1;
  for (int i = 0; i < B->max_slots; ++i)
    if (!B->slots[i].used) {
      idx = i;
      break;
    }
  if (idx < 0) return fail(LBM_EC_EBUSY, "no free slot");
  const Layout L = make_layout(*p);
  size_t off;
  if (!heap_alloc(B, L.total, &off)) return fail(LBM_EC_EBUSY, "not enough free workspace for this instance");
  // the step state of the running slots is on the device: read it before the
  // slot set changes
  if ((rc = pull_state(B))) {
    heap_free(B, off, L.total);
    return rc;
  }
  Slot& sl = B->slots[idx];
  sl = Slot();
  if ((rc = build_instance(&sl.inst, p, B->ws + off, B->s))) {
    heap_free(B, off, L.total);
    return rc;
  }
  sl.used = true;
  sl.off = off;
  sl.bytes = L.total;
  sl.target = n_steps;
  sl.hist = B->d_hist + ec::kHistCols * (size_t)B->hist_rows * idx;
  sl.hist_cap = B->hist_rows;
  EC_HIP(hipMemsetAsync(sl.hist, 0, sizeof(double) * ec::kHistCols * B->hist_rows, B->s));
  B->dirty = true;
  *slot = idx;
  return LBM_EC_OK;
}

int lbm_ec_batch_step(lbm_ec_batch_t* B, int64_t n) {
  if (!B) return fail(LBM_EC_EINVAL, "NULL argument");
  if (n < 0) return fail(LBM_EC_EINVAL, "negative step count");
  int rc;
  if (B->dirty && (rc = rebuild(B))) return rc;
  if (B->order.empty()) return LBM_EC_OK;
  for (int64_t k = 0; k + kGraphSteps <= n; k += kGraphSteps) EC_HIP(hipGraphLaunch(B->g_many, B->s));
  for (int64_t k = 0; k < n % kGraphSteps; ++k) EC_HIP(hipGraphLaunch(B->g_one, B->s));
  return LBM_EC_OK;
}

int lbm_ec_batch_poll(lbm_ec_batch_t* B, int32_t* done_slots, int32_t cap, int32_t* n_done) {
  if (!B || !n_done || (cap > 0 && !done_slots)) return fail(LBM_EC_EINVAL, "NULL argument");
  int rc = pull_state(B);
  if (rc) return rc;
  int n = 0;
  for (int i = 0; i < B->max_slots; ++i) {
    Slot& sl = B->slots[i];
    if (sl.used && !sl.reported && sl.inst.steps >= sl.target && n < cap) {
      done_slots[n++] = i;
      sl.reported = true;
      B->dirty = true;  // drop the finished slot from the launch tables
    }
  }
  *n_done = n;
  return LBM_EC_OK;
}

int64_t lbm_ec_batch_steps_done(lbm_ec_batch_t* B, int32_t slot) {
  if (!B || slot < 0 || slot >= B->max_slots || !B->slots[slot].used) return -1;
  if (pull_state(B)) return -1;
  return B->slots[slot].inst.steps;
}

int lbm_ec_batch_fields(lbm_ec_batch_t* B, int32_t slot, double* rho, double* ux, double* uy, double* rho_c,
                        double* phi) {
  if (!B || slot < 0 || slot >= B->max_slots || !B->slots[slot].used) return fail(LBM_EC_EINVAL, "bad slot");
  lbm_ec* h = &B->slots[slot].inst;
  EC_HIP(h->fp32 ? ec::launch_fields<float>(h->c, h->b, rho, ux, uy, rho_c, phi, nullptr, B->s)
                 : ec::launch_fields<double>(h->c, h->b, rho, ux, uy, rho_c, phi, nullptr, B->s));
  return LBM_EC_OK;
}

int lbm_ec_batch_fields_rho_m1(lbm_ec_batch_t* B, int32_t slot, double* rho_m1) {
  if (!B || slot < 0 || slot >= B->max_slots || !B->slots[slot].used) return fail(LBM_EC_EINVAL, "bad slot");
  if (!rho_m1) return fail(LBM_EC_EINVAL, "NULL argument");
  lbm_ec* h = &B->slots[slot].inst;
  EC_HIP(h->fp32 ? ec::launch_fields<float>(h->c, h->b, nullptr, nullptr, nullptr, nullptr, nullptr, rho_m1, B->s)
                 : ec::launch_fields<double>(h->c, h->b, nullptr, nullptr, nullptr, nullptr, nullptr, rho_m1, B->s));
  return LBM_EC_OK;
}

int lbm_ec_batch_history(lbm_ec_batch_t* B, int32_t slot, double* out, int32_t rows) {
  if (!B || !out || slot < 0 || slot >= B->max_slots || !B->slots[slot].used) return fail(LBM_EC_EINVAL, "bad slot");
  if (rows < 0) return fail(LBM_EC_EINVAL, "rows must be non-negative");
  const int r = std::min(rows, B->hist_rows);
  EC_HIP(hipMemcpyAsync(out, B->slots[slot].hist, sizeof(double) * ec::kHistCols * r, hipMemcpyDeviceToHost, B->s));
  EC_HIP(hipStreamSynchronize(B->s));
  return LBM_EC_OK;
}

int lbm_ec_batch_set_T(lbm_ec_batch_t* B, int32_t slot, double T) {
  if (!B || slot < 0 || slot >= B->max_slots || !B->slots[slot].used) return fail(LBM_EC_EINVAL, "bad slot");
  int rc = pull_state(B);
  if (rc) return rc;
  if ((rc = continue_at(&B->slots[slot].inst, T))) return rc;
  B->dirty = true;  // the slot's constants changed
  return LBM_EC_OK;
}

int lbm_ec_batch_release(lbm_ec_batch_t* B, int32_t slot) {
  if (!B || slot < 0 || slot >= B->max_slots || !B->slots[slot].used) return fail(LBM_EC_EINVAL, "bad slot");
  int rc = pull_state(B);
  if (rc) return rc;
  EC_HIP(hipStreamSynchronize(B->s));
  Slot& sl = B->slots[slot];
  for (hipEvent_t e : sl.inst.prof.ev) (void)hipEventDestroy(e);
  heap_free(B, sl.off, sl.bytes);
  sl = Slot();
  // the device tables still list this slot until the next rebuild: make sure
  // its entry is never read back into a simulation admitted to the same slot
  for (int& q : B->order)
    if (q == slot) q = -1;
  B->dirty = true;
  return LBM_EC_OK;
}

size_t lbm_ec_batch_free_bytes(lbm_ec_batch_t* B) {
  if (!B) return 0;
  size_t best = 0;
  for (const Range& r : B->free_list) best = std::max(best, r.bytes);
  return best;
}

void lbm_ec_batch_destroy(lbm_ec_batch_t* B) {
  if (!B) return;
  (void)hipStreamSynchronize(B->s);
  drop_graphs(B);
  for (Slot& sl : B->slots)
    for (hipEvent_t e : sl.inst.prof.ev) (void)hipEventDestroy(e);
  if (B->own_stream) (void)hipStreamDestroy(B->s);
  delete B;
}

static int check_tuning(int32_t fft_threads, int32_t bx, int32_t by, int32_t tw) {
  if (fft_threads != 64 && fft_threads != 128 && fft_threads != 256 && fft_threads != 512)
    return fail(LBM_EC_EINVAL, "fft_threads must be 64, 128, 256 or 512");
  const int64_t t = (int64_t)bx * by;
  if (bx < 1 || by < 1 || t % 64 != 0 || t > 1024)
    return fail(LBM_EC_EINVAL, "collide block bx * by must be a multiple of 64 up to 1024");
  if (tw < 0 || tw > ec::kTileW) return fail(LBM_EC_EINVAL, "collide tile width must be 0 (default) .. 1024");
  return LBM_EC_OK;
}

int lbm_ec_set_tuning(lbm_ec_t* h, int32_t fft_threads, int32_t collide_bx, int32_t collide_by, int32_t collide_tw) {
  if (!h) return fail(LBM_EC_EINVAL, "handle is NULL");
  int rc = check_tuning(fft_threads, collide_bx, collide_by, collide_tw);
  if (rc) return rc;
  if (transform_lds(h->p.nx, h->p.precision, fft_threads) > ec::kMaxLds)
    return fail(LBM_EC_EINVAL, "too few transform threads for this nx (LDS of a block beyond 160 KiB)");
  h->tu.fft_threads = fft_threads;
  h->tu.cbx = collide_bx;
  h->tu.cby = collide_by;
  h->tu.ctw = collide_tw;
  h->c.TW = ec::tile_width(h->p.nx, collide_tw, h->fp32 ? 4 : 8);
  return LBM_EC_OK;
}

int lbm_ec_batch_set_tuning(lbm_ec_batch_t* B, int32_t fft_threads, int32_t collide_bx, int32_t collide_by,
                            int32_t collide_tw) {
  if (!B) return fail(LBM_EC_EINVAL, "NULL argument");
  int rc = check_tuning(fft_threads, collide_bx, collide_by, collide_tw);
  if (rc) return rc;
  B->tu.fft_threads = fft_threads;
  B->tu.cbx = collide_bx;
  B->tu.cby = collide_by;
  B->tu.ctw = collide_tw;
  B->dirty = true;
  return LBM_EC_OK;
}

int lbm_ec_params_default(lbm_ec_params* p) {
  if (!p) return fail(LBM_EC_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->nx = 122;
  p->ny = 100;
  p->T = 200.0;
  p->C = 10.0;
  p->M = 10.0;
  p->Fe = 4000.0;
  p->tau_plus = 0.8;
  p->Lambda = 0.25;
  p->Lambda_g = 1e-6;
  p->precision = LBM_EC_FP64;
  p->init_mode = LBM_EC_INIT_NOISE;
  p->noise_amp = 1e-3;
  p->seed = 181205711ull;
  p->instance_id = 0;
  p->charge_rates = LBM_EC_RATES_ANTISYMMETRIC;
  p->body_force_x = 0.0;
  return LBM_EC_OK;
}

int lbm_ec_validate(const lbm_ec_params* p) { return validate(p); }

size_t lbm_ec_workspace_bytes(const lbm_ec_params* p) {
  if (validate(p) != LBM_EC_OK) return 0;
  return make_layout(*p).total;
}

int lbm_ec_create(const lbm_ec_params* p, void* d_ws, size_t ws_bytes, void* hip_stream, lbm_ec_t** out) {
  g_err.clear();
  if (!out) return fail(LBM_EC_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (!d_ws) return fail(LBM_EC_EINVAL, "workspace is NULL");
  const Layout L = make_layout(*p);
  if (ws_bytes < L.total)
    return fail(LBM_EC_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  if (((uintptr_t)d_ws) % kAlign) return fail(LBM_EC_ENOMEM, "workspace must be 256-byte aligned");
  lbm_ec* h = new lbm_ec();
  rc = build_instance(h, p, (unsigned char*)d_ws, (hipStream_t)hip_stream);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return LBM_EC_OK;
}

int lbm_ec_step(lbm_ec_t* h, int64_t n) {
  if (!h) return fail(LBM_EC_EINVAL, "handle is NULL");
  if (n < 0) return fail(LBM_EC_EINVAL, "negative step count");
  if (h->p.precision == LBM_EC_FP64) return run_steps<double, double>(h, n);
  if (h->p.precision == LBM_EC_FP32_DEV) return run_steps<float, float>(h, n);
  return run_steps<float, double>(h, n);
}

int lbm_ec_set_y_solver(lbm_ec_t* h, int32_t solver) {
  if (!h) return fail(LBM_EC_EINVAL, "handle is NULL");
  if (solver != LBM_EC_Y_TRIDIAGONAL && solver != LBM_EC_Y_SPECTRAL) return fail(LBM_EC_EINVAL, "unknown y solver");
  if (solver == LBM_EC_Y_SPECTRAL) {
    const size_t lds = h->fp32 ? ec::yspec_lds_bytes<float>(h->p.ny) : ec::yspec_lds_bytes<double>(h->p.ny);
    if (lds > ec::kMaxLds)
      return fail(LBM_EC_EINVAL, "ny too large for the spectral y solve (two columns of 2 ny in LDS)");
    const size_t n = 4 * (size_t)h->plan_y.n;
    if (h->fp32) {
      const std::vector<float> tw = twiddle_table<float>(h->plan_y);
      EC_HIP(hipMemcpyAsync(h->b.twy, tw.data(), n * sizeof(float), hipMemcpyHostToDevice, h->s));
      EC_HIP(hipStreamSynchronize(h->s));
    } else {
      const std::vector<double> tw = twiddle_table<double>(h->plan_y);
      EC_HIP(hipMemcpyAsync(h->b.twy, tw.data(), n * sizeof(double), hipMemcpyHostToDevice, h->s));
      EC_HIP(hipStreamSynchronize(h->s));
    }
    // the chunk corrections that the inverse transform adds vanish with
    // zero interface values
    EC_HIP(hipMemsetAsync(h->b.iface, 0, (size_t)h->L.NC * 2 * h->L.MP * 2 * h->L.tsize, h->s));
    EC_HIP(hipStreamSynchronize(h->s));
  }
  h->ysolver = solver;
  return LBM_EC_OK;
}

int lbm_ec_set_T(lbm_ec_t* h, double T) {
  if (!h) return fail(LBM_EC_EINVAL, "handle is NULL");
  return continue_at(h, T);
}

int64_t lbm_ec_steps_done(const lbm_ec_t* h) { return h ? h->steps : -1; }

int lbm_ec_fields(lbm_ec_t* h, double* rho, double* ux, double* uy, double* rho_c, double* phi) {
  if (!h) return fail(LBM_EC_EINVAL, "handle is NULL");
  EC_HIP(h->fp32 ? ec::launch_fields<float>(h->c, h->b, rho, ux, uy, rho_c, phi, nullptr, h->s)
                 : ec::launch_fields<double>(h->c, h->b, rho, ux, uy, rho_c, phi, nullptr, h->s));
  return LBM_EC_OK;
}

int lbm_ec_fields_rho_m1(lbm_ec_t* h, double* rho_m1) {
  if (!h || !rho_m1) return fail(LBM_EC_EINVAL, "NULL argument");
  EC_HIP(h->fp32 ? ec::launch_fields<float>(h->c, h->b, nullptr, nullptr, nullptr, nullptr, nullptr, rho_m1, h->s)
                 : ec::launch_fields<double>(h->c, h->b, nullptr, nullptr, nullptr, nullptr, nullptr, rho_m1, h->s));
  return LBM_EC_OK;
}

int lbm_ec_poisson(lbm_ec_t* h, const double* d_rho_c, double* d_phi) {
  if (!h || !d_rho_c || !d_phi) return fail(LBM_EC_EINVAL, "NULL argument");
  int rc;
  if (h->fp32) {
    EC_HIP(ec::launch_charge_in<float>(h->c, h->b, d_rho_c, h->s));
    if ((rc = poisson_chain<float>(h, 2, 0))) return rc;
    EC_HIP(ec::launch_fields<float>(h->c, h->b, nullptr, nullptr, nullptr, nullptr, d_phi, nullptr, h->s));
  } else {
    EC_HIP(ec::launch_charge_in<double>(h->c, h->b, d_rho_c, h->s));
    if ((rc = poisson_chain<double>(h, 2, 0))) return rc;
    EC_HIP(ec::launch_fields<double>(h->c, h->b, nullptr, nullptr, nullptr, nullptr, d_phi, nullptr, h->s));
  }
  return LBM_EC_OK;
}

int lbm_ec_stats(lbm_ec_t* h, double* out) {
  if (!h || !out) return fail(LBM_EC_EINVAL, "NULL argument");
  EC_HIP(h->fp32 ? ec::launch_stats<float>(h->c, h->b, h->cur, h->s)
                 : ec::launch_stats<double>(h->c, h->b, h->cur, h->s));
  double tmp[16];
  EC_HIP(hipMemcpyAsync(tmp, h->b.stats, sizeof(tmp), hipMemcpyDeviceToHost, h->s));
  EC_HIP(hipStreamSynchronize(h->s));
  tmp[0] = (double)h->steps;
  for (int i = 0; i < 10; ++i) out[i] = tmp[i];
  if (tmp[6] > 0) return fail(LBM_EC_EUNSTABLE, "non-finite values or non-positive density in the state");
  return LBM_EC_OK;
}

int lbm_ec_profile_begin(lbm_ec_t* h, uint32_t class_mask) {
  if (!h) return fail(LBM_EC_EINVAL, "handle is NULL");
  h->prof.on = true;
  h->prof.mask = class_mask;
  h->prof.used = 0;
  h->prof.cls.clear();
  return LBM_EC_OK;
}

int lbm_ec_profile_end(lbm_ec_t* h, double* ms, int64_t* launches, int32_t n) {
  if (!h || !ms || !launches) return fail(LBM_EC_EINVAL, "NULL argument");
  Profiler& P = h->prof;
  P.on = false;
  for (int k = 0; k < n; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  EC_HIP(hipStreamSynchronize(h->s));
  for (size_t q = 0; q < P.cls.size(); ++q) {
    float t = 0.f;
    EC_HIP(hipEventElapsedTime(&t, P.ev[2 * q], P.ev[2 * q + 1]));
    const int c = P.cls[q];
    if (c < n) {
      ms[c] += (double)t;
      launches[c] += 1;
    }
  }
  P.used = 0;
  P.cls.clear();
  return LBM_EC_OK;
}

// ------------------------------------------------------------- checkpoints
// A checkpoint is [header, padded to 256 B][f][g][charge sums][tile edges]
// [phi][rows FP64][D][moments], each region 256-byte aligned: the
// post-collision populations with the charge density the collide tiles
// summed from them, and everything lbm_ec_fields reads, so a loaded
// instance continues bit for bit.  Version 4: the charge populations' x
// movers are stored shifted by their c_ix (version 3 stored them at their
// node), so older checkpoints are refused.
namespace {
constexpr char kCkptMagic[8] = {'L', 'B', 'M', 'E', 'C', 'C', 'K', '1'};
struct CkptHeader {
  char magic[8];
  uint32_t version, header_bytes;
  int32_t nx, ny, precision, charge_rates;
  // the reference rows of the stored deviations: zero for a rest start,
  // the closed-form hydrostatic rows otherwise
  int32_t rest_rows, pad;
  double T, C, M, Fe, tau_plus, Lambda, Lambda_g, body_force_x;
  int64_t steps;
  uint64_t total;
};
struct CkptLayout {
  size_t pop, phi, edges, rowsd, dmean, mom;  // region sizes
  size_t off_f, off_g, off_rq, off_eu, off_ed, off_phi, off_rowsd, off_dmean, off_mom, total;
};
CkptLayout ckpt_layout(const lbm_ec* h) {
  CkptLayout K{};
  const size_t ny = (size_t)h->p.ny, nx = (size_t)h->p.nx;
  K.pop = 9 * ny * h->L.P * h->L.tsize;
  K.phi = ny * h->L.P * h->L.tsize;
  K.edges = (size_t)ec::collide_tiles(h->c) * h->L.P * h->L.tsize;
  K.rowsd = (size_t)ec::ROWD_COUNT * ny * 8;
  K.dmean = (ny + 1) * 8;
  K.mom = 4 * ny * nx * 8;
  size_t o = align_up(sizeof(CkptHeader));
  K.off_f = o;
  o = align_up(o + K.pop);
  K.off_g = o;
  o = align_up(o + K.pop);
  K.off_rq = o;
  o = align_up(o + K.phi);
  K.off_eu = o;
  o = align_up(o + K.edges);
  K.off_ed = o;
  o = align_up(o + K.edges);
  K.off_phi = o;
  o = align_up(o + K.phi);
  K.off_rowsd = o;
  o = align_up(o + K.rowsd);
  K.off_dmean = o;
  o = align_up(o + K.dmean);
  K.off_mom = o;
  K.total = align_up(o + K.mom);
  return K;
}
void ckpt_fill(const lbm_ec* h, CkptHeader* H, uint64_t total) {
  std::memset(H, 0, sizeof(*H));
  std::memcpy(H->magic, kCkptMagic, 8);
  H->version = 4;
  H->header_bytes = (uint32_t)sizeof(CkptHeader);
  const lbm_ec_params& p = h->p;
  H->nx = p.nx;
  H->ny = p.ny;
  H->precision = p.precision;
  H->charge_rates = p.charge_rates;
  H->rest_rows = p.init_mode == LBM_EC_INIT_REST ? 1 : 0;
  H->T = p.T;
  H->C = p.C;
  H->M = p.M;
  H->Fe = p.Fe;
  H->tau_plus = p.tau_plus;
  H->Lambda = p.Lambda;
  H->Lambda_g = p.Lambda_g;
  H->body_force_x = p.body_force_x;
  H->steps = h->steps;
  H->total = total;
}
}  // namespace

size_t lbm_ec_checkpoint_bytes(const lbm_ec_t* h) { return h ? ckpt_layout(h).total : 0; }

int lbm_ec_save(lbm_ec_t* h, void* d_dst, size_t bytes) {
  if (!h || !d_dst) return fail(LBM_EC_EINVAL, "NULL argument");
  const CkptLayout K = ckpt_layout(h);
  if (bytes < K.total) return fail(LBM_EC_ENOMEM, "checkpoint buffer too small: need " + std::to_string(K.total));
  CkptHeader H;
  ckpt_fill(h, &H, K.total);
  unsigned char* d = (unsigned char*)d_dst;
  EC_HIP(hipMemcpyAsync(d, &H, sizeof(H), hipMemcpyHostToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_f, h->b.f[h->cur], K.pop, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_g, h->b.g[h->cur], K.pop, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_rq, h->b.rq, K.phi, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_eu, h->b.eu, K.edges, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_ed, h->b.ed, K.edges, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_phi, h->b.phi, K.phi, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_rowsd, h->b.rowsd, K.rowsd, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_dmean, h->b.dmean, K.dmean, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(d + K.off_mom, h->b.mom, K.mom, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipStreamSynchronize(h->s));  // the header is read from host memory
  return LBM_EC_OK;
}

int lbm_ec_load(lbm_ec_t* h, const void* d_src, size_t bytes) {
  if (!h || !d_src) return fail(LBM_EC_EINVAL, "NULL argument");
  const CkptLayout K = ckpt_layout(h);
  if (bytes < K.total) return fail(LBM_EC_EINVAL, "checkpoint buffer smaller than this instance's checkpoint");
  CkptHeader H, mine;
  const unsigned char* d = (const unsigned char*)d_src;
  EC_HIP(hipMemcpyAsync(&H, d, sizeof(H), hipMemcpyDeviceToHost, h->s));
  EC_HIP(hipStreamSynchronize(h->s));
  ckpt_fill(h, &mine, K.total);
  if (std::memcmp(H.magic, kCkptMagic, 8) != 0 || H.version != 4 || H.header_bytes != sizeof(CkptHeader))
    return fail(LBM_EC_EINVAL, "not a checkpoint of this library version");
  mine.steps = H.steps;
  if (std::memcmp(&H, &mine, sizeof(H)) != 0)
    return fail(LBM_EC_EINVAL,
                "checkpoint taken with other grid, precision, physical parameters or reference rows (rest start)");
  h->cur = 0;
  EC_HIP(hipMemcpyAsync(h->b.f[0], d + K.off_f, K.pop, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.g[0], d + K.off_g, K.pop, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.rq, d + K.off_rq, K.phi, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.eu, d + K.off_eu, K.edges, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.ed, d + K.off_ed, K.edges, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.phi, d + K.off_phi, K.phi, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.rowsd, d + K.off_rowsd, K.rowsd, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.dmean, d + K.off_dmean, K.dmean, hipMemcpyDeviceToDevice, h->s));
  EC_HIP(hipMemcpyAsync(h->b.mom, d + K.off_mom, K.mom, hipMemcpyDeviceToDevice, h->s));
  h->steps = H.steps;
  return LBM_EC_OK;
}

// ------------------------------------------- Poisson solve without allocation
// The scratch of lbm_ec_poisson_static: the Poisson-only layout of one grid
// (spectrum, potential, chunk and interface tables, twiddles, row tables, the
// charge field).  A file-scope device array, one copy per GPU, held until the
// process ends.  Host code never passes its name to a kernel or a copy: the
// name is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device.
}  // extern "C"

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up on first use).
int static_scratch(void** out) {
  int dev = -1;
  EC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EC_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LBM_EC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_EC_OK;
}

// The Poisson chain of lbm_ec_poisson on a handle whose buffers live in the
// scratch: same plan, tables, launch shapes and kernels, so the same result.
template <typename T>
int poisson_in_scratch(lbm_ec* h, unsigned char* ws, const double* d_rho_c, double* d_phi) {
  int rc = setup<T>(h, ws, false);  // tables only: nothing of the chain must start at zero
  if (rc) return rc;
  EC_HIP(ec::launch_charge_in<T>(h->c, h->b, d_rho_c, h->s));
  if ((rc = poisson_chain<T>(h, 2, 0))) return rc;
  EC_HIP(ec::launch_fields<T>(h->c, h->b, nullptr, nullptr, nullptr, nullptr, d_phi, nullptr, h->s));
  return LBM_EC_OK;
}
}  // namespace

extern "C" {

size_t lbm_ec_poisson_static_bytes(const lbm_ec_params* p) {
  if (validate(p) != LBM_EC_OK) return 0;
  return make_layout(*p, true).total;
}

int lbm_ec_poisson_static(const lbm_ec_params* p, const double* d_rho_c, double* d_phi, void* hip_stream) {
  g_err.clear();
  if (!p || !d_rho_c || !d_phi) return fail(LBM_EC_EINVAL, "NULL argument");
  int rc = validate(p);
  if (rc) return rc;
  const Layout L = make_layout(*p, true);
  if (L.total > kStaticScratchBytes)
    return fail(LBM_EC_EINVAL, "grid needs " + std::to_string(L.total) + " bytes of Poisson scratch; the static scratch holds " +
                                   std::to_string(kStaticScratchBytes));
  void* ptr = nullptr;
  if ((rc = static_scratch(&ptr))) return rc;
  lbm_ec h{};
  unsigned char* ws = (unsigned char*)ptr;
  bind_buffers(&h, p, L, ws, (hipStream_t)hip_stream);
  return h.fp32 ? poisson_in_scratch<float>(&h, ws, d_rho_c, d_phi)
                : poisson_in_scratch<double>(&h, ws, d_rho_c, d_phi);
}

// Test hook of the failure detection: a NaN in one population of the current
// state (population 0 of node (0, 0)).  Waits for the stream.
namespace {
int poison_instance(lbm_ec* h) {
  static const float kNanF = std::numeric_limits<float>::quiet_NaN();
  static const double kNanD = std::numeric_limits<double>::quiet_NaN();
  const void* src = h->fp32 ? (const void*)&kNanF : (const void*)&kNanD;
  EC_HIP(hipMemcpyAsync(h->b.f[h->cur], src, h->L.tsize, hipMemcpyHostToDevice, h->s));
  EC_HIP(hipStreamSynchronize(h->s));
  return LBM_EC_OK;
}
}  // namespace

int lbm_ec_debug_poison(lbm_ec_t* h) {
  if (!h) return fail(LBM_EC_EINVAL, "handle is NULL");
  return poison_instance(h);
}

int lbm_ec_batch_debug_poison(lbm_ec_batch_t* B, int32_t slot) {
  if (!B || slot < 0 || slot >= B->max_slots || !B->slots[slot].used) return fail(LBM_EC_EINVAL, "bad slot");
  int rc = pull_state(B);  // the slot's current buffer is kept on the device
  if (rc) return rc;
  return poison_instance(&B->slots[slot].inst);
}

void lbm_ec_destroy(lbm_ec_t* h) {
  if (!h) return;
  for (hipEvent_t e : h->prof.ev) (void)hipEventDestroy(e);
  delete h;
}

const char* lbm_ec_last_error(void) { return g_err.c_str(); }

}  // extern "C"
