// Host float64 plan: rescaling (eq. hypnorm), sector and square placement
// (Section 2.1), the coordinate maps T and P1 (eqs. transformT, transformP),
// lattice spacing (eq. lpsamples) and extent, row bands and per-slowness
// tables.  Compiled with -ffp-contract=off: the trapezoid cut is an integer
// decision that must come out exactly as the definition j*dt >= q0*x_k
// evaluated in float64.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

namespace hrt {

namespace {

constexpr double kPi = 3.14159265358979323846;

bool is_even_5smooth(int64_t m) {
  if (m < 2 || (m & 1)) return false;
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  return m == 1;
}

int64_t next_even_5smooth(int64_t n) {
  int64_t m = std::max<int64_t>(n, 2);
  while (!is_even_5smooth(m)) ++m;
  return m;
}

// Number of integers k >= 0 with 2 sigma k < M: the non-negative half of the
// band-limit rectangle L along one axis.
int kept_nonneg(int M, double sigma) {
  int k = 0;
  while (2.0 * sigma * static_cast<double>(k) < static_cast<double>(M)) ++k;
  return k;
}

struct TraceScan {
  double dphi = 0, deta = 0, eta_min = 1e300, eta_max = -1e300;
  int64_t kept = 0;
};

}  // namespace

bool fft_fits_inplace(const FftFactors& f, int batch, int threads, int values) {
  if (f.npass < 1) return false;
  for (int p = 0; p < f.npass; ++p) {
    const int64_t r = f.radix[p];
    const int64_t bfly = static_cast<int64_t>(batch) * f.n / r;
    if ((bfly + threads - 1) / threads > inplace_units(static_cast<int>(r), values)) return false;
  }
  return true;
}

FftFactors factor_fft(int n, int max_radix) {
  FftFactors f;
  f.n = n;
  int m = n;
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  if (m != 1 || n < 2) { f.npass = -1; return f; }
  // greedy: the largest supported radix that divides what is left, so that
  // few passes (LDS round trips) remain
  m = n;
  while (m > 1) {
    for (int r : kFftRadices) {
      if (r <= max_radix && m % r == 0) {
        if (f.npass < kMaxPasses) f.radix[f.npass] = r;
        ++f.npass;
        m /= r;
        break;
      }
    }
  }
  if (f.npass > kMaxPasses) f.npass = -1;
  return f;
}

void bspline_weights(double f, double w[4]) {
  const double g = 1.0 - f;
  w[0] = g * g * g / 6.0;
  w[1] = 2.0 / 3.0 - f * f + 0.5 * f * f * f;
  w[2] = 2.0 / 3.0 - g * g + 0.5 * g * g * g;
  w[3] = f * f * f / 6.0;
}

void gauss_legendre(int order, int panels, double lo, double hi,
                    std::vector<double>& nodes, std::vector<double>& weights) {
  std::vector<double> x(order), w(order);
  for (int i = 0; i < (order + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (order + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= order; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = order * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute the derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= order; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = order * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[order - 1 - i] = z;
    w[i] = w[order - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  nodes.resize(static_cast<size_t>(order) * panels);
  weights.resize(nodes.size());
  const double h = (hi - lo) / panels;
  for (int p = 0; p < panels; ++p) {
    const double mid = lo + (p + 0.5) * h;
    for (int i = 0; i < order; ++i) {
      nodes[static_cast<size_t>(p) * order + i] = mid + 0.5 * h * x[i];
      weights[static_cast<size_t>(p) * order + i] = 0.5 * h * w[i];
    }
  }
}

static hrt_status fail(std::string& err, hrt_status s, const char* msg) {
  err = msg;
  return s;
}

hrt_status split_part(const hrt_desc& d, int n_t, const int32_t* t_edges, int n_q,
                      const int32_t* q_edges, int part, hrt_desc& sub, PartView& view,
                      std::string& err) {
  if (n_t < 1 || n_q < 1 || !t_edges || !q_edges)
    return fail(err, HRT_ERR_INVALID_ARG, "a split needs at least one band per axis");
  if (part < 0 || part >= n_t * n_q) return fail(err, HRT_ERR_INVALID_ARG, "no such part");
  if (t_edges[0] != 0 || t_edges[n_t] != d.nt || q_edges[0] != 0 || q_edges[n_q] != d.nq)
    return fail(err, HRT_ERR_INVALID_ARG, "band edges must start at 0 and end at nt / nq");
  for (int i = 0; i < n_t; ++i)
    if (t_edges[i + 1] <= t_edges[i])
      return fail(err, HRT_ERR_INVALID_ARG, "time band edges must increase");
  for (int i = 0; i < n_q; ++i)
    if (q_edges[i + 1] <= q_edges[i])
      return fail(err, HRT_ERR_INVALID_ARG, "slowness band edges must increase");
  const int it = part % n_t, iq = part / n_t;
  const int j_lo = t_edges[it], j_hi = t_edges[it + 1];
  const int l_lo = q_edges[iq], l_hi = q_edges[iq + 1];
  sub = d;
  sub.nt = std::min(d.nt, j_hi + kPartMargin);
  sub.q0 = d.q0 + static_cast<double>(l_lo) * d.dq;
  sub.nq = l_hi - l_lo;
  // traces with a kept sample (j dt >= q0 x_k) at some j < j_hi, plus one
  // whose trapezoid weight in x is then that of an inner trace of the whole
  // grid or multiplies nothing
  const double t_last = static_cast<double>(j_hi - 1) * d.dt;
  int nk = 0;
  while (nk < d.nx && t_last >= sub.q0 * (d.x0 + static_cast<double>(nk) * d.dx)) ++nk;
  sub.nx = std::min(d.nx, nk + 1);
  const double t_end = static_cast<double>(sub.nt - 1) * d.dt;
  int ni = 0;
  while (ni < d.ntau && d.tau0 + static_cast<double>(ni) * d.dtau <= t_end) ++ni;
  sub.ntau = ni;
  if (nk == 0 || ni == 0)
    return fail(err, HRT_ERR_INVALID_ARG, "a part holds no kept sample or no Radon sample");
  view = PartView{};
  view.j_lo = j_lo;
  view.j_hi = j_hi;
  view.data_ld = d.nt;
  view.radon_ld = d.ntau;
  view.radon_row0 = l_lo;
  view.nx_fill = d.nx;
  return HRT_OK;
}

hrt_status build_geometry(const hrt_desc& d, int64_t lds_bytes, Geometry& g,
                          std::string& err, const PartView* view) {
  if (d.nt < 4 || d.nx < 4 || d.ntau < 4 || d.nq < 4)
    return fail(err, HRT_ERR_INVALID_ARG, "every grid needs at least 4 samples");
  if (!(d.dt > 0) || !(d.dx > 0) || !(d.dtau > 0) || !(d.dq > 0))
    return fail(err, HRT_ERR_INVALID_ARG, "sampling intervals must be positive");
  if (!(d.q0 >= 0) || !(d.x0 >= 0) || !(d.tau0 >= 0))
    return fail(err, HRT_ERR_INVALID_ARG, "need q0 >= 0, x0 >= 0, tau0 >= 0");
  if (d.tau0 + (d.ntau - 1) * d.dtau > (d.nt - 1) * d.dt)
    return fail(err, HRT_ERR_INVALID_ARG, "tau range exceeds the time range");
  if (!(d.oversample >= 1.5))
    return fail(err, HRT_ERR_INVALID_ARG, "oversampling must be >= 1.5");
  if (d.flags & ~(HRT_TUNE_MASK | HRT_ACCUMULATE_OUTPUT | HRT_DETERMINISTIC))
    return fail(err, HRT_ERR_INVALID_ARG, "unknown flags");
  if (static_cast<int64_t>(d.nt) * d.nx > (int64_t(1) << 31) ||
      static_cast<int64_t>(d.ntau) * d.nq > (int64_t(1) << 31))
    return fail(err, HRT_ERR_UNSUPPORTED, "panels above 2^31 samples");

  g = Geometry{};
  g.d = d;
  if (view) g.view = *view;
  PartView& v = g.view;
  if (v.j_hi < 0) v.j_hi = d.nt;
  if (v.data_ld == 0) v.data_ld = d.nt;
  if (v.radon_ld == 0) v.radon_ld = d.ntau;
  if (v.nx_fill == 0) v.nx_fill = d.nx;
  if (v.j_lo < 0 || v.j_hi > d.nt || v.j_lo >= v.j_hi || v.data_ld < d.nt ||
      v.radon_ld < d.ntau || v.radon_row0 < 0 || v.nx_fill < d.nx)
    return fail(err, HRT_ERR_INVALID_ARG, "part placement outside the arrays");
  if (static_cast<int64_t>(v.nx_fill) * v.data_ld >= (int64_t{1} << 31) ||
      static_cast<int64_t>(v.radon_row0 + d.nq) * v.radon_ld >= (int64_t{1} << 31))
    return fail(err, HRT_ERR_UNSUPPORTED, "more than 2^31 samples in one array");
  // eq. hypnorm: rescale to the unit square
  g.T = (d.nt - 1) * d.dt;
  g.X = d.x0 + (d.nx - 1) * d.dx;
  const double qh_min = d.q0 * g.X / g.T;
  const double qh_max = (d.q0 + (d.nq - 1) * d.dq) * g.X / g.T;

  // Section 2.1: sector opening and mid angle, inscribed square
  const double psi_min = std::atan(qh_min * qh_min);
  const double psi_max = std::atan(qh_max * qh_max);
  g.beta = psi_max - psi_min;
  g.alpha = 0.5 * (psi_max + psi_min);
  if (!(g.beta > 1e-9))
    return fail(err, HRT_ERR_GEOMETRY, "slowness range too narrow for a sector");
  const double s2a = std::sin(2.0 * g.alpha);
  const double sb = std::sin(g.beta), cb = std::cos(g.beta);
  g.a = sb / std::sqrt(s2a * sb + cb * (s2a + sb) + 1.0);
  // corners (s,y) = (0,0) and (1,1) on the -beta/2 and +beta/2 rays
  g.O1 = g.a * std::sin(g.alpha + kPi / 4) / (std::sqrt(2.0) * std::tan(g.beta / 2));
  g.O2 = g.a * std::cos(g.alpha + kPi / 4) * std::tan(g.beta / 2) / std::sqrt(2.0);
  g.ca = std::cos(g.alpha);
  g.sa = std::sin(g.alpha);
  const double Au = g.a * (g.ca * -0.5 - g.sa * -0.5) + g.O1;
  const double Av = g.a * (g.sa * -0.5 + g.ca * -0.5) + g.O2;
  g.a_r = std::hypot(Au, Av) * cb;
  g.AeA = Au * g.ca + Av * g.sa;
  if (!(g.a_r > 0) || !(g.AeA > 0))
    return fail(err, HRT_ERR_GEOMETRY, "degenerate log-polar placement");

  // trapezoid: keep (j, k) iff j*dt >= q0*(x0 + k*dx)
  g.jmin.assign(d.nx, d.nt);
  for (int k = 0; k < d.nx; ++k) {
    const double xk = d.x0 + static_cast<double>(k) * d.dx;
    const double thr = d.q0 * xk;
    int j = static_cast<int>(std::max(0.0, std::floor(thr / d.dt) - 2.0));
    while (j < d.nt && !(static_cast<double>(j) * d.dt >= thr)) ++j;
    while (j > 0 && static_cast<double>(j - 1) * d.dt >= thr) --j;
    g.jmin[k] = j;
  }

  // data samples mapped by (t^2, x^2) -> T -> P1; eq. lpsamples maxima over
  // neighbour pairs with both samples kept
  auto map = [&](int j, int k, double& phi, double& eta) {
    const double th = (static_cast<double>(j) * d.dt) / g.T;
    const double xh = (d.x0 + static_cast<double>(k) * d.dx) / g.X;
    const double ds = th * th - 0.5, dy = xh * xh - 0.5;
    const double u = g.a * (g.ca * ds - g.sa * dy) + g.O1;
    const double v = g.a * (g.sa * ds + g.ca * dy) + g.O2;
    phi = std::atan2(v, u);
    eta = 0.5 * std::log(u * u + v * v);
  };
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nth = std::min<unsigned>(nth, static_cast<unsigned>(d.nx));
  std::vector<TraceScan> part(nth);
  auto scan = [&](unsigned w) {
    TraceScan& s = part[w];
    const int k0 = static_cast<int>(static_cast<int64_t>(d.nx) * w / nth);
    const int k1 = static_cast<int>(static_cast<int64_t>(d.nx) * (w + 1) / nth);
    std::vector<double> pp(d.nt), pe(d.nt), cp(d.nt), ce(d.nt);
    // previous trace (k0 - 1) for the offset-neighbour differences
    // kept samples of trace k inside the data band: [first(k), j_hi)
    auto first = [&](int k) { return std::max(g.jmin[k], v.j_lo); };
    if (k0 > 0)
      for (int j = first(k0 - 1); j < v.j_hi; ++j) map(j, k0 - 1, pp[j], pe[j]);
    for (int k = k0; k < k1; ++k) {
      const int jm = first(k);
      for (int j = jm; j < v.j_hi; ++j) {
        map(j, k, cp[j], ce[j]);
        s.eta_min = std::min(s.eta_min, ce[j]);
        s.eta_max = std::max(s.eta_max, ce[j]);
        if (j > jm) {
          s.dphi = std::max(s.dphi, std::fabs(cp[j] - cp[j - 1]));
          s.deta = std::max(s.deta, std::fabs(ce[j] - ce[j - 1]));
        }
        if (k > 0 && j >= first(k - 1)) {
          s.dphi = std::max(s.dphi, std::fabs(cp[j] - pp[j]));
          s.deta = std::max(s.deta, std::fabs(ce[j] - pe[j]));
        }
      }
      s.kept += std::max(0, v.j_hi - jm);
      std::swap(pp, cp);
      std::swap(pe, ce);
    }
  };
  {
    std::vector<std::thread> ts;
    for (unsigned w = 1; w < nth; ++w) ts.emplace_back(scan, w);
    scan(0);
    for (auto& t : ts) t.join();
  }
  double eta_min = 1e300, eta_max = -1e300;
  for (const auto& s : part) {
    g.dtheta0 = std::max(g.dtheta0, s.dphi);
    g.drho0 = std::max(g.drho0, s.deta);
    eta_min = std::min(eta_min, s.eta_min);
    eta_max = std::max(eta_max, s.eta_max);
    g.n_kept += s.kept;
  }
  if (!(g.dtheta0 > 0) || !(g.drho0 > 0))
    return fail(err, HRT_ERR_GEOMETRY, "kept samples do not span the lattice");

  // lattice: spacing, kernel half-width, extent (even 5-smooth sizes)
  g.sigma = d.oversample;
  g.dtheta = g.dtheta0 / g.sigma;
  g.drho = g.drho0 / g.sigma;
  g.beta_k = g.beta + 4.0 * g.dtheta;
  if (!(g.beta_k < 1.5))
    return fail(err, HRT_ERR_GEOMETRY, "sector too wide (beta_k >= 1.5 rad)");
  const double ln_ar = std::fabs(std::log(g.a_r));
  const double ln_cb = std::fabs(std::log(std::cos(g.beta_k)));
  const double mt_min = std::ceil(2.0 * g.beta_k / g.dtheta) + 1.0;
  const double mr_min = std::ceil((ln_ar + ln_cb) / g.drho) + 9.0;
  if (mt_min > 1e6 || mr_min > 1e6)
    return fail(err, HRT_ERR_UNSUPPORTED, "log-polar lattice above 10^6 per axis");
  g.Mt = static_cast<int>(next_even_5smooth(static_cast<int64_t>(mt_min)));
  g.Mr = static_cast<int>(next_even_5smooth(static_cast<int64_t>(mr_min)));
  g.K1 = kept_nonneg(g.Mt, g.sigma);
  g.K2 = kept_nonneg(g.Mr, g.sigma);

  // placement on the lattice (integer shifts leave the circular
  // convolution unchanged)
  g.ctheta = g.Mt / 2;
  g.crho = static_cast<int>(std::ceil(ln_ar / g.drho)) + 3;
  // Radon-side radii: e^rho = A + B tau^2, monotone in tau
  const int nq = d.nq;
  g.qA.resize(nq);
  g.qB.resize(nq);
  g.q_i0.resize(nq);
  g.q_w.resize(4 * static_cast<size_t>(nq));
  g.q_scale.resize(nq);
  double rho_min = 1e300, rho_max = -1e300;
  const double th_lo = d.tau0 / g.T;
  const double th_hi = (d.tau0 + (d.ntau - 1) * d.dtau) / g.T;
  for (int l = 0; l < nq; ++l) {
    const double qh = (d.q0 + l * d.dq) * g.X / g.T;
    const double psi = std::atan(qh * qh);
    const double theta = g.alpha - psi;
    g.qA[l] = g.O1 * std::cos(theta) + g.O2 * std::sin(theta) +
              0.5 * g.a * (std::sin(psi) - std::cos(psi));
    g.qB[l] = g.a * std::cos(psi);
    g.q_scale[l] = static_cast<float>(g.X * std::cos(psi) / g.a);
    const double xg = theta / g.dtheta + g.ctheta;
    const double i0 = std::floor(xg);
    double w[4];
    bspline_weights(xg - i0, w);
    g.q_i0[l] = static_cast<int32_t>(i0) - 1;
    for (int t = 0; t < 4; ++t) g.q_w[4 * l + t] = static_cast<float>(w[t]);
    const double e_lo = g.qA[l] + g.qB[l] * th_lo * th_lo;
    const double e_hi = g.qA[l] + g.qB[l] * th_hi * th_hi;
    if (!(e_lo > 0))
      return fail(err, HRT_ERR_GEOMETRY, "Radon sample maps to a non-positive radius");
    rho_min = std::min(rho_min, std::log(e_lo));
    rho_max = std::max(rho_max, std::log(e_hi));
  }
  const double yg_min = std::min(eta_min, rho_min) / g.drho + g.crho;
  const double yg_max = std::max(eta_max, rho_max) / g.drho + g.crho;
  g.u0 = static_cast<int>(std::floor(yg_min)) - 2;
  g.u0 -= (g.u0 & 1);
  g.u1 = static_cast<int>(std::floor(yg_max)) + 4;
  if ((g.u1 - g.u0) & 1) ++g.u1;
  if (g.u0 < 0 || g.u1 > g.Mr)
    return fail(err, HRT_ERR_GEOMETRY, "points fall outside the log-polar lattice");
  const int xq_min = *std::min_element(g.q_i0.begin(), g.q_i0.end());
  const int xq_max = *std::max_element(g.q_i0.begin(), g.q_i0.end()) + 3;
  if (xq_min < 0 || xq_max >= g.Mt)
    return fail(err, HRT_ERR_GEOMETRY, "angles fall outside the log-polar lattice");

  // angle columns any point's taps can reach: both point sets lie within
  // [-beta/2, beta/2]
  {
    const double half = 0.5 * g.beta / g.dtheta;
    g.xw0 = std::max(0, static_cast<int>(std::floor(g.ctheta - half)) - 3);
    int xw1 = std::min(g.Mt, static_cast<int>(std::ceil(g.ctheta + half)) + 4);
    while ((xw1 - g.xw0) % 4 != 0) {  // whole float4 rows
      if (xw1 < g.Mt) ++xw1;
      else if (g.xw0 > 0) --g.xw0;
      else return fail(err, HRT_ERR_UNSUPPORTED, "angle window not a multiple of 4");
    }
    g.W = xw1 - g.xw0;
  }
  if (xq_min < g.xw0 || xq_max >= g.xw0 + g.W)
    return fail(err, HRT_ERR_GEOMETRY, "angles fall outside the log-polar window");
  {
    int ib = 0;
    while ((int64_t{1} << ib) < static_cast<int64_t>(g.W) + 1) ++ib;
    g.x_frac_bits = std::min(24, 31 - ib);
    if (g.x_frac_bits < 16)
      return fail(err, HRT_ERR_UNSUPPORTED, "angle window too wide for the point entries");
  }
  if (static_cast<int64_t>(d.nx) * d.nt >= (int64_t{1} << 31) ||
      static_cast<int64_t>(d.nq) * d.ntau >= (int64_t{1} << 31))
    return fail(err, HRT_ERR_UNSUPPORTED, "more than 2^31 samples in one array");

  // FFT factorisations (needed by the LDS layout)
  if ((g.Mt + 63) / 64 + 64 > 256 || (g.Mr + 63) / 64 + 64 > 256)
    return fail(err, HRT_ERR_UNSUPPORTED, "lattice axis above 12288 points");
  g.fft_t = factor_fft(g.Mt, (d.flags & HRT_TUNE_ROW_RADIX8) ? 8 : 16);
  g.fft_r = factor_fft(g.Mr, (d.flags & HRT_TUNE_COL_RADIX8) ? 8 : 16);
  if (g.fft_t.npass < 0 || g.fft_r.npass < 0)
    return fail(err, HRT_ERR_GEOMETRY, "lattice size is not 5-smooth");

  // row bands and the band kernels' LDS layout
  const int64_t seq = static_cast<int64_t>(padded_len(g.Mt)) * 8;  // one padded sequence
  // largest group of sequences the in-place FFT takes at once (0: none)
  auto inplace_group = [&](int B) {
    int grp = 0;
    for (int b = 1; b <= B; ++b)
      if (fft_fits_inplace(g.fft_t, b, kBandThreads, kInplaceValues)) grp = b;
    return grp;
  };
  // columns a spread chunk may span: its 64-bit accumulator of R rows fills
  // kSpreadLds (at most the whole window)
  auto spread_cols = [&](int R) {
    const int64_t c = int64_t{kSpreadLds} / (int64_t{R} * 8);
    return static_cast<int>(std::min<int64_t>(g.W, c & ~int64_t{3}));
  };
  auto layout = [&](int R, bool commit) {
    const int64_t spread = static_cast<int64_t>(R) * spread_cols(R) * 8;
    const int rr = std::min(R, kRowRows);  // rows of a row-FFT item
    const int grp = inplace_group(rr / 2);
    const int64_t pairs = (rr / 2) * seq;
    const int64_t row = pairs + (grp ? 0 : pairs);
    const int64_t gather = static_cast<int64_t>(R + 3) * g.W * 4;
    if (commit) {
      g.spread_cols = spread_cols(R);
      g.spread_bytes = static_cast<int>(spread);
      g.row_bytes = static_cast<int>(row);
      g.gather_bytes = static_cast<int>(gather);
      g.row_group = grp ? grp : rr / 2;
      g.row_scratch = grp ? -1 : static_cast<int>(pairs);
      g.row_rows = rr;
      g.row_sub_shift = 0;
      while ((rr << g.row_sub_shift) < R) ++g.row_sub_shift;
    }
    return std::max(std::max(spread, row), gather);
  };
  // band heights 2, 4, 8, ...: a band holds a power-of-two number of row
  // pairs, and the last band an even number of rows not above it
  g.R = (d.flags & HRT_TUNE_BAND2) ? 2 : (d.flags & HRT_TUNE_BAND4) ? 4 : kMaxBandRows;
  g.spread_chunk = (d.flags & HRT_TUNE_SPREAD_HALF) ? kSpreadChunk / 2 : kSpreadChunk;
  g.gather_chunk = (d.flags & HRT_TUNE_GATHER_DOUBLE) ? 2 * kGatherChunk : kGatherChunk;
  while (g.R > 2 && layout(g.R, false) > lds_bytes) g.R /= 2;
  if (layout(g.R, false) > lds_bytes || spread_cols(g.R) < 8)
    return fail(err, HRT_ERR_UNSUPPORTED, "angle axis too long for the LDS row bands");
  layout(g.R, true);
  // one column per workgroup by default: two per workgroup (fewer, fuller
  // workgroups) measured slower at C3, the column pass being short of waves
  g.col_batch = (d.flags & HRT_TUNE_COL_PAIRS) ? 2 : 1;
  g.inplace_col = fft_fits_inplace(g.fft_r, g.col_batch, kColThreads, kInplaceValues);
  g.col_bytes = (g.inplace_col ? g.col_batch : 2) * padded_len(g.Mr) * 8;
  if (g.col_bytes > lds_bytes + kBandStaticLds)
    return fail(err, HRT_ERR_UNSUPPORTED, "log-radius axis too long for an LDS column");
  g.nbands = (g.u1 - g.u0 + g.R - 1) / g.R;

  return HRT_OK;
}

namespace {

// Lattice coordinates (column, row) and smear weight of data sample (j, k):
// (t^2, x^2) -> T -> P1, W = 2 a^2 t^ e^-eta w_t w_x dt^ dx^ (eqs. f,
// transformT, transformP; trapezoid rule in t and x).
void place_data(const Geometry& g, int j, int k, double& xg, double& yg, double& w) {
  const hrt_desc& d = g.d;
  const double th = (static_cast<double>(j) * d.dt) / g.T;
  const double xh = (d.x0 + static_cast<double>(k) * d.dx) / g.X;
  const double ds = th * th - 0.5, dy = xh * xh - 0.5;
  const double u = g.a * (g.ca * ds - g.sa * dy) + g.O1;
  const double v = g.a * (g.sa * ds + g.ca * dy) + g.O2;
  const double r2 = u * u + v * v;
  xg = std::atan2(v, u) / g.dtheta + g.ctheta;
  yg = 0.5 * std::log(r2) / g.drho + g.crho;
  const double wt = (j == 0 || j == d.nt - 1) ? 0.5 : 1.0;
  const double wx = (k == 0 || k == d.nx - 1) ? 0.5 : 1.0;
  w = 2.0 * g.a * g.a * th * wt * wx * (d.dt / g.T) * (d.dx / g.X) / std::sqrt(r2);
}

// Row coordinate of Radon sample (i, l): e^rho = A_l + B_l tau^2 (eq. B3tauq).
double radon_row(const Geometry& g, int i, int l) {
  const double th = (g.d.tau0 + static_cast<double>(i) * g.d.dtau) / g.T;
  return std::log(g.qA[l] + g.qB[l] * th * th) / g.drho + g.crho;
}

// Cuts every band's list into ceil(n / max_entries) chunks of equal size
// (a band with an empty list still gets one empty chunk).
void make_chunks(int nb, int max_entries, BandLists& L) {
  L.chunk_off.clear();
  L.chunk_band.clear();
  L.band_chunk.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    L.band_chunk[b] = static_cast<int32_t>(L.chunk_band.size());
    const int64_t lo = L.off[b], n = L.off[b + 1] - lo;
    const int64_t m = std::max<int64_t>(1, (n + max_entries - 1) / max_entries);
    for (int64_t i = 0; i < m; ++i) {
      L.chunk_off.push_back(lo + n * i / m);
      L.chunk_band.push_back(b);
    }
  }
  L.band_chunk[nb] = static_cast<int32_t>(L.chunk_band.size());
  L.chunk_off.push_back(L.off[nb]);
}

// Spread chunks: consecutive entries of a band, at most the band's equal
// share of ceil(n / max_entries) chunks each, cut earlier where the window
// columns the stencils touch would span more than g.spread_cols (the
// columns [c_lo, c_hi) of a chunk are rounded out to multiples of 4).  A
// band's list runs in sample order, which moves steadily along the angle
// inside one band, so a chunk spans a fraction of the window.  Records each
// chunk's columns and the place of its partial rows (R x wc floats).
void make_spread_chunks(const Geometry& g, int max_entries, BandLists& L) {
  const int nb = g.nbands;
  L.chunk_off.clear();
  L.chunk_band.clear();
  L.chunk_col.clear();
  L.chunk_hp.clear();
  L.band_chunk.assign(nb + 1, 0);
  int64_t hp = 0;
  auto close = [&](int b, int64_t start, int c_lo, int c_hi) {
    L.chunk_off.push_back(start);
    L.chunk_band.push_back(b);
    const int wc = c_hi > c_lo ? c_hi - c_lo : 0;
    L.chunk_col.push_back(wc ? c_lo : 0);
    L.chunk_col.push_back(wc);
    L.chunk_hp.push_back(hp);
    hp += static_cast<int64_t>(g.R) * wc;
  };
  for (int b = 0; b < nb; ++b) {
    L.band_chunk[b] = static_cast<int32_t>(L.chunk_band.size());
    const int64_t lo = L.off[b], hi = L.off[b + 1], n = hi - lo;
    const int64_t m = std::max<int64_t>(1, (n + max_entries - 1) / max_entries);
    const int64_t share = std::max<int64_t>(1, (n + m - 1) / m);
    int64_t start = lo;
    int c_lo = 0, c_hi = 0;  // empty column range
    for (int64_t i = lo; i < hi; ++i) {
      const int cx = static_cast<int>(L.e[i].xq >> g.x_frac_bits) - 1;  // first tap column
      const int a = cx & ~3, z = (cx + 4 + 3) & ~3;
      const int n_lo = i == start ? a : std::min(c_lo, a);
      const int n_hi = i == start ? z : std::max(c_hi, z);
      if (i > start && (i - start == share || n_hi - n_lo > g.spread_cols)) {
        close(b, start, c_lo, c_hi);
        start = i;
        c_lo = a;
        c_hi = z;
      } else {
        c_lo = n_lo;
        c_hi = n_hi;
      }
    }
    close(b, start, c_lo, c_hi);
  }
  L.band_chunk[nb] = static_cast<int32_t>(L.chunk_band.size());
  L.chunk_off.push_back(L.off[nb]);
  L.hp_floats = hp;
}

// Band lists of one point set.  `place(p, xg, yg, w)` gives the coordinates
// of point p in [0, npts) and returns false for points outside the
// trapezoid.  Points are placed in parallel over contiguous index ranges,
// counted per band, then written at per-(thread, band) offsets, so every
// list comes out in increasing index order.
template <class PlaceF>
hrt_status build_lists(const Geometry& g, int64_t npts, PlaceF place, BandLists& spread,
                       BandLists& own, std::string& err) {
  // place(p, xg, yg, w, idx) also gives the index stored in the entry
  const int nb = g.nbands;
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nth = static_cast<unsigned>(std::min<int64_t>(nth, std::max<int64_t>(1, npts / 4096)));
  std::vector<std::vector<int64_t>> cs(nth, std::vector<int64_t>(nb, 0)), co = cs;
  std::vector<int> bad(nth, 0);
  const double xs = std::ldexp(1.0, g.x_frac_bits), ys = std::ldexp(1.0, kYFracBits);
  // bands whose rows meet the stencil rows iy-1 .. iy+2, and the band of iy
  auto bands_of = [&](int iy, int& b_lo, int& b_hi, int& b_own) {
    b_lo = std::max(0, (iy - 1 - g.u0) / g.R);
    b_hi = std::min(nb - 1, (iy + 2 - g.u0) / g.R);
    b_own = (iy - g.u0) / g.R;
  };
  auto pass = [&](unsigned w, bool fill, std::vector<int64_t>* ps, std::vector<int64_t>* po) {
    const int64_t p0 = npts * w / nth, p1 = npts * (w + 1) / nth;
    for (int64_t p = p0; p < p1; ++p) {
      double xg, yg, wt;
      uint32_t idx = 0;
      if (!place(p, xg, yg, wt, idx)) continue;
      const double fy = std::floor(yg);
      const int iy = static_cast<int>(fy);
      const double xr = xg - g.xw0;
      if (!(iy - 1 >= g.u0 && iy + 2 < g.u1 && xr >= 1.0 && xr + 3.0 < g.W)) {
        bad[w] = 1;
        continue;
      }
      int b_lo, b_hi, b_own;
      bands_of(iy, b_lo, b_hi, b_own);
      const uint32_t xq = static_cast<uint32_t>(std::llround(xr * xs));
      for (int b = b_lo; b <= b_hi; ++b) {
        if (!fill) { ++cs[w][b]; continue; }
        const double base = g.u0 + b * g.R - 2;
        PointEntry e{idx, xq,
                     static_cast<uint32_t>(std::llround((yg - base) * ys)),
                     static_cast<float>(wt)};
        spread.e[(*ps)[b]++] = e;
        if (b == b_own) own.e[(*po)[b]++] = e;
      }
      if (!fill) ++co[w][b_own];
    }
  };
  auto run = [&](bool fill, std::vector<std::vector<int64_t>>* ps,
                 std::vector<std::vector<int64_t>>* po) {
    std::vector<std::thread> ts;
    for (unsigned w = 1; w < nth; ++w)
      ts.emplace_back(pass, w, fill, ps ? &(*ps)[w] : nullptr, po ? &(*po)[w] : nullptr);
    pass(0, fill, ps ? &(*ps)[0] : nullptr, po ? &(*po)[0] : nullptr);
    for (auto& t : ts) t.join();
  };
  run(false, nullptr, nullptr);
  for (int b : bad)
    if (b) return fail(err, HRT_ERR_GEOMETRY, "a sample falls outside the band layout");
  // offsets: band-major, thread-minor
  auto offsets = [&](std::vector<std::vector<int64_t>>& c, BandLists& L) {
    L.off.assign(nb + 1, 0);
    std::vector<std::vector<int64_t>> at(nth, std::vector<int64_t>(nb));
    int64_t o = 0;
    for (int b = 0; b < nb; ++b) {
      L.off[b] = o;
      for (unsigned w = 0; w < nth; ++w) {
        at[w][b] = o;
        o += c[w][b];
      }
    }
    L.off[nb] = o;
    L.e.resize(static_cast<size_t>(o));
    return at;
  };
  auto ps = offsets(cs, spread);
  auto po = offsets(co, own);
  run(true, &ps, &po);
  make_spread_chunks(g, g.spread_chunk, spread);
  make_chunks(nb, g.gather_chunk, own);
  return HRT_OK;
}

// Largest over the cells of any band of the sum of |w| x B3 x B3 of the
// entries of a spread list, with the coordinates decoded as the kernels
// decode them.
double list_cmax(const Geometry& g, const BandLists& L) {
  const int nb = g.nbands;
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nth = std::min<unsigned>(nth, static_cast<unsigned>(nb));
  std::vector<double> best(nth, 0.0);
  auto work = [&](unsigned w) {
    std::vector<double> cell;
    for (int b = static_cast<int>(w); b < nb; b += static_cast<int>(nth)) {
      const int n0 = g.u0 + b * g.R;
      const int nr = std::min(g.R, g.u1 - n0);
      cell.assign(static_cast<size_t>(nr) * g.W, 0.0);
      for (int64_t i = L.off[b]; i < L.off[b + 1]; ++i) {
        const PointEntry& e = L.e[i];
        const double x = std::ldexp(static_cast<double>(e.xq), -g.x_frac_bits);
        const double y = std::ldexp(static_cast<double>(e.yq), -kYFracBits);
        const double fx = std::floor(x), fy = std::floor(y);
        const int cx = static_cast<int>(fx) - 1, cy = static_cast<int>(fy) - 3;
        double wx[4], wy[4];
        bspline_weights(x - fx, wx);
        bspline_weights(y - fy, wy);
        for (int bb = 0; bb < 4; ++bb) {
          const int rl = cy + bb;
          if (rl < 0 || rl >= nr) continue;
          for (int aa = 0; aa < 4; ++aa)
            cell[static_cast<size_t>(rl) * g.W + cx + aa] += std::fabs(e.w) * wx[aa] * wy[bb];
        }
      }
      for (double c : cell) best[w] = std::max(best[w], c);
    }
  };
  std::vector<std::thread> ts;
  for (unsigned w = 1; w < nth; ++w) ts.emplace_back(work, w);
  work(0);
  for (auto& t : ts) t.join();
  return *std::max_element(best.begin(), best.end());
}

}  // namespace

hrt_status build_point_tables(const Geometry& g, PointTables& t, std::string& err) {
  const hrt_desc& d = g.d;
  const PartView& v = g.view;
  hrt_status s = build_lists(
      g, static_cast<int64_t>(d.nx) * d.nt,
      [&](int64_t p, double& xg, double& yg, double& w, uint32_t& idx) {
        const int k = static_cast<int>(p / d.nt), j = static_cast<int>(p % d.nt);
        if (j < g.jmin[k] || j < v.j_lo || j >= v.j_hi) return false;
        place_data(g, j, k, xg, yg, w);
        idx = static_cast<uint32_t>(static_cast<int64_t>(k) * v.data_ld + j);
        return true;
      },
      t.data_spread, t.data_own, err);
  if (s != HRT_OK) return s;
  std::vector<double> qx(d.nq);
  for (int l = 0; l < d.nq; ++l) {
    const double qh = (d.q0 + l * d.dq) * g.X / g.T;
    qx[l] = (g.alpha - std::atan(qh * qh)) / g.dtheta + g.ctheta;
  }
  s = build_lists(
      g, static_cast<int64_t>(d.nq) * d.ntau,
      [&](int64_t p, double& xg, double& yg, double& w, uint32_t& idx) {
        const int l = static_cast<int>(p / d.ntau), i = static_cast<int>(p % d.ntau);
        idx = static_cast<uint32_t>(static_cast<int64_t>(v.radon_row0 + l) * v.radon_ld + i);
        xg = qx[l];
        yg = radon_row(g, i, l);
        w = g.q_scale[l];
        return true;
      },
      t.radon_spread, t.radon_own, err);
  if (s != HRT_OK) return s;
  t.cmax_data = list_cmax(g, t.data_spread);
  t.cmax_radon = list_cmax(g, t.radon_spread);
  return HRT_OK;
}

void alg_bytes_kernels(const Geometry& g, bool adjoint, double out[3]) {
  const double U = g.u1 - g.u0;
  const double spec = 8.0 * g.K1 * U;  // complex64 half spectrum, used rows
  const double n_data_in = 4.0 * static_cast<double>(g.n_kept);
  const double n_data_out = 4.0 * static_cast<double>(g.d.nx) * g.d.nt;
  const double n_radon = 4.0 * static_cast<double>(g.d.nq) * g.d.ntau;
  out[0] = (adjoint ? n_radon : n_data_in) + spec;
  out[1] = 2.0 * spec + 8.0 * g.K1 * static_cast<double>(g.K2);
  out[2] = spec + (adjoint ? n_data_out : n_radon);
}

double alg_bytes_forward(const Geometry& g) {
  double b[3];
  alg_bytes_kernels(g, false, b);
  return b[0] + b[1] + b[2];
}

double alg_bytes_adjoint(const Geometry& g) {
  double b[3];
  alg_bytes_kernels(g, true, b);
  return b[0] + b[1] + b[2];
}

void fill_info(const Geometry& g, hrt_info* o) {
  o->T = g.T;
  o->X = g.X;
  o->alpha = g.alpha;
  o->beta = g.beta;
  o->a = g.a;
  o->O1 = g.O1;
  o->O2 = g.O2;
  o->a_r = g.a_r;
  o->dtheta0 = g.dtheta0;
  o->drho0 = g.drho0;
  o->dtheta = g.dtheta;
  o->drho = g.drho;
  o->beta_k = g.beta_k;
  o->m_theta = g.Mt;
  o->m_rho = g.Mr;
  o->k1_kept = g.K1;
  o->k2_kept = g.K2;
  o->row_lo = g.u0;
  o->row_hi = g.u1;
  o->band_rows = g.R;
  o->n_bands = g.nbands;
  o->n_kept = g.n_kept;
  o->workspace_bytes = 0;
  o->alg_bytes_fwd = alg_bytes_forward(g);
  o->alg_bytes_adj = alg_bytes_adjoint(g);
}

}  // namespace hrt
