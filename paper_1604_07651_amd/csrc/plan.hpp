// Host-side plan of the log-polar hyperbolic Radon transform: float64
// geometry, lattice sizing, row bands and the small per-trace / per-slowness
// tables the kernels read.  Pure C++ (no HIP), so hrt_plan_describe works on
// a machine without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hrt.h"

namespace hrt {

// FFT passes: at most 8, radices from this list, largest first.
constexpr int kMaxPasses = 8;
constexpr int kFftRadices[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
// Tallest row band of the spread / gather kernels, and the rows one
// workgroup of the row FFT kernels takes (a band of R rows is R / kRowRows
// row items, or one item when it is lower).
constexpr int kMaxBandRows = 8;
constexpr int kRowRows = 4;
// Dynamic LDS of a spread workgroup: the 64-bit accumulator of the band's
// rows over the chunk's columns, which bounds the columns a spread chunk may
// span (800 at 8 rows; 38 and 30 KB measured slower at C3).
constexpr int kSpreadLds = 50 * 1024;
// Static LDS of the band kernels (twiddles, reduction slots), rounded up.
constexpr int kBandStaticLds = 4096;
// Threads of the band kernels and of the column kernel.
constexpr int kBandThreads = 512;
constexpr int kColThreads = 256;
// The in-place FFT holds at most this many complex values per thread.
constexpr int kInplaceValues = 16;
// Point lists are cut into chunks of at most these many entries by default
// (spread: each chunk writes one partial of its band's rows over the
// columns it spans; gather: one workgroup).
constexpr int kSpreadChunk = 5120;
constexpr int kGatherChunk = 4096;
// Fraction bits of the log-radius coordinate in a point entry (the integer
// part, the row relative to the band's first tap row, needs 3 bits).
constexpr int kYFracBits = 28;

// LDS layout of the FFT sequences: element e of a sequence sits at slot
// lpad(e) = e + e/16, so that the stores of the early passes, R*Ns complex
// values apart, spread over the LDS banks instead of piling onto a few; a
// sequence of n elements takes padded_len(n) slots.
constexpr int lpad(int e) { return e + (e >> 4); }
constexpr int padded_len(int n) { return n + (n >> 4) + 2; }

// Butterflies a thread holds in an in-place radix-R pass with at most
// `values` complex values per thread (capped at 2 to bound the registers of
// small radices).
constexpr int inplace_units(int R, int values) { return values / R < 2 ? values / R : 2; }

// True when the in-place FFT can hold all butterflies of `batch` sequences
// of f.n points with `threads` threads: ceil(batch*n/R / threads) <=
// inplace_units(R, values) for every radix R of f.
struct FftFactors;
bool fft_fits_inplace(const FftFactors& f, int batch, int threads, int values);

// Mixed-radix factorisation of an FFT length (radices of kFftRadices).
struct FftFactors {
  int n = 0;
  int npass = 0;
  int radix[kMaxPasses] = {};
};

// Radices are taken largest first from kFftRadices, up to max_radix.
FftFactors factor_fft(int n, int max_radix = 16);

// Where a plan's grids sit in the caller's arrays, and the part of its data
// grid it takes in (Section 4, eq. tsplit: the integral over t cut at
// intermediate times).  The defaults are the whole grids in arrays
// [nx][nt] and [nq][ntau].
struct PartView {
  int j_lo = 0, j_hi = -1;        // data samples j in [j_lo, j_hi) (-1: nt)
  int data_ld = 0, radon_ld = 0;  // row strides of the two arrays (0: nt, ntau)
  int radon_row0 = 0;             // the plan's first slowness row in the Radon array
  int nx_fill = 0;                // traces of the data array (0: nx)
};

// Samples a part's data and Radon rows reach beyond its last time sample:
// the reach of the cubic interpolation in time of the direct summation.
constexpr int kPartMargin = 2;

// The sub-problem of part `part` = iq * n_t + it of a split of the grids of
// `d` into time bands [t_edges[it], t_edges[it + 1]) and slowness bands
// [q_edges[iq], q_edges[iq + 1]) (Section 4, eq. tsplit, and the slowness
// split of Section 5).  The part is a plain problem of its own: data
// samples 0 .. min(nt, j_hi + kPartMargin) - 1 (rescaled by its own T) of
// the traces that hold kept samples in its band plus one, its slowness rows,
// and the Radon samples tau_i <= its last time; `view` places it in the
// whole arrays and restricts its data samples to its band.
hrt_status split_part(const hrt_desc& d, int n_t, const int32_t* t_edges, int n_q,
                      const int32_t* q_edges, int part, hrt_desc& sub, PartView& view,
                      std::string& err);

// Everything the plan derives from the grids (Sections 2.1, 2.2, 4).
struct Geometry {
  hrt_desc d{};
  PartView view;              // resolved: no defaults left
  // eq. hypnorm
  double T = 0, X = 0;
  // Section 2.1: sector, square, first contribution
  double alpha = 0, beta = 0, a = 0, O1 = 0, O2 = 0, a_r = 0;
  double ca = 0, sa = 0;      // cos(alpha), sin(alpha)
  double AeA = 0;             // (corner A) . (cos alpha, sin alpha) > 0
  // eq. lpsamples and lattice extent
  double dtheta0 = 0, drho0 = 0, dtheta = 0, drho = 0, beta_k = 0, sigma = 0;
  int Mt = 0, Mr = 0;         // lattice size (angle, log radius)
  int K1 = 0, K2 = 0;         // non-negative frequencies inside L per axis
  // lattice placement: node m sits at theta = (m - ctheta) dtheta, node n at
  // rho = (n - crho) drho; all used nodes fall inside the array.
  int ctheta = 0, crho = 0;
  int u0 = 0, u1 = 0;         // lattice rows touched by any point [u0, u1)
  int R = 0, nbands = 0;      // row band height (a power of two) and band count
  int row_rows = 0;           // rows of a row-FFT item: min(R, kRowRows)
  int row_sub_shift = 0;      // log2 of the row items per band
  // row FFTs (forward and inverse): in place `row_group` sequences at a
  // time, or through an LDS scratch of `row_group` sequences at byte offset
  // row_scratch (-1 when in place); the column FFT in place or not
  int row_group = 0, row_scratch = -1;
  bool inplace_col = false;
  int col_batch = 1;          // columns per workgroup of the column kernel
  int xw0 = 0, W = 0;         // angle columns [xw0, xw0 + W) points can touch (W % 4 == 0)
  int x_frac_bits = 0;         // fraction bits of the angle coordinate in a point entry
  int spread_cols = 0;         // most window columns one spread chunk spans (% 4 == 0)
  int spread_chunk = 0;        // most entries of a spread chunk
  int gather_chunk = 0;        // most entries of a gather chunk
  // dynamic LDS per workgroup of the spread, row FFT, column and gather
  // kernels
  int spread_bytes = 0, row_bytes = 0, col_bytes = 0, gather_bytes = 0;
  int64_t n_kept = 0;          // kept samples inside the data band
  std::vector<int32_t> jmin;  // [nx] first kept time sample of each trace
  // Radon side, per slowness l
  std::vector<double> qA, qB;     // e^rho = qA + qB tau^2
  std::vector<int32_t> q_i0;      // first angle tap of the column
  std::vector<float> q_w;         // 4 angle tap weights of the column
  std::vector<float> q_scale;     // X cos(psi)/a
  FftFactors fft_t, fft_r;
};

// One point of a band's list, 16 bytes: the sample's linear index in its
// array (k*data_ld + j for data, (radon_row0 + l)*radon_ld + i for Radon;
// k*nt + j and l*ntau + i for a whole-grid plan), its lattice coordinates
// in fixed point relative to the band (angle: column - xw0 with
// x_frac_bits fraction bits; log radius: row - (n0 - 2) with kYFracBits
// fraction bits, n0 the band's first row), and its weight (the smear weight
// of a data sample, X cos(psi)/a of a Radon sample).
struct PointEntry {
  uint32_t idx;
  uint32_t xq;
  uint32_t yq;
  float w;
};

// Per-band point lists in one array, band b at [off[b], off[b+1]), each in
// increasing idx order.  `spread` lists every sample whose 4x4 stencil
// reaches a row of the band (a sample can be in two or three lists); `own`
// lists the samples whose base row floor(row coordinate) lies in the band
// (each sample once).
struct BandLists {
  std::vector<PointEntry> e;
  std::vector<int64_t> off;
  // the lists cut into chunks: chunk c covers e[chunk_off[c] .. chunk_off[c+1])
  // of band chunk_band[c]; band b has chunks [band_chunk[b], band_chunk[b+1])
  std::vector<int64_t> chunk_off;
  std::vector<int32_t> chunk_band;
  std::vector<int32_t> band_chunk;
  // spread lists only: the window columns [c_lo, c_lo + wc) that chunk c's
  // stencils touch (c_lo and wc multiples of 4, wc <= spread_cols; wc = 0
  // for an empty chunk) as chunk_col[2c], chunk_col[2c+1], and where its
  // partial rows, R x wc floats, start in the partial buffer (hp_floats in
  // all)
  std::vector<int32_t> chunk_col;
  std::vector<int64_t> chunk_hp;
  int64_t hp_floats = 0;
};

struct PointTables {
  BandLists data_spread, data_own, radon_spread, radon_own;
  // largest sum of |weight| x tap over the cells of a band, per point set:
  // bounds every accumulated cell by this times the largest |input|
  double cmax_data = 0, cmax_radon = 0;
};

// Places every kept data sample and every Radon sample on the lattice in
// float64 (eqs. transformT, transformP, B3tx2, B3tauq) and sorts them into
// the band lists.
hrt_status build_point_tables(const Geometry& g, PointTables& t, std::string& err);

// Validates `d` and computes the geometry.  `lds_bytes` is the per-workgroup
// LDS the band kernels may use (it bounds the band height).  With a `view`,
// only data samples inside its band count (eq. lpsamples, the lattice rows,
// the point lists).  Returns HRT_OK or an error with a message in `err`.
hrt_status build_geometry(const hrt_desc& d, int64_t lds_bytes, Geometry& g,
                          std::string& err, const PartView* view = nullptr);

// Algorithmic bytes of one forward / adjoint (per kernel: inputs read once,
// outputs written once).
double alg_bytes_forward(const Geometry& g);
double alg_bytes_adjoint(const Geometry& g);
// Per kernel of one direction: [0] spread+row FFT, [1] column pass,
// [2] row inverse FFT + gather.
void alg_bytes_kernels(const Geometry& g, bool adjoint, double out[3]);

void fill_info(const Geometry& g, hrt_info* out);

// Composite Gauss-Legendre rule of `order` nodes per panel on [lo, hi].
void gauss_legendre(int order, int panels, double lo, double hi,
                    std::vector<double>& nodes, std::vector<double>& weights);

// Cubic B-spline weights of the four taps of a point whose fractional
// lattice offset is f in [0, 1).
void bspline_weights(double f, double w[4]);

}  // namespace hrt
