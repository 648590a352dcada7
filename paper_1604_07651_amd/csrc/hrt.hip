// gfx950 kernels and C ABI of the log-polar hyperbolic Radon transform.
//
// One direction of the transform (lp_kernels.hpp) is an absmax pass and
// three kernels over an Mt x Mr lattice (angle theta x log radius rho) whose
// rows [u0, u1) are all that any point touches.  Only the non-negative half
// spectrum along theta inside the band limit L (k1 < K1) ever reaches HBM,
// stored column-major as S[k1][row].  Point coordinates are placed once per
// plan in float64 on the host (eqs. transformT, transformP; the Radon side
// e^rho = A_l + B_l tau^2) and kept on the device as per-band lists of
// entries of 16 bytes (data) or 8 bytes (Radon, the angle coordinate and
// weight coming from a per-slowness table); everything on the lattice is
// float32 with float32 accumulation, except inside one chunk of the
// spread, whose taps (float64 products of a float32 sample and its float32
// B-spline weights) are summed exactly in 64-bit fixed point and rounded
// once to float32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "direct_kernels.hpp"
#include "hrt.h"
#include "lp_kernels.hpp"
#include "plan.hpp"
#include "ista_kernels.hpp"
#include "plan_kernels.hpp"

namespace hrt {
constexpr uint64_t kMagic = 0x6872745f706c616eull;
constexpr uint64_t kGraphMagic = 0x6872745f67726170ull;
constexpr uint64_t kBatchMagic = 0x6872745f62617463ull;
constexpr uint64_t kSplitMagic = 0x6872745f73706c74ull;
static_assert(kTwLds * sizeof(float2) + kNtBand / 64 * sizeof(float) <= kBandStaticLds,
              "static LDS");
static_assert(sizeof(PointEntry) == sizeof(uint4), "point entry layout");
// work-item lists of a plan's launches
enum {
  kItAbsmax = 0,       // partial maxima
  kItSpreadData = 1,   // chunks of the data spread list
  kItSpreadRadon = 2,  // chunks of the Radon spread list
  kItBands = 3,        // bands (row FFTs)
  kItCols = 4,         // column groups (column pass)
  kItGatherRadon = 5,  // chunks of the Radon owned list (forward gather)
  kItGatherData = 6,   // chunks of the data owned list (adjoint gather)
  kItemSets = 7
};
}  // namespace hrt

// ==================================================================== ABI ==

using namespace hrt;

struct hrt_plan_s {
  uint64_t magic;
  int device;
  Geometry g;
  hrt_info info;
  DevGeo dg;
  DirectGeo dd;
  int64_t direct_rows_bytes = 0;  // LDS of k_direct_adj_rows; 0: use k_direct_adj
  FftDev ft, fr;
  float2* S = nullptr;
  float2* K = nullptr;
  float2* tw_t = nullptr;
  float2* tw_r = nullptr;
  int* jmin = nullptr;
  // point lists (kDataSpread ... kRadonOwn), cut into chunks
  uint4* ent[4] = {};       // data lists: 16-byte entries
  uint2* ent2[4] = {};      // Radon lists: {sample index, log-radius coordinate}
  uint2* q_tab = nullptr;   // per slowness: {angle coordinate, weight bits}
  uint64_t rdiv_m = 0;      // idx / radon_ld = (idx * rdiv_m) >> rdiv_s
  int rdiv_s = 0;
  int64_t* chunk_off[4] = {};
  int* chunk_band[4] = {};
  int* band_chunk[4] = {};
  int2* chunk_col[4] = {};       // spread lists: columns {c_lo, wc} of each chunk
  int64_t* chunk_hp[4] = {};     // spread lists: start of each chunk's partial rows
  int64_t hp_floats[4] = {};     // spread lists: floats of all partial rows
  int nchunks[4] = {};
  float* Hp = nullptr;      // partial rows of the spread chunks (float32)
  float* Cr = nullptr;      // real lattice rows after the inverse row FFT
  float* absmax = nullptr;  // kAbsMaxBlocks partial maxima of the current input
  float* gmax = nullptr;    // partial maxima of the forward's output, one per gather chunk
  double* dot = nullptr;    // kDotBlocks partial sums of the power iteration
  DevGeo* geo_dev = nullptr;         // the plan's descriptor, on the device
  int2* items[kItemSets] = {};       // work items (gather 0, index)
  int nitems[kItemSets] = {};
  // the XCD of every band (row FFT and gather items) and the band of every
  // chunk of the two owned lists, for the XCD-aware order of batches
  std::vector<int> band_xcd;
  std::vector<int32_t> own_chunk_band[2];  // [0] Radon, [1] data
  // per-kernel timing (hrt_profile_begin / hrt_profile_end)
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_stage;
  int prof_used = 0;
};

namespace {

thread_local std::string g_last_error;

hrt_status set_err(hrt_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

hrt_status hip_err(hipError_t e, const char* what) {
  return set_err(HRT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HRT_HIP(call, what)                                        \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return hip_err(e_, what);                \
  } while (0)

FftDev to_dev(const FftFactors& f) {
  FftDev d{};
  d.n = f.n;
  d.npass = f.npass;
  d.codes = 0;
  for (int i = 0; i < f.npass; ++i)
    d.codes |= static_cast<unsigned long long>(f.radix[i]) << (8 * i);
  return d;
}

// Two-level twiddle table of length n: exp(-2 pi i 64 a / n) for
// a < ceil(n / 64), then exp(-2 pi i b / n) for b < 64.
std::vector<float2> twiddles(int n) {
  const int nhi = (n + 63) / 64;
  std::vector<float2> t(nhi + 64);
  const double two_pi = 6.283185307179586476925286766559;
  auto put = [&](int i, double j) {
    const double a = -two_pi * j / n;
    t[i] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(std::sin(a)));
  };
  for (int a = 0; a < nhi; ++a) put(a, 64.0 * a);
  for (int b = 0; b < 64; ++b) put(nhi + b, b);
  return t;
}

// Workgroup i of a launch runs on XCD i mod kXcds (the dispatcher deals
// workgroups round-robin over the XCDs, each with its own L2).  A single
// plan's row FFT and gather items are ordered so that a band's work runs on
// one XCD: the real rows its inverse row FFT writes are read by its gather
// chunks from the same L2.  (The spread keeps plain order: there, balance
// over the XCDs matters more than locality.)  `per_xcd[x]` lists the items
// of the bands given to XCD x; item i of the result comes from queue
// i mod kXcds, and where a queue has run out the item is (0, -1), a
// workgroup that exits at once.
constexpr int kXcds = 8;
std::vector<int2> xcd_order(const std::vector<std::vector<int2>>& per_xcd) {
  size_t len = 0;
  for (const auto& q : per_xcd) len = std::max(len, q.size());
  std::vector<int2> out(len * kXcds, make_int2(0, -1));
  for (int x = 0; x < kXcds; ++x)
    for (size_t k = 0; k < per_xcd[x].size(); ++k) out[k * kXcds + x] = per_xcd[x][k];
  return out;
}

// Row-FFT items of a plan: band b's rows from s * row_rows on are item
// (b << row_sub_shift) + s, for every s whose rows exist.
std::vector<int> row_items(const Geometry& g) {
  std::vector<int> out;
  for (int b = 0; b < g.nbands; ++b) {
    const int rows = std::min(g.R, g.u1 - (g.u0 + b * g.R));
    for (int s = 0; s * g.row_rows < rows; ++s) out.push_back((b << g.row_sub_shift) + s);
  }
  return out;
}

// Allocation-failure injection, for tests of the clean-up paths:
// HRT_FAIL_ALLOC=k (k >= 1) in the environment makes the k-th device
// allocation of every plan creation fail with HRT_ERR_OOM.
thread_local long g_fail_countdown = 0;
void arm_fail_alloc() {
  const char* e = std::getenv("HRT_FAIL_ALLOC");
  g_fail_countdown = e ? std::max(0L, std::atol(e)) : 0;
}

template <typename T>
hrt_status dev_alloc(T** p, size_t count, size_t& total) {
  if (g_fail_countdown > 0 && --g_fail_countdown == 0) {
    *p = nullptr;
    return set_err(HRT_ERR_OOM, "injected allocation failure (HRT_FAIL_ALLOC)");
  }
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e != hipSuccess) return set_err(HRT_ERR_OOM, "hipMalloc failed");
  total += bytes;
  return HRT_OK;
}

template <typename T>
hrt_status upload(T* dst, const std::vector<T>& src) {
  if (src.empty()) return HRT_OK;
  HRT_HIP(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice),
          "upload");
  return HRT_OK;
}

void free_plan(hrt_plan_s* p) {
  void* ptrs[] = {p->S, p->K, p->tw_t, p->tw_r, p->jmin, p->absmax, p->gmax, p->Hp, p->Cr,
                  p->dot, p->geo_dev, p->q_tab};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (int2* q : p->items)
    if (q) (void)hipFree(q);
  for (int i = 0; i < 4; ++i) {
    void* lists[] = {p->ent[i], p->ent2[i], p->chunk_off[i], p->chunk_band[i],
                     p->band_chunk[i], p->chunk_col[i], p->chunk_hp[i]};
    for (void* q : lists)
      if (q) (void)hipFree(q);
  }
}

double b_squared(double xi) {  // (sinc^4)^2 of the cubic B-spline
  if (xi == 0.0) return 1.0;
  const double pi = 3.14159265358979323846;
  const double s = std::sin(pi * xi) / (pi * xi);
  const double s2 = s * s, s4 = s2 * s2;
  return s4 * s4;
}

// Kernel spectrum of eq. finiteconv, divided by the B-spline transforms of
// eq. B3tauq, restricted to L (k1 < K1, |k2| < K2), by composite
// Gauss-Legendre quadrature in float64 on the device.
hrt_status build_kernel(hrt_plan_s* p) {
  const Geometry& g = p->g;
  const double Pt = g.Mt * g.dtheta, Pr = g.Mr * g.drho;
  const double rate = (g.Mt / (2.0 * g.sigma)) / Pt +
                      (g.Mr / (2.0 * g.sigma)) * std::tan(g.beta_k) / Pr;
  const int panels = static_cast<int>(std::ceil(g.beta_k * rate)) + 4;
  std::vector<double> nodes, weights;
  gauss_legendre(20, panels, 0.0, g.beta_k, nodes, weights);
  const int N = static_cast<int>(nodes.size());
  std::vector<double> s1(g.K1), s2(g.K2);
  for (int k = 0; k < g.K1; ++k) s1[k] = 1.0 / b_squared(static_cast<double>(k) / g.Mt);
  for (int k = 0; k < g.K2; ++k) s2[k] = 1.0 / b_squared(static_cast<double>(k) / g.Mr);
  double *dn = nullptr, *dw = nullptr, *E1 = nullptr, *ds1 = nullptr, *ds2 = nullptr;
  double2* E2 = nullptr;
  size_t tmp = 0;
  hrt_status st = HRT_OK;
  auto cleanup = [&]() {
    void* ptrs[] = {dn, dw, E1, E2, ds1, ds2};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
  };
  if ((st = dev_alloc(&dn, N, tmp)) || (st = dev_alloc(&dw, N, tmp)) ||
      (st = dev_alloc(&E1, static_cast<size_t>(g.K1) * N, tmp)) ||
      (st = dev_alloc(&E2, static_cast<size_t>(g.K2) * N, tmp)) ||
      (st = dev_alloc(&ds1, g.K1, tmp)) || (st = dev_alloc(&ds2, g.K2, tmp)) ||
      (st = upload(dn, nodes)) || (st = upload(dw, weights)) ||
      (st = upload(ds1, s1)) || (st = upload(ds2, s2))) {
    cleanup();
    return st;
  }
  const int64_t total = static_cast<int64_t>(g.K1 + g.K2) * N;
  k_zeta_tables<<<static_cast<unsigned>((total + 255) / 256), 256>>>(
      N, g.K1, g.K2, dn, dw, 1.0 / Pt, 1.0 / Pr, E1, E2);
  dim3 grid((g.K2 + 15) / 16, (g.K1 + 15) / 16);
  k_zeta_gemm<<<grid, 256>>>(N, g.K1, g.K2, E1, E2, ds1, ds2,
                             1.0 / (g.dtheta * g.drho), p->K);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  cleanup();
  if (e != hipSuccess) return hip_err(e, "kernel spectrum");
  return HRT_OK;
}

// Live plans: a destroyed or foreign handle is recognised without touching
// the memory it points to.
std::mutex g_plans_mu;
std::set<const hrt_plan_s*> g_plans;

hrt_status check_plan(hrt_plan_t p) {
  if (!p) return set_err(HRT_ERR_INVALID_ARG, "null plan");
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    if (!g_plans.count(p)) return set_err(HRT_ERR_BAD_HANDLE, "not a live plan");
  }
  if (p->magic != kMagic) return set_err(HRT_ERR_BAD_HANDLE, "not a live plan");
  return HRT_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

std::mutex g_attr_mu;

}  // namespace

// Per-call workspace of hrt_forward_noalloc: a fixed array in device memory
// that every GPU the library runs on holds until the process ends.  In host
// code the name `scratch` is only a stand-in for the symbol; its device
// address comes from hipGetSymbolAddress, taken once per device (with that
// device current) when the first plan is created there.
constexpr size_t kStaticScratchBytes = size_t{64} << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch array (the device current).
hrt_status static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_err(HRT_ERR_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return hip_err(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HRT_OK;
}

// Where one forward's workspace (half spectrum, spread partial rows, real
// rows, input maxima) sits in the scratch array: 256-byte aligned pieces.
struct ScratchLayout {
  size_t S = 0, Hp = 0, Cr = 0, absmax = 0, total = 0;
};
ScratchLayout scratch_layout(const Geometry& g, int64_t hp_floats) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  ScratchLayout L;
  L.S = 0;
  L.Hp = L.S + up(static_cast<size_t>(g.K1) * g.Mr * sizeof(float2));
  L.Cr = L.Hp + up(static_cast<size_t>(hp_floats) * sizeof(float));
  L.absmax = L.Cr + up(static_cast<size_t>(g.u1 - g.u0) * g.W * sizeof(float));
  L.total = L.absmax + up(kAbsMaxBlocks * sizeof(float));
  return L;
}
}  // namespace

extern "C" {

const char* hrt_status_string(hrt_status s) {
  switch (s) {
    case HRT_OK: return "ok";
    case HRT_ERR_INVALID_ARG: return "invalid argument";
    case HRT_ERR_GEOMETRY: return "geometry not representable";
    case HRT_ERR_OOM: return "out of device memory";
    case HRT_ERR_HIP: return "HIP error";
    case HRT_ERR_BAD_HANDLE: return "bad plan handle";
    case HRT_ERR_UNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

const char* hrt_last_error(void) { return g_last_error.c_str(); }

hrt_status hrt_plan_describe(const hrt_desc* desc, hrt_info* out) {
  if (!desc || !out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  Geometry g;
  std::string err;
  hrt_status s = build_geometry(*desc, 163840 - kBandStaticLds, g, err);
  if (s != HRT_OK) return set_err(s, err);
  fill_info(g, out);
  return HRT_OK;
}

// A plan for the grids of `desc`, placed in the caller's arrays by `view`
// (null: the whole grids).
static hrt_status create_plan(const hrt_desc* desc, const PartView* view, hrt_plan_t* out) {
  if (!desc || !out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  arm_fail_alloc();
  int dev = 0;
  HRT_HIP(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t prop;
  HRT_HIP(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  int lds_max = 0;
  HRT_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
          "hipDeviceGetAttribute");
  // the band kernels also hold twiddles and reduction slots in static LDS
  const int64_t lds = std::min<int64_t>(lds_max, 163840) - kBandStaticLds;
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  {
    void* sp = nullptr;  // this device's scratch address, taken once
    hrt_status ss = static_scratch(dev, &sp);
    if (ss != HRT_OK) return ss;
  }

  auto* p = new hrt_plan_s();
  p->magic = kMagic;
  p->device = dev;
  std::string err;
  hrt_status s = build_geometry(*desc, lds, p->g, err, view);
  if (s != HRT_OK) {
    delete p;
    return set_err(s, err);
  }
  const Geometry& g = p->g;
  // first kept sample of every trace of the data array (none beyond the
  // plan's traces)
  std::vector<int32_t> jmin_fill(g.jmin);
  jmin_fill.resize(static_cast<size_t>(g.view.nx_fill), g.d.nt);
  if (static_cast<int64_t>(g.col_bytes) > std::min<int64_t>(lds_max, 163840) - 4096) {
    delete p;
    return set_err(HRT_ERR_UNSUPPORTED, "log-radius axis too long for an LDS column");
  }

  size_t total = 0;
  const std::vector<float2> twt = twiddles(g.Mt), twr = twiddles(g.Mr);
  if ((s = dev_alloc(&p->S, static_cast<size_t>(g.K1) * g.Mr, total)) ||
      (s = dev_alloc(&p->K, static_cast<size_t>(g.K1) * g.K2, total)) ||
      (s = dev_alloc(&p->tw_t, twt.size(), total)) ||
      (s = dev_alloc(&p->tw_r, twr.size(), total)) ||
      (s = dev_alloc(&p->jmin, jmin_fill.size(), total)) ||
      (s = dev_alloc(&p->absmax, kAbsMaxBlocks, total)) ||
      (s = dev_alloc(&p->dot, kDotBlocks, total)) ||
      (s = upload(p->tw_t, twt)) || (s = upload(p->tw_r, twr)) ||
      (s = upload(p->jmin, jmin_fill))) {
    free_plan(p);
    delete p;
    return s;
  }
  // placed points, sorted into the band lists
  float cmax_data = 0.0f, cmax_radon = 0.0f;
  std::vector<int32_t> chunk_band_host[4];  // band of every chunk, per list
  {
    PointTables tab;
    if ((s = build_point_tables(g, tab, err)) != HRT_OK) {
      free_plan(p);
      delete p;
      return set_err(s, err);
    }
    // padded for the float32 rounding of the taps
    cmax_data = static_cast<float>(tab.cmax_data * (1.0 + 1e-5));
    cmax_radon = static_cast<float>(tab.cmax_radon * (1.0 + 1e-5));
    const BandLists* lists[4] = {&tab.data_spread, &tab.data_own, &tab.radon_spread,
                                 &tab.radon_own};
    // Radon lists travel as {sample index, log-radius coordinate}: a Radon
    // point's angle coordinate and weight are its slowness's, so they sit
    // once per slowness in q_tab.  The row of an index comes from a
    // multiply-shift division, checked here against the exact one for
    // every entry.
    const uint64_t ld = static_cast<uint64_t>(g.view.radon_ld);
    int lg = 0;
    while ((uint64_t{1} << lg) < ld) ++lg;
    p->rdiv_s = 32 + lg;
    p->rdiv_m = ((uint64_t{1} << p->rdiv_s) + ld - 1) / ld;
    std::vector<uint2> qtab(static_cast<size_t>(std::max(g.d.nq, 1)), make_uint2(0u, 0u));
    std::vector<char> qseen(qtab.size(), 0);
    for (int i = 0; i < 4; ++i) {
      const BandLists& L = *lists[i];
      const bool radon = i == kRadonSpread || i == kRadonOwn;
      chunk_band_host[i] = L.chunk_band;
      p->nchunks[i] = static_cast<int>(L.chunk_band.size());
      std::vector<uint2> compact;
      if (radon) {
        compact.resize(L.e.size());
        for (size_t k = 0; k < L.e.size(); ++k) {
          const PointEntry& E = L.e[k];
          const uint64_t row = E.idx / ld;
          const int l = static_cast<int>(row) - g.view.radon_row0;
          uint32_t wbits;
          std::memcpy(&wbits, &E.w, sizeof wbits);
          if (((static_cast<uint64_t>(E.idx) * p->rdiv_m) >> p->rdiv_s) != row || l < 0 ||
              l >= g.d.nq || (qseen[l] && (qtab[l].x != E.xq || qtab[l].y != wbits))) {
            free_plan(p);
            delete p;
            return set_err(HRT_ERR_GEOMETRY, "Radon point entries disagree with their slowness");
          }
          qtab[l] = make_uint2(E.xq, wbits);
          qseen[l] = 1;
          compact[k] = make_uint2(E.idx, E.yq);
        }
      }
      if ((!radon && (s = dev_alloc(&p->ent[i], std::max<size_t>(1, L.e.size()), total))) ||
          (radon && (s = dev_alloc(&p->ent2[i], std::max<size_t>(1, compact.size()), total))) ||
          (s = dev_alloc(&p->chunk_off[i], L.chunk_off.size(), total)) ||
          (s = dev_alloc(&p->chunk_band[i], L.chunk_band.size(), total)) ||
          (s = dev_alloc(&p->band_chunk[i], L.band_chunk.size(), total)) ||
          (s = upload(p->chunk_off[i], L.chunk_off)) ||
          (s = upload(p->chunk_band[i], L.chunk_band)) ||
          (s = upload(p->band_chunk[i], L.band_chunk)) ||
          (radon && (s = upload(p->ent2[i], compact)))) {
        free_plan(p);
        delete p;
        return s;
      }
      if (i == kDataSpread || i == kRadonSpread) {
        p->hp_floats[i] = L.hp_floats;
        std::vector<int2> cols(L.chunk_band.size());
        for (size_t c = 0; c < cols.size(); ++c)
          cols[c] = make_int2(L.chunk_col[2 * c], L.chunk_col[2 * c + 1]);
        if ((s = dev_alloc(&p->chunk_col[i], cols.size(), total)) ||
            (s = dev_alloc(&p->chunk_hp[i], L.chunk_hp.size(), total)) ||
            (s = upload(p->chunk_col[i], cols)) || (s = upload(p->chunk_hp[i], L.chunk_hp))) {
          free_plan(p);
          delete p;
          return s;
        }
      }
      if (!radon && !L.e.empty()) {
        hipError_t e = hipMemcpy(p->ent[i], L.e.data(), L.e.size() * sizeof(PointEntry),
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) {
          free_plan(p);
          delete p;
          return hip_err(e, "upload point lists");
        }
      }
    }
    if ((s = dev_alloc(&p->q_tab, qtab.size(), total)) || (s = upload(p->q_tab, qtab))) {
      free_plan(p);
      delete p;
      return s;
    }
    // the partial rows of the spread chunks (of whichever direction needs
    // more), and the real rows after the inverse FFT
    const size_t parts = static_cast<size_t>(std::max<int64_t>(
        1, std::max(p->hp_floats[kDataSpread], p->hp_floats[kRadonSpread])));
    if ((s = dev_alloc(&p->Hp, parts, total)) ||
        (s = dev_alloc(&p->Cr, static_cast<size_t>(g.u1 - g.u0) * g.W, total)) ||
        (s = dev_alloc(&p->gmax, static_cast<size_t>(p->nchunks[kRadonOwn]), total))) {
      free_plan(p);
      delete p;
      return s;
    }
  }
  hipError_t e = hipMemset(p->S, 0, static_cast<size_t>(g.K1) * g.Mr * sizeof(float2));
  if (e != hipSuccess) {
    free_plan(p);
    delete p;
    return hip_err(e, "hipMemset");
  }
  if ((s = build_kernel(p)) != HRT_OK) {
    free_plan(p);
    delete p;
    return s;
  }
  {
    // dynamic LDS above the default limit must be granted per kernel; the
    // grant is process-wide, so always the largest the kernel can take
    // (the device limit less its static LDS), whatever this plan needs
    std::lock_guard<std::mutex> lk(g_attr_mu);
    const int64_t cap = std::min<int64_t>(lds_max, 163840);
    const void* fns[] = {reinterpret_cast<const void*>(&k_spread<0, false>),
                         reinterpret_cast<const void*>(&k_spread<1, false>),
                         reinterpret_cast<const void*>(&k_rowfft<0, false>),
                         reinterpret_cast<const void*>(&k_rowfft<1, false>),
                         reinterpret_cast<const void*>(&k_colfft<false, false>),
                         reinterpret_cast<const void*>(&k_colfft<true, false>),
                         reinterpret_cast<const void*>(&k_rowifft<false>),
                         reinterpret_cast<const void*>(&k_gather<0, false>),
                         reinterpret_cast<const void*>(&k_gather<1, false>),
                         reinterpret_cast<const void*>(&k_spread<0, true>),
                         reinterpret_cast<const void*>(&k_spread<1, true>),
                         reinterpret_cast<const void*>(&k_rowfft<0, true>),
                         reinterpret_cast<const void*>(&k_rowfft<1, true>),
                         reinterpret_cast<const void*>(&k_colfft<false, true>),
                         reinterpret_cast<const void*>(&k_colfft<true, true>),
                         reinterpret_cast<const void*>(&k_rowifft<true>),
                         reinterpret_cast<const void*>(&k_gather<0, true>),
                         reinterpret_cast<const void*>(&k_gather<1, true>)};
    const int need[] = {g.spread_bytes, g.spread_bytes, g.row_bytes, g.row_bytes,
                        g.col_bytes,    g.col_bytes,    g.row_bytes, g.gather_bytes,
                        g.gather_bytes, g.spread_bytes, g.spread_bytes, g.row_bytes,
                        g.row_bytes,    g.col_bytes,    g.col_bytes,    g.row_bytes,
                        g.gather_bytes, g.gather_bytes};
    constexpr int nfn = sizeof(fns) / sizeof(fns[0]);
    struct {
      const void* fn;
      size_t bytes;
    } attrs[nfn];
    for (int i = 0; i < nfn; ++i) {
      hipFuncAttributes fa;
      hipError_t r = hipFuncGetAttributes(&fa, fns[i]);
      if (r != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        delete p;
        return hip_err(r, "hipFuncGetAttributes");
      }
      const int64_t room = cap - static_cast<int64_t>(fa.sharedSizeBytes);
      if (static_cast<int64_t>(need[i]) > room) {
        free_plan(p);
        delete p;
        return set_err(HRT_ERR_UNSUPPORTED, "lattice rows exceed the LDS of a workgroup");
      }
      attrs[i] = {fns[i], static_cast<size_t>(room)};
    }
    for (const auto& a : attrs) {
      hipError_t r = hipFuncSetAttribute(a.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(a.bytes));
      if (r != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        delete p;
        return hip_err(r, "hipFuncSetAttribute");
      }
    }
    // the direct adjoint stages a slowness's hyperbola times and panel row
    // in LDS when they fit; otherwise it takes the per-sample search
    {
      const void* fn = reinterpret_cast<const void*>(&k_direct_adj_rows);
      hipFuncAttributes fa;
      hipError_t r = hipFuncGetAttributes(&fa, fn);
      if (r == hipSuccess) {
        const int64_t room = cap - static_cast<int64_t>(fa.sharedSizeBytes);
        r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(room));
        const int64_t need = static_cast<int64_t>(direct_adj_rows_bytes(g.d.nt, g.d.ntau));
        if (r == hipSuccess && need <= room) p->direct_rows_bytes = need;
      }
      if (r != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        delete p;
        return hip_err(r, "direct adjoint attributes");
      }
    }
  }
  DevGeo& G = p->dg;
  G.nt = g.d.nt; G.nx = g.d.nx;
  G.Mt = g.Mt; G.Mr = g.Mr; G.K1 = g.K1; G.K2 = g.K2; G.u0 = g.u0; G.u1 = g.u1;
  G.R = g.R; G.nbands = g.nbands;
  G.row_rows = g.row_rows; G.row_sub_shift = g.row_sub_shift;
  G.xw0 = g.xw0; G.W = g.W; G.x_frac_bits = g.x_frac_bits; G.spread_cols = g.spread_cols;
  G.row_group = g.row_group; G.row_scratch = g.row_scratch;
  G.col_inplace = g.inplace_col ? 1 : 0;
  G.col_batch = g.col_batch;
  G.knorm = static_cast<float>(1.0 / (static_cast<double>(g.Mt) * g.Mr));
  G.cmax_data = cmax_data;
  G.cmax_radon = cmax_radon;
  G.jmin = p->jmin;
  p->ft = to_dev(g.fft_t);
  p->fr = to_dev(g.fft_r);
  G.ntau = g.d.ntau; G.nq = g.d.nq;
  G.absmax_blocks = kAbsMaxBlocks;
  G.data_off = 0; G.radon_off = 0;
  G.data_ld = g.view.data_ld; G.radon_ld = g.view.radon_ld;
  G.j_lo = g.view.j_lo; G.j_hi = g.view.j_hi;
  G.radon_row0 = g.view.radon_row0; G.nx_fill = g.view.nx_fill;
  G.accumulate = 0;
  G.ft = p->ft; G.fr = p->fr;
  G.tw_t = p->tw_t; G.tw_r = p->tw_r;
  G.K = p->K; G.S = p->S; G.Hp = p->Hp; G.Cr = p->Cr; G.absmax = p->absmax;
  G.gmax = nullptr;
  G.q_tab = p->q_tab;
  G.rdiv_m = p->rdiv_m;
  G.rdiv_s = p->rdiv_s;
  for (int i = 0; i < 4; ++i)
    G.lists[i] = DevList{p->ent[i], p->ent2[i], p->chunk_off[i], p->chunk_band[i],
                         p->band_chunk[i], p->chunk_col[i], p->chunk_hp[i], p->nchunks[i]};
  {
    // the descriptor and the single-gather work lists on the device
    std::vector<int2> it[kItemSets];
    for (int b = 0; b < kAbsMaxBlocks; ++b) it[kItAbsmax].push_back(make_int2(0, b));
    for (int c = 0; c < (g.K1 + g.col_batch - 1) / g.col_batch; ++c)
      it[kItCols].push_back(make_int2(0, c));
    for (int c = 0; c < p->nchunks[kDataSpread]; ++c) it[kItSpreadData].push_back(make_int2(0, c));
    for (int c = 0; c < p->nchunks[kRadonSpread]; ++c)
      it[kItSpreadRadon].push_back(make_int2(0, c));
    // bands to XCDs: sorted by their gather chunks, dealt in snake order,
    // so that every XCD gets as many bands (row items) as the others, and
    // about as many gather chunks
    std::vector<int64_t> weight(g.nbands, 0);
    for (int32_t b : chunk_band_host[kDataOwn]) ++weight[b];
    for (int32_t b : chunk_band_host[kRadonOwn]) ++weight[b];
    const std::vector<int> rows = row_items(g);
    std::vector<int> order(g.nbands), xcd(g.nbands);
    for (int b = 0; b < g.nbands; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return weight[a] > weight[b]; });
    for (int k = 0; k < g.nbands; ++k) {
      const int lap = k / kXcds, pos = k % kXcds;
      xcd[order[k]] = (lap & 1) ? kXcds - 1 - pos : pos;
    }
    auto by_xcd = [&](const std::vector<int32_t>& chunk_band) {
      std::vector<std::vector<int2>> q(kXcds);
      for (size_t c = 0; c < chunk_band.size(); ++c)
        q[xcd[chunk_band[c]]].push_back(make_int2(0, static_cast<int>(c)));
      return xcd_order(q);
    };
    p->band_xcd = xcd;
    p->own_chunk_band[0] = chunk_band_host[kRadonOwn];
    p->own_chunk_band[1] = chunk_band_host[kDataOwn];
    it[kItGatherRadon] = by_xcd(chunk_band_host[kRadonOwn]);
    it[kItGatherData] = by_xcd(chunk_band_host[kDataOwn]);
    {
      std::vector<std::vector<int2>> q(kXcds);
      for (int r : rows) q[xcd[r >> g.row_sub_shift]].push_back(make_int2(0, r));
      it[kItBands] = xcd_order(q);
    }
    std::vector<DevGeo> one(1, G);
    if ((s = dev_alloc(&p->geo_dev, 1, total)) || (s = upload(p->geo_dev, one))) {
      free_plan(p);
      delete p;
      return s;
    }
    for (int k = 0; k < kItemSets; ++k) {
      p->nitems[k] = static_cast<int>(it[k].size());
      if ((s = dev_alloc(&p->items[k], std::max<size_t>(1, it[k].size()), total)) ||
          (s = upload(p->items[k], it[k]))) {
        free_plan(p);
        delete p;
        return s;
      }
    }
  }

  DirectGeo& D = p->dd;
  D.nt = g.d.nt; D.nx = g.d.nx; D.ntau = g.d.ntau; D.nq = g.d.nq;
  D.dt = static_cast<float>(g.d.dt); D.inv_dt = static_cast<float>(1.0 / g.d.dt);
  D.x0 = static_cast<float>(g.d.x0); D.dx = static_cast<float>(g.d.dx);
  D.tau0 = static_cast<float>(g.d.tau0); D.dtau = static_cast<float>(g.d.dtau);
  D.q0 = static_cast<float>(g.d.q0); D.dq = static_cast<float>(g.d.dq);

  fill_info(g, &p->info);
  p->info.workspace_bytes = static_cast<int64_t>(total);
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_plans.insert(p);
  }
  *out = p;
  return HRT_OK;
}

hrt_status hrt_plan_create(const hrt_desc* desc, hrt_plan_t* out) {
  return create_plan(desc, nullptr, out);
}

namespace {
// Records the profiling events around one kernel launch (no-op unless a
// profile is active and has room).
struct StageTimer {
  hrt_plan_s* p;
  hipStream_t st;
  int slot = -1;
  StageTimer(hrt_plan_s* plan, hipStream_t s, int stage) : p(plan), st(s) {
    if (p->prof_used < static_cast<int>(p->prof_stage.size())) {
      slot = p->prof_used++;
      p->prof_stage[slot] = stage;
      (void)hipEventRecord(p->prof_ev[2 * slot], st);
    }
  }
  ~StageTimer() {
    if (slot >= 0) (void)hipEventRecord(p->prof_ev[2 * slot + 1], st);
  }
};
}  // namespace

// The six launches of one direction on stream `st` (arguments checked by
// the caller; the device current).  With `accumulate` the gather adds into
// `out` (the parts of a split after the first).  With `chained` the two
// directions run as R^T R: the forward's gather also stores the partial
// maxima of its output, and the adjoint that takes that output as its
// input uses them instead of launching its own input maximum (five
// launches).
static void run_chain(hrt_plan_t p, const float* in, float* out, hipStream_t st, bool adjoint,
                      bool accumulate, bool chained = false, const DevGeo* ws = nullptr) {
  const Geometry& g = p->g;
  const size_t sb = g.spread_bytes, rb = g.row_bytes, cb = g.col_bytes, gb = g.gather_bytes;
  DevGeo G = ws ? *ws : p->dg;
  G.accumulate = accumulate ? 1 : 0;
  if (chained && !adjoint) G.gmax = p->gmax;
  if (chained && adjoint) {
    G.absmax = p->gmax;
    G.absmax_blocks = p->nchunks[kRadonOwn];
  }
  const int* ni = p->nitems;
  int2* const* it = p->items;
  const int t0 = adjoint ? 6 : 0;  // profile slots
  if (!adjoint) {
    { StageTimer t(p, st, t0);
      k_absmax<0, false><<<ni[kItAbsmax], 256, 0, st>>>(G, nullptr, nullptr, in); }
    { StageTimer t(p, st, t0 + 1);
      k_spread<0, false><<<ni[kItSpreadData], kNtBand, sb, st>>>(G, nullptr, it[kItSpreadData], in); }
    { StageTimer t(p, st, t0 + 2);
      k_rowfft<0, false><<<ni[kItBands], kNtBand, rb, st>>>(G, nullptr, it[kItBands]); }
    { StageTimer t(p, st, t0 + 3);
      k_colfft<false, false><<<ni[kItCols], kNtCol, cb, st>>>(G, nullptr, nullptr); }
    { StageTimer t(p, st, t0 + 4);
      k_rowifft<false><<<ni[kItBands], kNtBand, rb, st>>>(G, nullptr, it[kItBands]); }
    { StageTimer t(p, st, t0 + 5);
      k_gather<0, false><<<ni[kItGatherRadon], kNtBand, gb, st>>>(G, nullptr, it[kItGatherRadon], out); }
  } else {
    if (!chained) {
      StageTimer t(p, st, t0);
      k_absmax<1, false><<<ni[kItAbsmax], 256, 0, st>>>(G, nullptr, nullptr, in);
    }
    { StageTimer t(p, st, t0 + 1);
      k_spread<1, false><<<ni[kItSpreadRadon], kNtBand, sb, st>>>(G, nullptr, it[kItSpreadRadon], in); }
    { StageTimer t(p, st, t0 + 2);
      k_rowfft<1, false><<<ni[kItBands], kNtBand, rb, st>>>(G, nullptr, it[kItBands]); }
    { StageTimer t(p, st, t0 + 3);
      k_colfft<true, false><<<ni[kItCols], kNtCol, cb, st>>>(G, nullptr, nullptr); }
    { StageTimer t(p, st, t0 + 4);
      k_rowifft<false><<<ni[kItBands], kNtBand, rb, st>>>(G, nullptr, it[kItBands]); }
    { StageTimer t(p, st, t0 + 5);
      k_gather<1, false><<<ni[kItGatherData], kNtBand, gb, st>>>(G, nullptr, it[kItGatherData], out); }
  }
}

// `user_call`: the public forward / adjoint, which honour the plan's
// HRT_ACCUMULATE_OUTPUT (internal chains always overwrite).
static hrt_status launch_chain(hrt_plan_t p, const float* in, float* out, void* stream,
                               bool adjoint, bool user_call = false) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  const bool accumulate = user_call && (p->g.d.flags & HRT_ACCUMULATE_OUTPUT);
  if (!in || !out) return set_err(HRT_ERR_INVALID_ARG, "null array");
  const size_t n_data = static_cast<size_t>(p->g.d.nx) * p->g.d.nt;
  const size_t n_radon = static_cast<size_t>(p->g.d.nq) * p->g.d.ntau;
  const size_t n_in = adjoint ? n_radon : n_data;
  const size_t n_out = adjoint ? n_data : n_radon;
  const char* ib = reinterpret_cast<const char*>(in);
  const char* ob = reinterpret_cast<const char*>(out);
  if (ib < ob + n_out * sizeof(float) && ob < ib + n_in * sizeof(float))
    return set_err(HRT_ERR_INVALID_ARG, "input and output overlap");
  DeviceGuard guard(p->device);
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  run_chain(p, in, out, reinterpret_cast<hipStream_t>(stream), adjoint, accumulate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, adjoint ? "adjoint launch" : "forward launch");
  return HRT_OK;
}

// (only for a plan that check_plan has accepted)
static bool accumulates(hrt_plan_t p) { return p->g.d.flags & HRT_ACCUMULATE_OUTPUT; }

hrt_status hrt_forward(hrt_plan_t p, const float* f, float* g, void* stream) {
  return launch_chain(p, f, g, stream, false, true);
}

hrt_status hrt_adjoint(hrt_plan_t p, const float* g, float* f, void* stream) {
  return launch_chain(p, g, f, stream, true, true);
}

hrt_status hrt_forward_noalloc(hrt_plan_t p, const float* f, float* g, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!f || !g) return set_err(HRT_ERR_INVALID_ARG, "null array");
  const size_t nd = static_cast<size_t>(p->g.d.nx) * p->g.d.nt * sizeof(float);
  const size_t nr = static_cast<size_t>(p->g.d.nq) * p->g.d.ntau * sizeof(float);
  const char* fb = reinterpret_cast<const char*>(f);
  const char* gb = reinterpret_cast<const char*>(g);
  if (fb < gb + nr && gb < fb + nd) return set_err(HRT_ERR_INVALID_ARG, "input and output overlap");
  const ScratchLayout L = scratch_layout(p->g, p->hp_floats[kDataSpread]);
  if (L.total > kStaticScratchBytes)
    return set_err(HRT_ERR_UNSUPPORTED,
                   "the plan's forward workspace (" + std::to_string(L.total) +
                       " bytes) exceeds the static workspace of hrt_forward_noalloc (" +
                       std::to_string(kStaticScratchBytes) + " bytes)");
  DeviceGuard guard(p->device);
  void* base = nullptr;
  if ((s = static_scratch(p->device, &base)) != HRT_OK) return s;
  unsigned char* b = static_cast<unsigned char*>(base);
  DevGeo G = p->dg;
  G.S = reinterpret_cast<float2*>(b + L.S);
  G.Hp = reinterpret_cast<float*>(b + L.Hp);
  G.Cr = reinterpret_cast<float*>(b + L.Cr);
  G.absmax = reinterpret_cast<float*>(b + L.absmax);
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  run_chain(p, f, g, reinterpret_cast<hipStream_t>(stream), false, accumulates(p), false, &G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "forward launch");
  return HRT_OK;
}

namespace {
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

int vec_blocks(int64_t n) {
  return static_cast<int>(std::min<int64_t>(2048, std::max<int64_t>(1, (n + kVecThreads - 1) / kVecThreads)));
}
}  // namespace

hrt_status hrt_ista_iterate(hrt_plan_t p, const float* f, const float* mask, float* g,
                            float* work_data, float* work_radon, int32_t iters, float c2,
                            float mu, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!f || !g || !work_data || !work_radon) return set_err(HRT_ERR_INVALID_ARG, "null array");
  if (iters < 0 || !(c2 > 0.0f) || !(mu >= 0.0f))
    return set_err(HRT_ERR_INVALID_ARG, "need iters >= 0, c2 > 0, mu >= 0");
  const size_t nd = static_cast<size_t>(p->g.d.nx) * p->g.d.nt * sizeof(float);
  const size_t nr = static_cast<size_t>(p->g.d.nq) * p->g.d.ntau * sizeof(float);
  if (overlaps(g, nr, work_radon, nr) || overlaps(g, nr, work_data, nd) ||
      overlaps(g, nr, f, nd) || overlaps(work_data, nd, work_radon, nr) ||
      overlaps(work_data, nd, f, nd) || overlaps(work_radon, nr, f, nd) ||
      (mask && (overlaps(mask, nd, work_data, nd) || overlaps(mask, nd, g, nr) ||
                overlaps(mask, nd, work_radon, nr))))
    return set_err(HRT_ERR_INVALID_ARG, "arrays overlap");
  DeviceGuard guard(p->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t n_data = static_cast<int64_t>(p->g.d.nx) * p->g.d.nt;
  const int64_t n_radon = static_cast<int64_t>(p->g.d.nq) * p->g.d.ntau;
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  for (int it = 0; it < iters; ++it) {
    // the arrays were checked above; every launch of the iteration,
    // the element-wise ones included, is checked after it
    run_chain(p, g, work_data, st, true, false);
    k_residual<<<vec_blocks(n_data), kVecThreads, 0, st>>>(f, mask, work_data, n_data);
    run_chain(p, work_data, work_radon, st, false, false);
    k_soft_update<<<vec_blocks(n_radon), kVecThreads, 0, st>>>(g, work_radon, c2,
                                                               0.5f * c2 * mu, n_radon);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "ista launch");
  }
  return HRT_OK;
}

struct hrt_graph_s {
  uint64_t magic;
  int device;
  hipGraphExec_t exec;
  void* owned;  // device memory the graph's kernels read (freed with it)
};

// Captures what `enqueue` launches on a private stream of `device` into an
// executable graph; the graph takes ownership of `owned` (also on failure).
extern "C++" template <class EnqueueF>
static hrt_status capture_graph(int device, EnqueueF enqueue, void* owned, hrt_graph_t* out) {
  DeviceGuard guard(device);
  auto drop = [&](hrt_status s) {
    if (owned) (void)hipFree(owned);
    return s;
  };
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return drop(hip_err(e, "hipStreamCreate"));
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return drop(hip_err(e, "hipStreamBeginCapture"));
  }
  hrt_status s = enqueue(cs);
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (s != HRT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return drop(s);
  }
  if (e != hipSuccess) return drop(hip_err(e, "hipStreamEndCapture"));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return drop(hip_err(e, "hipGraphInstantiate"));
  *out = new hrt_graph_s{kGraphMagic, device, exec, owned};
  return HRT_OK;
}

hrt_status hrt_ista_graph_create(hrt_plan_t p, const float* f, const float* mask, float* g,
                                 float* work_data, float* work_radon, int32_t iters, float c2,
                                 float mu, hrt_graph_t* out) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (!p->prof_ev.empty()) return set_err(HRT_ERR_INVALID_ARG, "profiling is active");
  return capture_graph(
      p->device,
      [&](hipStream_t cs) {
        return hrt_ista_iterate(p, f, mask, g, work_data, work_radon, iters, c2, mu, cs);
      },
      nullptr, out);
}

hrt_status hrt_graph_launch(hrt_graph_t gr, void* stream) {
  if (!gr || gr->magic != kGraphMagic) return set_err(HRT_ERR_BAD_HANDLE, "bad graph handle");
  DeviceGuard guard(gr->device);
  HRT_HIP(hipGraphLaunch(gr->exec, reinterpret_cast<hipStream_t>(stream)), "hipGraphLaunch");
  return HRT_OK;
}

void hrt_graph_destroy(hrt_graph_t gr) {
  if (!gr || gr->magic != kGraphMagic) return;
  DeviceGuard guard(gr->device);
  (void)hipDeviceSynchronize();
  (void)hipGraphExecDestroy(gr->exec);
  if (gr->owned) (void)hipFree(gr->owned);
  gr->magic = 0;
  delete gr;
}

hrt_status hrt_normal(hrt_plan_t p, const float* f, float* g, float* fa, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!f || !g || !fa) return set_err(HRT_ERR_INVALID_ARG, "null array");
  const size_t nd = static_cast<size_t>(p->g.d.nx) * p->g.d.nt * sizeof(float);
  const size_t nr = static_cast<size_t>(p->g.d.nq) * p->g.d.ntau * sizeof(float);
  if (overlaps(f, nd, g, nr) || overlaps(g, nr, fa, nd))
    return set_err(HRT_ERR_INVALID_ARG, "input and output overlap");
  if (accumulates(p))
    return set_err(HRT_ERR_INVALID_ARG, "hrt_normal overwrites its outputs: not with "
                                        "HRT_ACCUMULATE_OUTPUT");
  DeviceGuard guard(p->device);
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  run_chain(p, f, g, st, false, false, true);
  run_chain(p, g, fa, st, true, false, true);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "normal launch");
  return HRT_OK;
}

hrt_status hrt_opnorm2(hrt_plan_t p, int32_t iters, uint64_t seed, float* work_data,
                       float* work_data2, float* work_radon, double* out, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!work_data || !work_data2 || !work_radon || !out || iters < 1)
    return set_err(HRT_ERR_INVALID_ARG, "null array or iters < 1");
  const int64_t n_data = static_cast<int64_t>(p->g.d.nx) * p->g.d.nt;
  const size_t nd = static_cast<size_t>(n_data) * sizeof(float);
  const size_t nr = static_cast<size_t>(p->g.d.nq) * p->g.d.ntau * sizeof(float);
  if (overlaps(work_data, nd, work_data2, nd) || overlaps(work_data, nd, work_radon, nr) ||
      overlaps(work_data2, nd, work_radon, nr))
    return set_err(HRT_ERR_INVALID_ARG, "arrays overlap");
  DeviceGuard guard(p->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // seeded start vector (splitmix64 -> uniform in [-1, 1))
  std::vector<float> v0(static_cast<size_t>(n_data));
  uint64_t z = seed;
  for (float& x : v0) {
    z += 0x9e3779b97f4a7c15ull;
    uint64_t t = z;
    t = (t ^ (t >> 30)) * 0xbf58476d1ce4e5b9ull;
    t = (t ^ (t >> 27)) * 0x94d049bb133111ebull;
    t ^= t >> 31;
    x = static_cast<float>(static_cast<double>(t >> 11) * 0x1.0p-52 - 1.0);
  }
  HRT_HIP(hipMemcpyAsync(work_data, v0.data(), nd, hipMemcpyHostToDevice, st), "upload start");
  std::vector<double> part(kDotBlocks);
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  auto dot = [&](const float* a, const float* b, double& r) -> hrt_status {
    k_dot64<<<kDotBlocks, kVecThreads, 0, st>>>(a, b, n_data, p->dot);
    HRT_HIP(hipGetLastError(), "power iteration dot launch");
    HRT_HIP(hipMemcpyAsync(part.data(), p->dot, kDotBlocks * sizeof(double),
                           hipMemcpyDeviceToHost, st),
            "read partial sums");
    HRT_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    r = 0.0;
    for (double x : part) r += x;
    return HRT_OK;
  };
  double vv = 0.0, lambda = 0.0;
  if ((s = dot(work_data, work_data, vv)) != HRT_OK) return s;
  k_scale<<<vec_blocks(n_data), kVecThreads, 0, st>>>(work_data, work_data, 1.0 / std::sqrt(vv),
                                                       n_data);
  HRT_HIP(hipGetLastError(), "power iteration scale launch");
  for (int it = 0; it < iters; ++it) {
    // w = R* R v, lambda = <v, w> for |v| = 1, then v = w / |w|
    if ((s = hrt_normal(p, work_data, work_radon, work_data2, stream)) != HRT_OK) return s;
    double vw = 0.0, ww = 0.0;
    if ((s = dot(work_data, work_data2, vw)) != HRT_OK) return s;
    if ((s = dot(work_data2, work_data2, ww)) != HRT_OK) return s;
    lambda = vw;
    if (!(ww > 0.0)) break;
    k_scale<<<vec_blocks(n_data), kVecThreads, 0, st>>>(work_data, work_data2,
                                                         1.0 / std::sqrt(ww), n_data);
    HRT_HIP(hipGetLastError(), "power iteration scale launch");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "power iteration");
  *out = lambda;
  return HRT_OK;
}

hrt_status hrt_demultiple(hrt_plan_t p, const float* f, const float* g, double qb0,
                          double qb_slope, float* out, float* work_radon, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!f || !g || !out || !work_radon) return set_err(HRT_ERR_INVALID_ARG, "null array");
  const hrt_desc& d = p->g.d;
  const int64_t n_data = static_cast<int64_t>(d.nx) * d.nt;
  const int64_t n_radon = static_cast<int64_t>(d.nq) * d.ntau;
  const size_t nd = n_data * sizeof(float), nr = n_radon * sizeof(float);
  if (overlaps(out, nd, f, nd) || overlaps(out, nd, g, nr) || overlaps(out, nd, work_radon, nr) ||
      overlaps(work_radon, nr, g, nr) || overlaps(work_radon, nr, f, nd))
    return set_err(HRT_ERR_INVALID_ARG, "arrays overlap");
  DeviceGuard guard(p->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  k_mute_multiples<<<vec_blocks(n_radon), kVecThreads, 0, st>>>(
      g, work_radon, d.ntau, d.nq, d.tau0, d.dtau, d.q0, d.dq, qb0, qb_slope);
  HRT_HIP(hipGetLastError(), "demultiple mute launch");
  if ((s = launch_chain(p, work_radon, out, stream, true)) != HRT_OK) return s;
  k_residual<<<vec_blocks(n_data), kVecThreads, 0, st>>>(f, nullptr, out, n_data);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "demultiple launch");
  return HRT_OK;
}

hrt_status hrt_direct_forward(hrt_plan_t p, const float* f, float* g, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!f || !g) return set_err(HRT_ERR_INVALID_ARG, "null array");
  DeviceGuard guard(p->device);
  const DirectGeo& D = p->dd;
  dim3 grid((D.ntau + 255) / 256, D.nq);
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  k_direct_fwd<<<grid, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(D, f, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "direct forward launch");
  return HRT_OK;
}

hrt_status hrt_direct_adjoint(hrt_plan_t p, const float* g, float* f, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!f || !g) return set_err(HRT_ERR_INVALID_ARG, "null array");
  DeviceGuard guard(p->device);
  const DirectGeo& D = p->dd;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  if (p->direct_rows_bytes > 0) {
    k_direct_adj_rows<<<D.nx, kDirectThreads, static_cast<size_t>(p->direct_rows_bytes), st>>>(
        D, g, f);
  } else {
    dim3 grid((D.nt + 255) / 256, D.nx);
    k_direct_adj<<<grid, 256, 0, st>>>(D, g, f);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "direct adjoint launch");
  return HRT_OK;
}

// ------------------------------------------------------------ batches --

struct hrt_batch_s {
  uint64_t magic;
  int device;
  bool owns_plans = true;
  std::vector<hrt_plan_t> plans;
  std::vector<int64_t> data_off, radon_off;  // n + 1 each, in floats
  DevGeo* geos = nullptr;                    // one descriptor per gather
  int64_t* radon_off_dev = nullptr;          // radon_off on the device
  float2* ista_par = nullptr;                // (c^2, c^2 mu / 2) per gather
  std::vector<float2> ista_par_host;         // host source of the last upload
  int2* items[kItemSets] = {};
  int nitems[kItemSets] = {};
  int spread_bytes = 0, row_bytes = 0, col_bytes = 0, gather_bytes = 0;
};

namespace {
void free_batch(hrt_batch_s* b) {
  if (b->geos) (void)hipFree(b->geos);
  if (b->radon_off_dev) (void)hipFree(b->radon_off_dev);
  if (b->ista_par) (void)hipFree(b->ista_par);
  for (int2* q : b->items)
    if (q) (void)hipFree(q);
  if (b->owns_plans)
    for (hrt_plan_t q : b->plans) hrt_plan_destroy(q);
  b->magic = 0;
  delete b;
}

// Device tables of a batch whose plans, offsets (data_off, radon_off) and
// LDS sizes are set: one descriptor per plan (gathers with `accumulate[i]`
// add into their output) and the work items, largest gathers first so that
// the small ones fill in at the end of each launch.
hrt_status build_batch_tables(hrt_batch_s* b, const std::vector<int>& accumulate) {
  const int n = static_cast<int>(b->plans.size());
  std::vector<DevGeo> geos(n);
  std::vector<int> order(n);
  std::vector<int64_t> work(n);
  for (int i = 0; i < n; ++i) {
    const hrt_plan_s* pl = b->plans[i];
    geos[i] = pl->dg;
    geos[i].data_off = b->data_off[i];
    geos[i].radon_off = b->radon_off[i];
    geos[i].absmax_blocks = kAbsMaxBlocksBatch;
    geos[i].accumulate = accumulate[i];
    work[i] = static_cast<int64_t>(pl->g.d.nx) * pl->g.d.nt;
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  std::vector<int2> it[kItemSets];
  // row FFT and gather items XCD-aware as for a single plan, each gather's
  // band-to-XCD map rotated by the bands before it
  std::vector<std::vector<int2>> qb(kXcds), qr(kXcds), qd(kXcds);
  int rot = 0;
  for (int i : order) {
    const hrt_plan_s* pl = b->plans[i];
    auto X = [&](int band) { return (pl->band_xcd[band] + rot) % kXcds; };
    for (int k = 0; k < kAbsMaxBlocksBatch; ++k) it[kItAbsmax].push_back(make_int2(i, k));
    for (int k = 0; k < pl->nchunks[kDataSpread]; ++k) it[kItSpreadData].push_back(make_int2(i, k));
    for (int k = 0; k < pl->nchunks[kRadonSpread]; ++k)
      it[kItSpreadRadon].push_back(make_int2(i, k));
    for (int r : row_items(pl->g)) qb[X(r >> pl->g.row_sub_shift)].push_back(make_int2(i, r));
    for (int k = 0; k < pl->nitems[kItCols]; ++k) it[kItCols].push_back(make_int2(i, k));
    for (int k = 0; k < pl->nchunks[kRadonOwn]; ++k)
      qr[X(pl->own_chunk_band[0][k])].push_back(make_int2(i, k));
    for (int k = 0; k < pl->nchunks[kDataOwn]; ++k)
      qd[X(pl->own_chunk_band[1][k])].push_back(make_int2(i, k));
    rot = (rot + pl->g.nbands) % kXcds;
  }
  it[kItBands] = xcd_order(qb);
  it[kItGatherRadon] = xcd_order(qr);
  it[kItGatherData] = xcd_order(qd);
  for (const hrt_plan_s* pl : b->plans) {
    b->spread_bytes = std::max(b->spread_bytes, pl->g.spread_bytes);
    b->row_bytes = std::max(b->row_bytes, pl->g.row_bytes);
    b->col_bytes = std::max(b->col_bytes, pl->g.col_bytes);
    b->gather_bytes = std::max(b->gather_bytes, pl->g.gather_bytes);
  }
  DeviceGuard guard(b->device);
  size_t total = 0;
  hrt_status s = HRT_OK;
  if ((s = dev_alloc(&b->geos, n, total)) || (s = upload(b->geos, geos))) return s;
  for (int k = 0; k < kItemSets; ++k) {
    b->nitems[k] = static_cast<int>(it[k].size());
    if ((s = dev_alloc(&b->items[k], std::max<size_t>(1, it[k].size()), total)) ||
        (s = upload(b->items[k], it[k])))
      return s;
  }
  return HRT_OK;
}

hrt_status check_batch(hrt_batch_t b) {
  if (!b || b->magic != kBatchMagic) return set_err(HRT_ERR_BAD_HANDLE, "bad batch handle");
  return HRT_OK;
}
}  // namespace

hrt_status hrt_batch_create(const hrt_desc* descs, int32_t n, hrt_batch_t* out) {
  if (!descs || !out || n < 1) return set_err(HRT_ERR_INVALID_ARG, "null argument or n < 1");
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (descs[i].flags & HRT_ACCUMULATE_OUTPUT)
      return set_err(HRT_ERR_INVALID_ARG, "batches do not take HRT_ACCUMULATE_OUTPUT");
  auto* b = new hrt_batch_s();
  b->magic = kBatchMagic;
  HRT_HIP(hipGetDevice(&b->device), "hipGetDevice");
  b->data_off.assign(n + 1, 0);
  b->radon_off.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    hrt_plan_t pl = nullptr;
    hrt_status s = hrt_plan_create(&descs[i], &pl);
    if (s != HRT_OK) {
      const std::string e = g_last_error;
      free_batch(b);
      return set_err(s, "gather " + std::to_string(i) + ": " + e);
    }
    b->plans.push_back(pl);
    const Geometry& g = pl->g;
    b->data_off[i + 1] = b->data_off[i] + static_cast<int64_t>(g.d.nx) * g.d.nt;
    b->radon_off[i + 1] = b->radon_off[i] + static_cast<int64_t>(g.d.nq) * g.d.ntau;
  }
  hrt_status s = build_batch_tables(b, std::vector<int>(n, 0));
  if (s == HRT_OK) {
    DeviceGuard guard(b->device);
    size_t total = 0;
    if ((s = dev_alloc(&b->radon_off_dev, b->radon_off.size(), total)) == HRT_OK &&
        (s = upload(b->radon_off_dev, b->radon_off)) == HRT_OK)
      s = dev_alloc(&b->ista_par, static_cast<size_t>(n), total);
  }
  if (s != HRT_OK) {
    free_batch(b);
    return s;
  }
  *out = b;
  return HRT_OK;
}

hrt_status hrt_batch_offsets(hrt_batch_t b, int64_t* data_off, int64_t* radon_off) {
  hrt_status s = check_batch(b);
  if (s != HRT_OK) return s;
  for (size_t i = 0; i < b->data_off.size(); ++i) {
    if (data_off) data_off[i] = b->data_off[i];
    if (radon_off) radon_off[i] = b->radon_off[i];
  }
  return HRT_OK;
}

hrt_status hrt_batch_plan(hrt_batch_t b, int32_t i, hrt_plan_t* out) {
  hrt_status s = check_batch(b);
  if (s != HRT_OK) return s;
  if (!out || i < 0 || i >= static_cast<int32_t>(b->plans.size()))
    return set_err(HRT_ERR_INVALID_ARG, "gather index out of range");
  *out = b->plans[i];
  return HRT_OK;
}

// The six batched launches of one direction (arguments checked by the
// caller; the device current).
static void run_batch(hrt_batch_t b, const float* in, float* out, hipStream_t st, bool adjoint) {
  const DevGeo none{};
  const DevGeo* geo = b->geos;
  int2* const* it = b->items;
  const int* ni = b->nitems;
  const size_t sb = b->spread_bytes, rb = b->row_bytes, cb = b->col_bytes, gb = b->gather_bytes;
  if (!adjoint) {
    k_absmax<0, true><<<ni[kItAbsmax], 256, 0, st>>>(none, geo, it[kItAbsmax], in);
    k_spread<0, true><<<ni[kItSpreadData], kNtBand, sb, st>>>(none, geo, it[kItSpreadData], in);
    k_rowfft<0, true><<<ni[kItBands], kNtBand, rb, st>>>(none, geo, it[kItBands]);
    k_colfft<false, true><<<ni[kItCols], kNtCol, cb, st>>>(none, geo, it[kItCols]);
    k_rowifft<true><<<ni[kItBands], kNtBand, rb, st>>>(none, geo, it[kItBands]);
    k_gather<0, true><<<ni[kItGatherRadon], kNtBand, gb, st>>>(none, geo, it[kItGatherRadon],
                                                               out);
  } else {
    k_absmax<1, true><<<ni[kItAbsmax], 256, 0, st>>>(none, geo, it[kItAbsmax], in);
    k_spread<1, true><<<ni[kItSpreadRadon], kNtBand, sb, st>>>(none, geo, it[kItSpreadRadon],
                                                               in);
    k_rowfft<1, true><<<ni[kItBands], kNtBand, rb, st>>>(none, geo, it[kItBands]);
    k_colfft<true, true><<<ni[kItCols], kNtCol, cb, st>>>(none, geo, it[kItCols]);
    k_rowifft<true><<<ni[kItBands], kNtBand, rb, st>>>(none, geo, it[kItBands]);
    k_gather<1, true><<<ni[kItGatherData], kNtBand, gb, st>>>(none, geo, it[kItGatherData],
                                                              out);
  }
}

static hrt_status batch_chain(hrt_batch_t b, const float* in, float* out, void* stream,
                              bool adjoint) {
  hrt_status s = check_batch(b);
  if (s != HRT_OK) return s;
  if (!in || !out) return set_err(HRT_ERR_INVALID_ARG, "null array");
  const size_t nd = static_cast<size_t>(b->data_off.back()) * sizeof(float);
  const size_t nr = static_cast<size_t>(b->radon_off.back()) * sizeof(float);
  if (overlaps(in, adjoint ? nr : nd, out, adjoint ? nd : nr))
    return set_err(HRT_ERR_INVALID_ARG, "input and output overlap");
  DeviceGuard guard(b->device);
  (void)hipGetLastError();
  run_batch(b, in, out, reinterpret_cast<hipStream_t>(stream), adjoint);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, adjoint ? "batch adjoint launch" : "batch forward launch");
  return HRT_OK;
}

hrt_status hrt_batch_forward(hrt_batch_t b, const float* f, float* g, void* stream) {
  return batch_chain(b, f, g, stream, false);
}

hrt_status hrt_batch_adjoint(hrt_batch_t b, const float* g, float* f, void* stream) {
  return batch_chain(b, g, f, stream, true);
}

// Soft-thresholding iterations over a batch (arguments checked by the
// caller): per iteration the batched adjoint, the residual over all packed
// samples, the batched forward, the per-gather update with par[b].
static hrt_status batch_ista_enqueue(hrt_batch_t b, const float* f, const float* mask, float* g,
                                     float* work_data, float* work_radon, int32_t iters,
                                     const float2* par, hipStream_t st) {
  const int64_t n_data = b->data_off.back();
  const int n = static_cast<int>(b->plans.size());
  for (int it = 0; it < iters; ++it) {
    run_batch(b, g, work_data, st, true);
    k_residual<<<vec_blocks(n_data), kVecThreads, 0, st>>>(f, mask, work_data, n_data);
    run_batch(b, work_data, work_radon, st, false);
    k_soft_update_batch<<<vec_blocks(b->radon_off.back()), kVecThreads, 0, st>>>(
        g, work_radon, par, b->radon_off_dev, n);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "batch ista launch");
  return HRT_OK;
}

// Validates the batch ISTA arguments and packs (c2_i, c2_i mu_i / 2).
static hrt_status batch_ista_args(hrt_batch_t b, const float* f, const float* mask, float* g,
                                  float* work_data, float* work_radon, int32_t iters,
                                  const float* c2, const float* mu, std::vector<float2>& par) {
  hrt_status s = check_batch(b);
  if (s != HRT_OK) return s;
  if (!f || !g || !work_data || !work_radon || !c2 || !mu)
    return set_err(HRT_ERR_INVALID_ARG, "null array");
  if (iters < 0) return set_err(HRT_ERR_INVALID_ARG, "need iters >= 0");
  const size_t n = b->plans.size();
  par.resize(n);
  for (size_t i = 0; i < n; ++i) {
    if (!(c2[i] > 0.0f) || !(mu[i] >= 0.0f))
      return set_err(HRT_ERR_INVALID_ARG, "need c2 > 0 and mu >= 0 for every gather");
    par[i] = make_float2(c2[i], 0.5f * c2[i] * mu[i]);
  }
  const size_t nd = static_cast<size_t>(b->data_off.back()) * sizeof(float);
  const size_t nr = static_cast<size_t>(b->radon_off.back()) * sizeof(float);
  if (overlaps(g, nr, work_radon, nr) || overlaps(g, nr, work_data, nd) ||
      overlaps(g, nr, f, nd) || overlaps(work_data, nd, work_radon, nr) ||
      overlaps(work_data, nd, f, nd) || overlaps(work_radon, nr, f, nd) ||
      (mask && (overlaps(mask, nd, work_data, nd) || overlaps(mask, nd, g, nr) ||
                overlaps(mask, nd, work_radon, nr))))
    return set_err(HRT_ERR_INVALID_ARG, "arrays overlap");
  return HRT_OK;
}

hrt_status hrt_batch_ista_iterate(hrt_batch_t b, const float* f, const float* mask, float* g,
                                  float* work_data, float* work_radon, int32_t iters,
                                  const float* c2, const float* mu, void* stream) {
  std::vector<float2> par;
  hrt_status s = batch_ista_args(b, f, mask, g, work_data, work_radon, iters, c2, mu, par);
  if (s != HRT_OK) return s;
  DeviceGuard guard(b->device);
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the host source outlives the call, whenever the runtime performs the copy
  b->ista_par_host = std::move(par);
  HRT_HIP(hipMemcpyAsync(b->ista_par, b->ista_par_host.data(),
                         b->ista_par_host.size() * sizeof(float2), hipMemcpyHostToDevice, st),
          "upload ista parameters");
  return batch_ista_enqueue(b, f, mask, g, work_data, work_radon, iters, b->ista_par, st);
}

hrt_status hrt_batch_ista_graph_create(hrt_batch_t b, const float* f, const float* mask,
                                       float* g, float* work_data, float* work_radon,
                                       int32_t iters, const float* c2, const float* mu,
                                       hrt_graph_t* out) {
  if (!out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  std::vector<float2> par;
  hrt_status s = batch_ista_args(b, f, mask, g, work_data, work_radon, iters, c2, mu, par);
  if (s != HRT_OK) return s;
  DeviceGuard guard(b->device);
  // the graph's own copy of the parameters, so later calls cannot change it
  float2* gpar = nullptr;
  size_t total = 0;
  if ((s = dev_alloc(&gpar, par.size(), total)) != HRT_OK) return s;
  hipError_t e = hipMemcpy(gpar, par.data(), par.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(gpar);
    return hip_err(e, "upload ista parameters");
  }
  return capture_graph(
      b->device,
      [&](hipStream_t cs) {
        return batch_ista_enqueue(b, f, mask, g, work_data, work_radon, iters, gpar, cs);
      },
      gpar, out);
}

void hrt_batch_destroy(hrt_batch_t b) {
  if (!b || b->magic != kBatchMagic) return;
  DeviceGuard guard(b->device);
  (void)hipDeviceSynchronize();
  free_batch(b);
}

// ------------------------------------------------------------- splits --

struct hrt_split_s {
  uint64_t magic;
  int device;
  hrt_desc d;
  int n_t = 0, n_q = 0;
  std::vector<hrt_plan_t> parts;  // part iq * n_t + it
  // the parts grouped into phases run one after another, each phase batched
  // (one launch per kernel for all its parts); within a phase the parts'
  // outputs are disjoint, the first phase stores and the others add
  std::vector<hrt_batch_s*> phases[2];  // [0] forward, [1] adjoint
};

namespace {
void free_split(hrt_split_s* sp) {
  for (auto& ph : sp->phases)
    for (hrt_batch_s* b : ph) free_batch(b);
  for (hrt_plan_t q : sp->parts) hrt_plan_destroy(q);
  sp->magic = 0;
  delete sp;
}

hrt_status check_split(hrt_split_t sp) {
  if (!sp || sp->magic != kSplitMagic) return set_err(HRT_ERR_BAD_HANDLE, "bad split handle");
  return HRT_OK;
}
}  // namespace

hrt_status hrt_split_describe(const hrt_desc* desc, int32_t n_t, const int32_t* t_edges,
                              int32_t n_q, const int32_t* q_edges, int32_t part,
                              hrt_desc* sub_out, int32_t* window_out, hrt_info* info_out) {
  if (!desc) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  hrt_desc sub;
  PartView v;
  std::string err;
  hrt_status s = split_part(*desc, n_t, t_edges, n_q, q_edges, part, sub, v, err);
  if (s != HRT_OK) return set_err(s, err);
  if (sub_out) *sub_out = sub;
  if (window_out) {
    window_out[0] = v.j_lo;
    window_out[1] = v.j_hi;
    window_out[2] = v.radon_row0;
    window_out[3] = v.radon_row0 + sub.nq;
  }
  if (info_out) {
    Geometry g;
    s = build_geometry(sub, 163840 - kBandStaticLds, g, err, &v);
    if (s != HRT_OK) return set_err(s, err);
    fill_info(g, info_out);
  }
  return HRT_OK;
}

hrt_status hrt_split_create(const hrt_desc* desc, int32_t n_t, const int32_t* t_edges,
                            int32_t n_q, const int32_t* q_edges, hrt_split_t* out) {
  if (!desc || !out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (n_t < 1 || n_q < 1 || n_t > 64 || n_q > 64)
    return set_err(HRT_ERR_INVALID_ARG, "1 to 64 bands per axis");
  auto* sp = new hrt_split_s();
  sp->magic = kSplitMagic;
  sp->d = *desc;
  sp->n_t = n_t;
  sp->n_q = n_q;
  {
    hipError_t e = hipGetDevice(&sp->device);
    if (e != hipSuccess) {
      free_split(sp);
      return hip_err(e, "hipGetDevice");
    }
  }
  for (int part = 0; part < n_t * n_q; ++part) {
    hrt_desc sub;
    PartView v;
    std::string err;
    hrt_status s = split_part(*desc, n_t, t_edges, n_q, q_edges, part, sub, v, err);
    hrt_plan_t pl = nullptr;
    if (s == HRT_OK) {
      s = create_plan(&sub, &v, &pl);
      err = g_last_error;
    }
    if (s != HRT_OK) {
      free_split(sp);
      return set_err(s, "part " + std::to_string(part) + ": " + err);
    }
    sp->parts.push_back(pl);
  }
  // forward: phase 0 = the last time band of every slowness band (covering
  // every tau of its rows), phase k = time band k - 1; adjoint: phase 0 =
  // the first slowness band of every time band, phase k = slowness band k
  for (int dir = 0; dir < 2; ++dir) {
    const int nph = dir == 0 ? n_t : n_q;
    const int per = dir == 0 ? n_q : n_t;
    for (int k = 0; k < nph; ++k) {
      auto* b = new hrt_batch_s();
      b->magic = kBatchMagic;
      b->device = sp->device;
      b->owns_plans = false;
      for (int m = 0; m < per; ++m) {
        const int part = dir == 0 ? m * n_t + (k == 0 ? n_t - 1 : k - 1) : k * n_t + m;
        b->plans.push_back(sp->parts[part]);
      }
      b->data_off.assign(per + 1, 0);
      b->radon_off.assign(per + 1, 0);
      sp->phases[dir].push_back(b);
      const bool acc = k > 0 || (desc->flags & HRT_ACCUMULATE_OUTPUT);
      hrt_status s = build_batch_tables(b, std::vector<int>(per, acc ? 1 : 0));
      if (s != HRT_OK) {
        const std::string e = g_last_error;
        free_split(sp);
        return set_err(s, e);
      }
    }
  }
  *out = sp;
  return HRT_OK;
}

hrt_status hrt_split_query(hrt_split_t sp, int32_t part, hrt_info* out) {
  hrt_status s = check_split(sp);
  if (s != HRT_OK) return s;
  if (!out || part < 0 || part >= static_cast<int32_t>(sp->parts.size()))
    return set_err(HRT_ERR_INVALID_ARG, "null argument or part out of range");
  *out = sp->parts[part]->info;
  return HRT_OK;
}

static hrt_status split_chain(hrt_split_t sp, const float* in, float* out, void* stream,
                              bool adjoint) {
  hrt_status s = check_split(sp);
  if (s != HRT_OK) return s;
  if (!in || !out) return set_err(HRT_ERR_INVALID_ARG, "null array");
  const size_t nd = static_cast<size_t>(sp->d.nx) * sp->d.nt * sizeof(float);
  const size_t nr = static_cast<size_t>(sp->d.nq) * sp->d.ntau * sizeof(float);
  if (overlaps(in, adjoint ? nr : nd, out, adjoint ? nd : nr))
    return set_err(HRT_ERR_INVALID_ARG, "input and output overlap");
  DeviceGuard guard(sp->device);
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const auto& phases = sp->phases[adjoint ? 1 : 0];
  for (size_t k = 0; k < phases.size(); ++k) {
    hrt_batch_s* b = phases[k];
    const bool acc = k > 0 || (sp->d.flags & HRT_ACCUMULATE_OUTPUT);
    if (b->plans.size() == 1) run_chain(b->plans[0], in, out, st, adjoint, acc);
    else run_batch(b, in, out, st, adjoint);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, adjoint ? "split adjoint launch" : "split forward launch");
  return HRT_OK;
}

hrt_status hrt_split_forward(hrt_split_t sp, const float* f, float* g, void* stream) {
  return split_chain(sp, f, g, stream, false);
}

hrt_status hrt_split_adjoint(hrt_split_t sp, const float* g, float* f, void* stream) {
  return split_chain(sp, g, f, stream, true);
}

void hrt_split_destroy(hrt_split_t sp) {
  if (!sp || sp->magic != kSplitMagic) return;
  DeviceGuard guard(sp->device);
  (void)hipDeviceSynchronize();
  free_split(sp);
}

hrt_status hrt_query(hrt_plan_t p, hrt_info* out) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  *out = p->info;
  return HRT_OK;
}

hrt_status hrt_plan_kernel(hrt_plan_t p, float* host_out) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!host_out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  DeviceGuard guard(p->device);
  HRT_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  HRT_HIP(hipMemcpy(host_out, p->K,
                    static_cast<size_t>(p->g.K1) * p->g.K2 * sizeof(float2),
                    hipMemcpyDeviceToHost),
          "copy kernel");
  return HRT_OK;
}

static void release_profile(hrt_plan_t p) {
  for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
  p->prof_ev.clear();
  p->prof_stage.clear();
  p->prof_used = 0;
}

hrt_status hrt_profile_begin(hrt_plan_t p, int32_t max_records) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (max_records < 1 || max_records > (1 << 20))
    return set_err(HRT_ERR_INVALID_ARG, "max_records out of range");
  DeviceGuard guard(p->device);
  release_profile(p);
  p->prof_ev.resize(2 * static_cast<size_t>(max_records));
  for (auto& e : p->prof_ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      e = nullptr;
      p->prof_ev.clear();
      return hip_err(r, "hipEventCreate");
    }
  }
  p->prof_stage.assign(max_records, -1);
  p->prof_used = 0;
  return HRT_OK;
}

hrt_status hrt_profile_end(hrt_plan_t p, double* ms_sum, int64_t* count) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  DeviceGuard guard(p->device);
  double ms[HRT_PROFILE_SLOTS] = {};
  int64_t cnt[HRT_PROFILE_SLOTS] = {};
  hrt_status out = HRT_OK;
  for (int i = 0; i < p->prof_used; ++i) {
    float t = 0.f;
    hipError_t r = hipEventSynchronize(p->prof_ev[2 * i + 1]);
    if (r == hipSuccess) r = hipEventElapsedTime(&t, p->prof_ev[2 * i], p->prof_ev[2 * i + 1]);
    if (r != hipSuccess) {
      out = hip_err(r, "hipEventElapsedTime");
      break;
    }
    ms[p->prof_stage[i]] += t;
    cnt[p->prof_stage[i]] += 1;
  }
  release_profile(p);
  for (int i = 0; i < HRT_PROFILE_SLOTS; ++i) {
    if (ms_sum) ms_sum[i] = ms[i];
    if (count) count[i] = cnt[i];
  }
  return out;
}

void hrt_plan_destroy(hrt_plan_t p) {
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    if (!p || !g_plans.erase(p)) return;
  }
  DeviceGuard guard(p->device);
  (void)hipDeviceSynchronize();
  release_profile(p);
  free_plan(p);
  p->magic = 0;
  delete p;
}

}  // extern "C"
