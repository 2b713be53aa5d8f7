// Host side of the libnk C ABI (include/nk.h): argument validation,
// workspace planning and kernel launch sequencing on the caller's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nk.h"
#include "nk_kernels.h"

using nk::NetDesc;

// Scratch of nk_fc_nngp_static: the first-layer diagonals of both image
// sets (n1 + n2 floats).  One copy per device, held until the process ends.
// Host code never names it as an address: the device address of each
// device's copy comes from hipGetSymbolAddress (see fc_static_scratch).
constexpr int64_t kFcStaticFloats = (int64_t)1 << 21;  // 8 MiB: n1 + n2 <= 2,097,152
static __device__ __align__(256) float scratch[kFcStaticFloats];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return NK_OK;
}

int hip_fail(const char* where) {
  hipError_t e = hipGetLastError();
  return fail(NK_EHIP, "%s: %s", where, hipGetErrorString(e));
}

// ---- kernel timing ------------------------------------------------------
struct ProfRec {
  std::string name;
  hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::map<std::string, std::pair<int64_t, double>> g_prof_done;
thread_local bool g_capturing = false;  // no per-launch events inside a graph capture

// Brackets one launch with events when profiling is on.
struct ProfScope {
  bool on = false;
  ProfRec rec;
  hipStream_t s;
  ProfScope(const char* name, hipStream_t stream) : s(stream) {
    {
      std::lock_guard<std::mutex> g(g_prof_mu);
      on = g_prof_on && !g_capturing;
    }
    if (!on) return;
    rec.name = name;
    if (hipEventCreate(&rec.start) != hipSuccess) {
      on = false;
      return;
    }
    if (hipEventCreate(&rec.stop) != hipSuccess) {
      hipEventDestroy(rec.start);
      on = false;
      return;
    }
    hipEventRecord(rec.start, s);
  }
  ~ProfScope() {
    if (!on) return;
    hipEventRecord(rec.stop, s);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_pending.push_back(rec);
  }
};

struct Bump {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = (off + 255) & ~(size_t)255;
    off = o + bytes;
    return o;
  }
};

constexpr int kPairTile = 16;           // images per side of a pair-order tile
constexpr int64_t kDefaultChunk = 16384;  // pairs per stage pass for workspace queries
constexpr int64_t kDefaultChunk64 = 1024;  // the same for 64x64 inputs (4 MiB of pooled output per pair)
constexpr int64_t kPrepBlocks = 2048;     // images prepared per launch

constexpr size_t kLdsDynamicMax = 160 * 1024 - 1024;  // dynamic LDS per workgroup

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_myrtle(const nk_myrtle_cfg* c, NetDesc* net, bool allow64 = false) {
  if (!c) return fail(NK_EINVAL, "cfg is NULL");
  if (c->H <= 0 || c->W <= 0 || c->C <= 0 || c->n_stages <= 0)
    return fail(NK_EINVAL, "H, W, C and n_stages must be positive");
  if (!(c->sigma_w2 > 0.f) || !(c->sigma_b2 >= 0.f)) return fail(NK_EINVAL, "need sigma_w2 > 0 and sigma_b2 >= 0");
  if (c->n_stages > NK_MAX_STAGES) return fail(NK_EUNSUPPORTED, "n_stages > %d", NK_MAX_STAGES);
  for (int s = 0; s < c->n_stages; ++s)
    if (c->depth[s] < 0) return fail(NK_EINVAL, "negative depth");
  if (c->filter != 3) return fail(NK_EUNSUPPORTED, "only 3x3 filters are supported (filter = %d)", c->filter);
  if (c->H != c->W) return fail(NK_EUNSUPPORTED, "only square images are supported");
  if (c->C > 4) return fail(NK_EUNSUPPORTED, "at most 4 input channels are supported");
  if (!is_pow2(c->H) || c->H > 64) return fail(NK_EUNSUPPORTED, "H must be a power of two <= 64 (H = %d)", c->H);
  if (c->H == 64) {
    if (!allow64) return fail(NK_EUNSUPPORTED, "64x64 inputs: only the NNGP block (nk_myrtle_nngp) supports them");
    if (c->n_stages < 2) return fail(NK_EUNSUPPORTED, "64x64 inputs need at least two stages (the first one pools)");
    if (c->depth[0] > 2) return fail(NK_EUNSUPPORTED, "64x64 inputs: at most 2 conv layers in the first stage");
  }
  if ((c->H >> (c->n_stages - 1)) < 2)
    return fail(NK_EUNSUPPORTED, "the last stage must be at least 2 x 2 (H = %d, %d stages)", c->H, c->n_stages);
  if (c->depth[0] < 1) return fail(NK_EUNSUPPORTED, "the first stage needs at least one conv layer");
  for (int s = 0; s < c->n_stages; ++s)
    if (c->depth[s] > NK_MAX_DEPTH) return fail(NK_EUNSUPPORTED, "depth per stage must be <= %d", NK_MAX_DEPTH);
  net->hw = c->H;
  net->C = c->C;
  net->S = c->n_stages;
  for (int s = 0; s < NK_MAX_STAGES; ++s) net->depth[s] = s < c->n_stages ? c->depth[s] : 0;
  net->sw2 = c->sigma_w2;
  net->sb2 = c->sigma_b2;
  for (int s = 0; s < net->S; ++s) {
    const int N = net->hw >> s;
    const bool seed = s == 0, pool = s + 1 < net->S;
    // 160 KiB per workgroup, less 1 KiB for the kernels' static LDS
    const size_t lds = N == 64 ? nk::stage64_lds_bytes(net->depth[s], net->C) : nk::stage_lds_bytes(N, net->depth[s], pool, seed);
    if (lds > kLdsDynamicMax)
      return fail(NK_EUNSUPPORTED, "stage %d needs more than 160 KiB of LDS", s);
  }
  return NK_OK;
}

// Device address of this device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
int fc_static_scratch(float** out) {
  static std::atomic<float*> addr[nk::kMaxDevices];
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hip_fail("hipGetDevice");
  if (dev < 0 || dev >= nk::kMaxDevices) return fail(NK_EUNSUPPORTED, "device index %d out of range", dev);
  float* p = addr[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> g(mu);
    p = addr[dev].load(std::memory_order_relaxed);
    if (!p) {
      void* q = nullptr;
      if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q)
        return hip_fail("hipGetSymbolAddress(scratch)");
      p = static_cast<float*>(q);
      addr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return NK_OK;
}

struct MyrtlePlan {
  size_t tab1 = 0, tab2 = 0, scratch = 0, buf[NK_MAX_STAGES] = {0, 0, 0, 0};
  size_t total = 0;
};

MyrtlePlan plan_myrtle(const NetDesc& net, int64_t n1, int64_t n2, bool sym, int64_t chunk) {
  MyrtlePlan p;
  Bump b;
  const size_t tl = (size_t)nk::table_len(net) * sizeof(float2);
  p.tab1 = b.take(tl * n1);
  p.tab2 = sym ? p.tab1 : b.take(tl * n2);
  const int64_t pb = std::min<int64_t>(std::max(n1, n2), kPrepBlocks);
  p.scratch = b.take((size_t)nk::prep_scratch_doubles(net) * sizeof(double) * pb);
  for (int s = 1; s < net.S; ++s) {
    const size_t n = (size_t)(net.hw >> s);
    p.buf[s] = b.take(n * n * n * n * sizeof(float) * chunk);
  }
  p.total = b.off + 256;
  return p;
}

constexpr int64_t kPrepBwdBlocks = 256;  // images per self-recursion adjoint launch

struct BwdPlan {
  size_t tab1 = 0, tab2 = 0, scratch = 0, W1 = 0, W2 = 0, xb1 = 0, xb2 = 0, sums = 0, bscratch = 0;
  size_t buf[NK_MAX_STAGES] = {0, 0, 0, 0}, gbuf[NK_MAX_STAGES] = {0, 0, 0, 0};
  size_t total = 0;
};

BwdPlan plan_bwd(const NetDesc& net, int64_t n1, int64_t n2, bool sym, int64_t chunk) {
  BwdPlan p;
  Bump b;
  const size_t tl = (size_t)nk::table_len(net);
  const size_t img = (size_t)net.hw * net.hw * net.C;
  p.tab1 = b.take(tl * sizeof(float2) * n1);
  p.tab2 = sym ? p.tab1 : b.take(tl * sizeof(float2) * n2);
  const int64_t pb = std::min<int64_t>(std::max(n1, n2), kPrepBlocks);
  p.scratch = b.take((size_t)nk::prep_scratch_doubles(net) * sizeof(double) * pb);
  p.W1 = b.take(tl * sizeof(double) * n1);
  p.W2 = sym ? p.W1 : b.take(tl * sizeof(double) * n2);
  p.xb1 = b.take(img * sizeof(double) * n1);
  p.xb2 = sym ? p.xb1 : b.take(img * sizeof(double) * n2);
  p.sums = b.take(4 * sizeof(double));
  const int64_t pbb = std::min<int64_t>(std::max(n1, n2), kPrepBwdBlocks);
  p.bscratch = b.take((size_t)nk::prep_bwd_scratch_doubles(net) * sizeof(double) * pbb);
  for (int s = 1; s < net.S; ++s) {
    const size_t n = (size_t)(net.hw >> s);
    p.buf[s] = b.take(n * n * n * n * sizeof(float) * chunk);
    p.gbuf[s] = b.take(n * n * n * n * sizeof(float) * chunk);
  }
  p.total = b.off + 256;
  return p;
}

int64_t max_chunk_bwd(const NetDesc& net, int64_t n1, int64_t n2, bool sym, size_t ws_bytes, int64_t npairs) {
  const size_t fixed = plan_bwd(net, n1, n2, sym, 0).total;
  size_t per = 0;
  for (int s = 1; s < net.S; ++s) {
    const size_t n = (size_t)(net.hw >> s);
    per += 2 * n * n * n * n * sizeof(float);
  }
  if (ws_bytes < fixed + 512 * NK_MAX_STAGES) return 0;
  if (per == 0) return npairs;
  return std::min((int64_t)((ws_bytes - fixed - 512 * NK_MAX_STAGES) / per), npairs);
}

int64_t max_chunk(const NetDesc& net, int64_t n1, int64_t n2, bool sym, size_t ws_bytes, int64_t npairs) {
  const size_t fixed = plan_myrtle(net, n1, n2, sym, 0).total;
  size_t per = 0;
  for (int s = 1; s < net.S; ++s) {
    const size_t n = (size_t)(net.hw >> s);
    per += n * n * n * n * sizeof(float);
  }
  if (ws_bytes < fixed + 256 * NK_MAX_STAGES) return 0;
  if (per == 0) return npairs;
  int64_t c = (int64_t)((ws_bytes - fixed - 256 * NK_MAX_STAGES) / per);
  return std::min(c, npairs);
}

struct KrrPlan {
  size_t A = 0, mean = 0, info = 0, X = 0, B = 0, Z = 0, G = 0, sq = 0, loss = 0, total = 0;
};

// n: train size; w = max(m test, c targets)
KrrPlan krr_plan(int64_t n, int64_t w) {
  KrrPlan p;
  Bump b;
  w = std::max<int64_t>(w, 1);
  p.A = b.take(sizeof(double) * (size_t)n * n);
  p.mean = b.take(sizeof(double) * 2);
  p.info = b.take(sizeof(int) * 4);
  p.X = b.take(sizeof(double) * (size_t)n * w);
  p.B = b.take(sizeof(double) * (size_t)n * w);
  p.Z = b.take(sizeof(double) * (size_t)n * w);
  p.G = b.take(sizeof(double) * (size_t)w * w);
  p.sq = b.take(sizeof(double) * (size_t)w * w);
  p.loss = b.take(sizeof(double) * 2);
  p.total = b.off + 256;
  return p;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}


// ---- batched tiles (many uneven Gram tiles in one scheduled pass) --------

// Schedule and shape of a batched pass: pairs per stage pass, image-tile
// side of the pair order, persistent grid or one workgroup per unit, and the
// pairs-per-workgroup multiplier of the stage kernels of tiles of at most
// 16 x 16.
struct BatchParams {
  int64_t chunk = kDefaultChunk;
  int T = kPairTile;
  int persist = 0;
  int ppm = 1;
};

struct TuneRecord {
  BatchParams best;
  std::vector<nk_batched_candidate> cands;
};
std::mutex g_tune_mu;
std::map<std::string, TuneRecord> g_tune;  // per network (one process-wide choice)

std::string net_key(const NetDesc& net) {
  char b[160];
  snprintf(b, sizeof b, "hw%d C%d S%d d%d,%d,%d,%d b%d", net.hw, net.C, net.S, net.depth[0], net.depth[1],
           net.depth[2], net.depth[3], net.sb2 != 0.f ? 1 : 0);
  return b;
}

struct BatchLayout {
  std::vector<nk::TileDesc> desc;   // host copy of the tile table
  std::vector<std::pair<const float*, int64_t>> images;  // distinct image arrays and the rows used
  int64_t rows = 0;                 // table rows (images prepared)
  int64_t npairs = 0;
};

int batch_layout(const nk_tile* tiles, int32_t ntiles, const NetDesc& net, BatchLayout* L) {
  std::map<const float*, size_t> idx;
  for (int32_t t = 0; t < ntiles; ++t) {
    const nk_tile& u = tiles[t];
    if (!u.x1 || !u.x2 || !u.K) return fail(NK_EINVAL, "tile %d: null pointer", t);
    if (u.n1 <= 0 || u.n2 <= 0) return fail(NK_EINVAL, "tile %d: n1 and n2 must be positive", t);
    if (u.ldk < u.n2) return fail(NK_EINVAL, "tile %d: ldk < n2", t);
    const float* xs[2] = {u.x1, u.x2};
    const int64_t ns[2] = {u.n1, u.n2};
    for (int k = 0; k < 2; ++k) {
      auto it = idx.find(xs[k]);
      if (it == idx.end()) {
        idx[xs[k]] = L->images.size();
        L->images.push_back({xs[k], ns[k]});
      } else {
        L->images[it->second].second = std::max(L->images[it->second].second, ns[k]);
      }
    }
  }
  std::vector<int64_t> row0(L->images.size());
  for (size_t i = 0; i < L->images.size(); ++i) {
    row0[i] = L->rows;
    L->rows += L->images[i].second;
  }
  int64_t p = 0;
  for (int32_t t = 0; t < ntiles; ++t) {
    const nk_tile& u = tiles[t];
    nk::TileDesc d;
    memset(&d, 0, sizeof d);
    d.sym = (u.x1 == u.x2 && u.n1 == u.n2) ? 1 : 0;
    d.p_begin = p;
    d.n1 = u.n1;
    d.n2 = u.n2;
    d.t1 = row0[idx[u.x1]];
    d.t2 = row0[idx[u.x2]];
    d.x1 = u.x1;
    d.x2 = u.x2;
    d.K = u.K;
    d.ldk = u.ldk;
    p += nk::pair_count(u.n1, u.n2, d.sym);
    L->desc.push_back(d);
  }
  L->npairs = p;
  (void)net;
  return NK_OK;
}

struct BatchPlan {
  size_t desc = 0, tab = 0, scratch = 0, buf[NK_MAX_STAGES] = {0, 0, 0, 0};
  size_t total = 0;
};

BatchPlan plan_batched(const NetDesc& net, int64_t rows, int64_t ntiles, int64_t chunk) {
  BatchPlan p;
  Bump b;
  p.desc = b.take(sizeof(nk::TileDesc) * (size_t)std::max<int64_t>(ntiles, 1));
  p.tab = b.take((size_t)nk::table_len(net) * sizeof(float2) * rows);
  const int64_t pb = std::min<int64_t>(std::max<int64_t>(rows, 1), kPrepBlocks);
  p.scratch = b.take((size_t)nk::prep_scratch_doubles(net) * sizeof(double) * pb);
  for (int s = 1; s < net.S; ++s) {
    const size_t n = (size_t)(net.hw >> s);
    p.buf[s] = b.take(n * n * n * n * sizeof(float) * chunk);
  }
  p.total = b.off + 256;
  return p;
}

// Compute units of the current device (0 if unknown), queried once per device.
int cu_count() {
  static std::atomic<int> counts[nk::kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev < nk::kMaxDevices) {
    const int c = counts[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 0;
  if (dev < nk::kMaxDevices) counts[dev].store(n, std::memory_order_relaxed);
  return n;
}

// Stage passes of chunks [p_lo, p_hi) of a batched pass.
int run_batched_stages(const NetDesc& net, const nk::TileDesc* ddesc, int ntiles, const float2* tab, float* const* bufs,
                       const BatchParams& bp, int64_t p_lo, int64_t p_hi, int only_stage, hipStream_t stream) {
  for (int64_t p0 = p_lo; p0 < p_hi; p0 += bp.chunk) {
    const int64_t np = std::min(bp.chunk, p_hi - p0);
    for (int s = 0; s < net.S; ++s) {
      if (only_stage >= 0 && s != only_stage) continue;
      nk::StageArgs a;
      memset(&a, 0, sizeof a);
      a.T = bp.T;
      a.p0 = p0;
      a.np = np;
      a.tiles = ddesc;
      a.ntiles = ntiles;
      a.tab1 = tab;
      a.tab2 = tab;
      a.tablen = nk::table_len(net);
      a.taboff = nk::table_off(net, s);
      a.C = net.C;
      a.D = net.depth[s];
      a.sb2 = net.sb2;
      a.seed_scale = net.sw2 / 9.0f / (float)net.C;
      a.img_floats = (int64_t)net.hw * net.hw * net.C;
      const bool pool = s + 1 < net.S;
      a.in = s > 0 ? bufs[s] : nullptr;
      a.out = pool ? bufs[s + 1] : nullptr;
      if (bp.persist) {
        const int occ =
            nk::stage_occupancy(net.hw >> s, net.depth[s], s == 0, pool, net.sb2 != 0.f, net.C, bp.ppm);
        const int cus = cu_count();
        if (occ <= 0 || cus <= 0) return hip_fail("occupancy query");
        const int64_t ppwg = nk::stage_pairs_per_wg(net.hw >> s, pool, bp.ppm);
        const int64_t units = (np + ppwg - 1) / ppwg;
        // all workgroups resident (occupancy x CUs), a multiple of the 8 XCDs,
        // and no more than the units to share
        int64_t g = (int64_t)occ * cus / 8 * 8;
        a.persist = (int)std::max<int64_t>(8, std::min<int64_t>(g, (units + 7) / 8 * 8));
      }
      char nm[48];
      snprintf(nm, sizeof nm, "myrtle_stage%d_n%d", s + 1, net.hw >> s);
      ProfScope ps(nm, stream);
      if (nk::launch_stage(net.hw >> s, a, s == 0, pool, net.sb2 != 0.f, stream, bp.ppm))
        return hip_fail("stage kernel");
    }
  }
  return NK_OK;
}

// Times the first-stage kernel of the pass under each schedule candidate on
// the pass's own first pairs and keeps the fastest; then, under that
// schedule, times the stages of tiles of at most 16 x 16 with one and with
// two pairs-per-workgroup multiples and keeps the faster shape.  Results are
// identical under every candidate: the schedule only permutes pairs, and a
// pair's arithmetic does not depend on how many pairs share a workgroup.
int autotune(const NetDesc& net, const nk::TileDesc* ddesc, int ntiles, const float2* tab, float* const* bufs,
             int64_t npairs, int64_t max_chunk_ws, hipStream_t s, TuneRecord* rec) {
  // pairs per stage pass: the candidates that fit the workspace, cut to the
  // pass size (duplicates dropped)
  std::vector<int64_t> chunks;
  for (int64_t c : {(int64_t)8192, (int64_t)16384, (int64_t)32768}) {
    const int64_t e = std::min(std::min(c, max_chunk_ws), npairs);
    if (e > 0 && std::find(chunks.begin(), chunks.end(), e) == chunks.end()) chunks.push_back(e);
  }
  const int Ts[3] = {8, 16, 32};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return hip_fail("event");
  double best = 1e30;
  bool first = true;
  int rc = NK_OK;
  for (int64_t c : chunks) {
    const int64_t np = c;
    for (int T : Ts) {
      for (int persist = 0; persist <= 1; ++persist) {
        BatchParams bp;
        bp.chunk = c;
        bp.T = T;
        bp.persist = persist;
        if (first) {  // warm-up
          if ((rc = run_batched_stages(net, ddesc, ntiles, tab, bufs, bp, 0, np, 0, s))) goto done;
          first = false;
        }
        hipEventRecord(e0, s);
        if ((rc = run_batched_stages(net, ddesc, ntiles, tab, bufs, bp, 0, np, 0, s))) goto done;
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = hip_fail("tuning event");
          goto done;
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        nk_batched_candidate cd;
        memset(&cd, 0, sizeof cd);
        cd.chunk = c;
        cd.pair_tile = T;
        cd.persistent = persist;
        cd.us_per_pair = 1e3 * ms / (double)np;
        cd.kind = 0;
        cd.wg_pairs_mult = 1;
        rec->cands.push_back(cd);
        if (cd.us_per_pair < best) {
          best = cd.us_per_pair;
          rec->best = bp;
        }
      }
    }
  }
  {
    // kernel shape of the stages of tiles of at most 16 x 16
    int first_small = -1;
    for (int st = 0; st < net.S; ++st)
      if ((net.hw >> st) <= 16) {
        first_small = st;
        break;
      }
    if (first_small >= 0) {
      BatchParams bp = rec->best;
      const int64_t np = bp.chunk;
      // inputs of the first such stage for the first np pairs
      for (int st = 0; st < first_small; ++st)
        if ((rc = run_batched_stages(net, ddesc, ntiles, tab, bufs, bp, 0, np, st, s))) goto done;
      double best_shape = 1e30;
      for (int m = 1; m <= 2; ++m) {
        bp.ppm = m;
        for (int rep = 0; rep < 2; ++rep) {  // warm-up, then timed
          if (rep) hipEventRecord(e0, s);
          for (int st = first_small; st < net.S; ++st)
            if ((rc = run_batched_stages(net, ddesc, ntiles, tab, bufs, bp, 0, np, st, s))) goto done;
        }
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = hip_fail("tuning event");
          goto done;
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        nk_batched_candidate cd;
        memset(&cd, 0, sizeof cd);
        cd.chunk = bp.chunk;
        cd.pair_tile = bp.T;
        cd.persistent = bp.persist;
        cd.us_per_pair = 1e3 * ms / (double)np;
        cd.kind = 1;
        cd.wg_pairs_mult = m;
        rec->cands.push_back(cd);
        if (cd.us_per_pair < best_shape) {
          best_shape = cd.us_per_pair;
          rec->best.ppm = m;
        }
      }
    }
  }
done:
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}

struct GraphEntry {
  std::string sig;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;  // most recent last
hipStream_t g_cap_stream = nullptr;

void drop_graph(GraphEntry& e) {
  if (e.exec) hipGraphExecDestroy(e.exec);
  if (e.graph) hipGraphDestroy(e.graph);
  e.exec = nullptr;
  e.graph = nullptr;
}


// ---- neural tangent kernel -------------------------------------------------

// kappa of layer l of stage s (the scale of the next linear step on that
// ReLU output), as the variance tables fold it into beta: sigma_w2 / 9 inside
// a stage, times 1/16 per pool before the next layer, sigma_w2 / n^4 before
// the readout.
double layer_kappa(const NetDesc& net, int s, int l) {
  const double c = (double)net.sw2 / 9.0;
  if (l + 1 < net.depth[s]) return c;
  int s2 = s + 1;
  double f = 1.0 / 16.0;
  while (s2 < net.S && net.depth[s2] == 0) {
    f /= 16.0;
    ++s2;
  }
  const double n = (double)(net.hw >> s);
  return s2 < net.S ? c * f : (double)net.sw2 / (n * n * n * n);
}

MyrtlePlan plan_ntk(const NetDesc& net, int64_t n1, int64_t n2, bool sym, int64_t chunk) {
  // the NNGP plan with every chunk buffer twice (the carried NNGP and tangent tiles)
  MyrtlePlan p;
  Bump b;
  const size_t tl = (size_t)nk::table_len(net) * sizeof(float2);
  p.tab1 = b.take(tl * n1);
  p.tab2 = sym ? p.tab1 : b.take(tl * n2);
  const int64_t pb = std::min<int64_t>(std::max(n1, n2), kPrepBlocks);
  p.scratch = b.take((size_t)nk::prep_scratch_doubles(net) * sizeof(double) * pb);
  for (int s = 1; s < net.S; ++s) {
    const size_t n = (size_t)(net.hw >> s);
    p.buf[s] = b.take(2 * n * n * n * n * sizeof(float) * chunk);
  }
  p.total = b.off + 256;
  return p;
}

int64_t max_chunk_ntk(const NetDesc& net, int64_t n1, int64_t n2, bool sym, size_t ws_bytes, int64_t npairs) {
  const size_t fixed = plan_ntk(net, n1, n2, sym, 0).total;
  size_t per = 0;
  for (int s = 1; s < net.S; ++s) {
    const size_t n = (size_t)(net.hw >> s);
    per += 2 * n * n * n * n * sizeof(float);
  }
  if (ws_bytes < fixed + 256 * NK_MAX_STAGES) return 0;
  if (per == 0) return npairs;
  return std::min((int64_t)((ws_bytes - fixed - 256 * NK_MAX_STAGES) / per), npairs);
}

// Myrtle Gram block through the stage kernels (tables already prepared).
// First-stage output floats of one pair (the pooled covariance that the
// second stage reads), 0 for a one-stage network.
int64_t stage1_out_floats(const NetDesc& net) {
  if (net.S < 2) return 0;
  const int64_t q = net.hw >> 1;
  return q * q * q * q;
}

// keep1 (optional): the first stage's outputs go to keep1 at the pair's
// position in the block (pair p at keep1 + p * stage1_out_floats) instead of
// the chunk buffer, so that they outlive the pass.
int run_myrtle_pairs(const NetDesc& net, const float* x1, int64_t n1, const float* x2, int64_t n2, bool sym,
                     const float2* tab1, const float2* tab2, float* K, int64_t ldk, float* const* bufs,
                     int64_t chunk, hipStream_t stream, float* keep1 = nullptr) {
  const int64_t npairs = nk::pair_count(n1, n2, sym);
  for (int64_t p0 = 0; p0 < npairs; p0 += chunk) {
    const int64_t np = std::min(chunk, npairs - p0);
    float* b1 = keep1 ? keep1 + p0 * stage1_out_floats(net) : bufs[1];
    for (int s = 0; s < net.S; ++s) {
      nk::StageArgs a;
      memset(&a, 0, sizeof a);
      a.n1 = n1;
      a.n2 = n2;
      a.sym = sym ? 1 : 0;
      a.T = kPairTile;
      a.p0 = p0;
      a.np = np;
      a.x1 = x1;
      a.x2 = x2;
      a.tab1 = tab1;
      a.tab2 = tab2;
      a.tablen = nk::table_len(net);
      a.taboff = nk::table_off(net, s);
      a.C = net.C;
      a.D = net.depth[s];
      a.sb2 = net.sb2;
      a.seed_scale = net.sw2 / 9.0f / (float)net.C;
      a.img_floats = (int64_t)net.hw * net.hw * net.C;
      const bool pool = s + 1 < net.S;
      a.in = s > 0 ? (s == 1 ? b1 : bufs[s]) : nullptr;
      a.out = pool ? (s == 0 ? b1 : bufs[s + 1]) : nullptr;
      a.K = K;
      a.ldk = ldk;
      char nm[48];
      snprintf(nm, sizeof nm, "myrtle_stage%d_n%d", s + 1, net.hw >> s);
      ProfScope ps(nm, stream);
      const int rc = (net.hw >> s) == 64 ? nk::launch_stage64(a, net.sb2 != 0.f, stream)
                                         : nk::launch_stage(net.hw >> s, a, s == 0, pool, net.sb2 != 0.f, stream);
      if (rc) return hip_fail("stage kernel");
    }
  }
  return NK_OK;
}


int check_bwd_lds(const NetDesc& net) {
  for (int s = 0; s < net.S; ++s)
    if (nk::stage_bwd_lds_bytes(net.hw >> s, net.depth[s], s == 0) > kLdsDynamicMax)
      return fail(NK_EUNSUPPORTED, "adjoint of stage %d needs more than 160 KiB of LDS", s);
  return NK_OK;
}

// Adjoint pair passes of one Gram block for the cotangent dK: adds the
// table adjoints of both images into W1 / W2, the seed gradients into
// xb1 / xb2 and the sigma terms into sums (nothing is cleared; the self-chain
// reverse and the casts are the caller's).  Per chunk: the forward stages up
// to the last stage's input (the checkpoints), then the adjoint stages in
// reverse order.
// xj: accumulate x2's seed gradients into xb2 (false: not wanted; xb2 may
// then be null for 32x32 images); dk_t: dK is stored transposed.
// keep1 (optional): the first stage's outputs of the whole block, as
// run_myrtle_pairs left them for the same (x1, x2, sym); the first stage is
// then not re-run.
int bwd_block(const NetDesc& net, const float* x1, int64_t n1, const float* x2, int64_t n2, bool sym, const float* dK,
              int64_t lddk, const float2* tab1, const float2* tab2, double* W1, double* W2, double* xb1, double* xb2,
              double* sums, float* const* bufs, float* const* gbufs, int64_t chunk, hipStream_t s, bool xj = true,
              bool dk_t = false, float* keep1 = nullptr) {
  const int tl = nk::table_len(net);
  const int64_t npairs = nk::pair_count(n1, n2, sym);
  for (int64_t p0 = 0; p0 < npairs; p0 += chunk) {
    const int64_t np = std::min(chunk, npairs - p0);
    float* b1 = keep1 ? keep1 + p0 * stage1_out_floats(net) : bufs[1];
    for (int st = keep1 ? 1 : 0; st + 1 < net.S; ++st) {
      nk::StageArgs a;
      memset(&a, 0, sizeof a);
      a.n1 = n1; a.n2 = n2; a.sym = sym ? 1 : 0; a.T = kPairTile; a.p0 = p0; a.np = np;
      a.x1 = x1; a.x2 = x2; a.tab1 = tab1; a.tab2 = tab2;
      a.tablen = tl; a.taboff = nk::table_off(net, st);
      a.C = net.C; a.D = net.depth[st]; a.sb2 = net.sb2; a.seed_scale = net.sw2 / 9.0f / (float)net.C;
      a.img_floats = (int64_t)net.hw * net.hw * net.C;
      a.in = st > 0 ? (st == 1 ? b1 : bufs[st]) : nullptr;
      a.out = st == 0 ? b1 : bufs[st + 1];
      char nm[48];
      snprintf(nm, sizeof nm, "myrtle_stage%d_n%d", st + 1, net.hw >> st);
      ProfScope ps(nm, s);
      if (nk::launch_stage(net.hw >> st, a, st == 0, true, net.sb2 != 0.f, s)) return hip_fail("stage kernel");
    }
    for (int st = net.S - 1; st >= 0; --st) {
      nk::StageBwdArgs b;
      memset(&b, 0, sizeof b);
      b.n1 = n1; b.n2 = n2; b.sym = sym ? 1 : 0; b.T = kPairTile; b.p0 = p0; b.np = np;
      b.x1 = x1; b.x2 = x2; b.tab1 = tab1; b.tab2 = tab2;
      b.tablen = tl; b.taboff = nk::table_off(net, st);
      b.C = net.C; b.D = net.depth[st]; b.sb2 = net.sb2; b.seed_scale = net.sw2 / 9.0f / (float)net.C;
      b.img_floats = (int64_t)net.hw * net.hw * net.C;
      b.in = st > 0 ? (st == 1 ? b1 : bufs[st]) : nullptr;
      b.gin = st + 1 < net.S ? gbufs[st + 1] : nullptr;
      b.gout = st > 0 ? gbufs[st] : nullptr;
      b.dK = dK; b.lddk = lddk; b.last = st + 1 == net.S ? 1 : 0;
      b.W1 = W1; b.W2 = W2; b.xbar1 = xb1; b.xbar2 = xb2; b.sums = sums;
      b.xj = xj ? 1 : 0; b.dk_t = dk_t ? 1 : 0;
      char nm[48];
      snprintf(nm, sizeof nm, "myrtle_stage%d_n%d_bwd", st + 1, net.hw >> st);
      ProfScope ps(nm, s);
      if (nk::launch_stage_bwd(net.hw >> st, b, st == 0, s)) return hip_fail("adjoint stage kernel");
    }
  }
  return NK_OK;
}

// Workspace of nk_krr_mse_grad: both Gram blocks and their cotangents, the
// tables, adjoint sums and gradients of both image sets, the ridge solve and
// the chunk buffers (each stage's checkpoint and its adjoint).  keep: the
// first stage's outputs of every pair of both blocks are kept from the
// forward pass for the adjoint (keep1) instead of a chunk buffer for them.
struct KrrGradPlan {
  size_t kss = 0, kts = 0, dss = 0, dts = 0, tab_s = 0, tab_t = 0, scratch = 0, krr = 0, krr_bytes = 0;
  size_t W_s = 0, W_t = 0, xb_s = 0, xb_t = 0, sums = 0, bscratch = 0;
  size_t buf[NK_MAX_STAGES] = {0, 0, 0, 0}, gbuf[NK_MAX_STAGES] = {0, 0, 0, 0};
  size_t keep1 = 0;
  bool keep = false;
  size_t total = 0;
};

KrrGradPlan plan_krr_grad(const NetDesc& net, int64_t n, int64_t m, int64_t c, int64_t chunk, bool keep = false) {
  KrrGradPlan p;
  p.keep = keep && net.S > 1;
  Bump b;
  const size_t tl = (size_t)nk::table_len(net);
  const size_t img = (size_t)net.hw * net.hw * net.C;
  p.kss = b.take(sizeof(float) * (size_t)n * n);
  p.kts = b.take(sizeof(float) * (size_t)m * n);
  p.dss = b.take(sizeof(float) * (size_t)n * n);
  p.dts = b.take(sizeof(float) * (size_t)m * n);
  p.tab_s = b.take(tl * sizeof(float2) * n);
  p.tab_t = b.take(tl * sizeof(float2) * m);
  const int64_t pb = std::min<int64_t>(std::max(n, m), kPrepBlocks);
  p.scratch = b.take((size_t)nk::prep_scratch_doubles(net) * sizeof(double) * pb);
  p.krr_bytes = krr_plan(n, std::max(m, c)).total;
  p.krr = b.take(p.krr_bytes);
  p.W_s = b.take(tl * sizeof(double) * n);
  p.W_t = b.take(tl * sizeof(double) * m);
  p.xb_s = b.take(img * sizeof(double) * n);
  p.xb_t = b.take(img * sizeof(double) * m);
  p.sums = b.take(4 * sizeof(double));
  const int64_t pbb = std::min<int64_t>(std::max(n, m), kPrepBwdBlocks);
  p.bscratch = b.take((size_t)nk::prep_bwd_scratch_doubles(net) * sizeof(double) * pbb);
  for (int s = 1; s < net.S; ++s) {
    const size_t q = (size_t)(net.hw >> s);
    if (!(p.keep && s == 1)) p.buf[s] = b.take(q * q * q * q * sizeof(float) * chunk);
    p.gbuf[s] = b.take(q * q * q * q * sizeof(float) * chunk);
  }
  if (p.keep)
    p.keep1 = b.take((size_t)stage1_out_floats(net) * sizeof(float) *
                     (size_t)(nk::pair_count(n, n, 1) + nk::pair_count(n, m, 0)));
  p.total = b.off + 256;
  return p;
}

// ---- CNN-VEC ---------------------------------------------------------------

constexpr int kCvMaxDepth = 16;

int check_cv(const nk_cv_cfg* c) {
  if (!c) return fail(NK_EINVAL, "cfg is NULL");
  if (c->H <= 0 || c->W <= 0 || c->C <= 0 || c->depth <= 0) return fail(NK_EINVAL, "H, W, C, depth must be positive");
  if (!(c->sigma_w2 > 0.f) || !(c->sigma_b2 >= 0.f)) return fail(NK_EINVAL, "need sigma_w2 > 0 and sigma_b2 >= 0");
  if (c->H != c->W || !is_pow2(c->H) || c->H < 2 || c->H > 32)
    return fail(NK_EUNSUPPORTED, "need H == W a power of two in [2, 32]");
  if (c->C > 4) return fail(NK_EUNSUPPORTED, "C > 4");
  if (c->depth > kCvMaxDepth) return fail(NK_EUNSUPPORTED, "depth > %d", kCvMaxDepth);
  return 0;
}

struct CvPlan {
  size_t tab1, tab2, d1, d2, total;
};

CvPlan cv_plan(const nk_cv_cfg* c, int64_t n1, int64_t n2, bool sym) {
  CvPlan p{};
  Bump b;
  const size_t per = (size_t)c->depth * c->H * c->W * sizeof(float2);
  p.tab1 = b.take(per * (size_t)std::max<int64_t>(n1, 1));
  p.d1 = b.take(sizeof(float) * (size_t)std::max<int64_t>(n1, 1));
  if (!sym) {
    p.tab2 = b.take(per * (size_t)std::max<int64_t>(n2, 1));
    p.d2 = b.take(sizeof(float) * (size_t)std::max<int64_t>(n2, 1));
  }
  p.total = b.off + 256;
  return p;
}

// ---- approximate kernel ridge regression ---------------------------------

constexpr int64_t kApproxMaxSolve = 8192;  // sides of the matrices factored in LDS-held solves

struct ApproxPlan {
  size_t A, D, b, v, alpha, P, rhs2, Z, mu, S, Sinv, Kinv, I, prec, acc, info, total;
};

ApproxPlan approx_plan(const nk_approx_dims& d) {
  ApproxPlan p{};
  Bump b;
  const size_t r = (size_t)std::max<int64_t>(d.r, 1), n = (size_t)std::max<int64_t>(d.n, 1);
  const size_t m = (size_t)std::max<int64_t>(d.m, 1), c = (size_t)std::max<int64_t>(d.c, 1);
  const size_t mb = (size_t)std::max<int64_t>(std::max(d.max_block, d.r), 1);
  p.A = b.take(sizeof(double) * r * r);
  p.D = b.take(sizeof(double) * mb * mb);
  p.b = b.take(sizeof(double) * r * c);
  p.v = b.take(sizeof(double) * r * c);
  p.alpha = b.take(sizeof(double) * n * c);
  p.P = b.take(sizeof(double) * m * c);
  p.rhs2 = b.take(sizeof(double) * mb * (c + m));
  p.Z = b.take(sizeof(double) * mb * (c + m));
  p.mu = b.take(sizeof(double) * m * c);
  p.S = b.take(sizeof(double) * m * m);
  p.Sinv = b.take(sizeof(double) * m * m);
  p.Kinv = b.take(sizeof(double) * m * m);
  p.I = b.take(sizeof(double) * m * m);
  p.prec = b.take(sizeof(double) * m * m);
  p.acc = b.take(sizeof(double) * m * c);
  p.info = b.take(sizeof(int) * 4);
  p.total = b.off + 256;
  return p;
}

int approx_finish(hipStream_t s, const int* info_dev, const char* what) {
  int info = 0;
  if (hipMemcpyAsync(&info, info_dev, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return hip_fail(what);
  if (info) return fail(NK_ENOTPD, "%s: a factorised matrix is not positive definite", what);
  return ok();
}

// Nystrom and SoR share v = (K_rn K_nr + lam (K_rr + jitter I))^{-1} K_rn Y.
int approx_low_rank_v(const float* K_nr, int64_t n, int64_t r, int64_t ld_nr, const float* K_rr, int64_t ld_rr,
                      const float* Y, int64_t c, double lam, double jitter, void* ws, const ApproxPlan& ap,
                      hipStream_t s) {
  double* A = at<double>(ws, ap.A);
  double* D = at<double>(ws, ap.D);
  double* bb = at<double>(ws, ap.b);
  int* info = at<int>(ws, ap.info);
  if (nk::dn_gemm_ff(K_nr, ld_nr, true, K_nr, ld_nr, A, r, r, r, n, 1.0, 0.0, true, s) ||
      nk::dn_load_shift(K_rr, ld_rr, r, jitter, D, info, s) || nk::dn_axpby(A, D, r * r, 1.0, lam, s) ||
      nk::dn_gemm_ff(K_nr, ld_nr, true, Y, c, bb, c, r, c, n, 1.0, 0.0, true, s) ||
      nk::launch_cholesky(A, r, info, s) ||
      nk::launch_chol_solve(A, r, nullptr, bb, c, at<double>(ws, ap.v), s))
    return -3;
  return 0;
}

int check_approx_common(int64_t n, int64_t m, int64_t c, double lam, double jitter, const float* Y, float* pred) {
  if (!Y || !pred) return fail(NK_EINVAL, "null pointer argument");
  if (n <= 0 || m <= 0 || c <= 0) return fail(NK_EINVAL, "need n, m, c > 0");
  if (!(lam > 0.0) || !(jitter >= 0.0)) return fail(NK_EINVAL, "need lambda > 0 and jitter >= 0");
  return 0;
}

int check_blocks(int32_t p, const float* const* K_blocks, const int64_t* sizes, int64_t* n, int64_t* maxb) {
  if (p <= 0 || !K_blocks || !sizes) return fail(NK_EINVAL, "need p > 0 blocks with pointers and sizes");
  *n = 0;
  *maxb = 0;
  for (int32_t i = 0; i < p; ++i) {
    if (!K_blocks[i] || sizes[i] <= 0) return fail(NK_EINVAL, "block %d: null pointer or size <= 0", i);
    *n += sizes[i];
    *maxb = std::max(*maxb, sizes[i]);
  }
  if (*maxb > kApproxMaxSolve) return fail(NK_EUNSUPPORTED, "block larger than %lld", (long long)kApproxMaxSolve);
  return 0;
}

// ---- kernel regression by preconditioned conjugate gradients --------------

constexpr int kPcgMaxRank = 8192;  // LDS of a pivot step holds one row of L
constexpr int kPcgGroup = 16;      // right-hand sides per CG pass

// Row splits of U^T v: about 512 four-wave workgroups, >= 256 rows each.
int pc_lt_splits(int64_t n, int r) {
  if (r <= 0) return 1;
  const int64_t g = (r + 63) / 64;
  int64_t S = (512 + g - 1) / g;
  S = std::min<int64_t>(S, (n + 255) / 256);
  return (int)std::max<int64_t>(S, 1);
}

struct PcgPlan {
  size_t d, pv, pi, dpiv, mean, piv, L, Lr, M, info, W, wpart, R, X, Z, P, Q, kpart, part1, part2, st;
  int lt_splits;
  size_t total;
};

// what: 0 = pivoted Cholesky only, 1 = full solver, 2 = product only
PcgPlan pcg_plan(int64_t n, int r, int what) {
  PcgPlan p{};
  Bump b;
  const int64_t nb = (n + 255) / 256, nbz = (n + 63) / 64;
  const size_t G = kPcgGroup;
  if (what != 2) {
    p.d = b.take(sizeof(double) * n);
    p.pv = b.take(sizeof(double) * 2 * nb);
    p.pi = b.take(sizeof(int) * 2 * nb);
    p.dpiv = b.take(sizeof(double) * std::max(r, 1));
  }
  if (what == 1) {
    p.mean = b.take(sizeof(double) * 2);
    p.piv = b.take(sizeof(int) * std::max(r, 1));
    p.L = b.take(sizeof(double) * (size_t)n * r);
    p.Lr = b.take(sizeof(double) * (size_t)n * r);
    p.M = b.take(sizeof(double) * (size_t)r * r);
    p.info = b.take(sizeof(int) * 4);
    p.lt_splits = pc_lt_splits(n, r);
    p.W = b.take(sizeof(double) * std::max(r, 1) * G);
    p.wpart = b.take(sizeof(double) * (size_t)p.lt_splits * std::max(r, 1) * G);
    p.R = b.take(sizeof(double) * n * G);
    p.X = b.take(sizeof(double) * n * G);
    p.Z = b.take(sizeof(double) * n * G);
    p.P = b.take(sizeof(double) * n * G);
    p.Q = b.take(sizeof(double) * n * G);
    p.part2 = b.take(sizeof(double) * nbz * G);
    p.st = b.take(sizeof(double) * 7 * G);
  }
  if (what != 0) {
    p.kpart = b.take(sizeof(double) * (size_t)nk::kmv_splits(n) * n * G);
    p.part1 = b.take(sizeof(double) * nbz * G);
  }
  p.total = b.off + 256;
  return p;
}

// Event bracket of the library's timing records, for one launch inside a launcher.
struct ScopeHook : nk::ProfHook {
  const char* name;
  ProfScope* cur = nullptr;
  explicit ScopeHook(const char* nm) : name(nm) {}
  void begin(hipStream_t s) override {
    delete cur;
    cur = new ProfScope(name, s);
  }
  void end(hipStream_t) override {
    delete cur;
    cur = nullptr;
  }
  ~ScopeHook() override { delete cur; }
};

}  // namespace

extern "C" {

const char* nk_last_error(void) { return g_err.c_str(); }

int nk_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = on != 0;
  return NK_OK;
}

int nk_profile_read(nk_profile_entry* out, int max_entries, int reset) {
  std::vector<ProfRec> pend;
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    pend.swap(g_prof_pending);
  }
  int rc = NK_OK;
  std::map<std::string, std::pair<int64_t, double>> add;
  for (auto& r : pend) {
    float ms = 0.f;
    if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
      rc = fail(NK_EHIP, "profile event: %s", hipGetErrorString(hipGetLastError()));
    hipEventDestroy(r.start);
    hipEventDestroy(r.stop);
    auto& e = add[r.name];
    e.first += 1;
    e.second += ms;
  }
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto& kv : add) {
    auto& e = g_prof_done[kv.first];
    e.first += kv.second.first;
    e.second += kv.second.second;
  }
  if (rc) return rc;
  int n = 0;
  for (auto& kv : g_prof_done) {
    if (out && n < max_entries) {
      memset(&out[n], 0, sizeof out[n]);
      strncpy(out[n].name, kv.first.c_str(), sizeof out[n].name - 1);
      out[n].launches = kv.second.first;
      out[n].total_ms = kv.second.second;
    }
    ++n;
  }
  if (reset) g_prof_done.clear();
  return n;
}

const char* nk_version(void) { return "libnk 0.1 (gfx950)"; }

size_t nk_workspace_size(int op, const void* cfg, int64_t n1, int64_t n2) {
  if (n1 < 0 || n2 < 0) return 0;
  switch (op) {
    case NK_OP_FC: {
      Bump b;
      b.take(sizeof(float) * (size_t)n1);
      b.take(sizeof(float) * (size_t)n2);
      return b.off + 256;
    }
    case NK_OP_MYRTLE: {
      NetDesc net;
      if (check_myrtle(static_cast<const nk_myrtle_cfg*>(cfg), &net, true)) return 0;
      const int64_t np = std::max<int64_t>(1, nk::pair_count(n1, n2, 0));
      return plan_myrtle(net, n1, n2, false, std::min(np, net.hw > 32 ? kDefaultChunk64 : kDefaultChunk)).total +
             256 * NK_MAX_STAGES;
    }
    case NK_OP_MYRTLE_BWD: {
      NetDesc net;
      if (check_myrtle(static_cast<const nk_myrtle_cfg*>(cfg), &net)) return 0;
      const int64_t np = std::max<int64_t>(1, nk::pair_count(n1, n2, 0));
      return plan_bwd(net, n1, n2, false, std::min(np, kDefaultChunk)).total + 512 * NK_MAX_STAGES;
    }
    case NK_OP_KRR:
      return krr_plan(n1, n2).total;
    case NK_OP_MYRTLE_NTK: {
      NetDesc net;
      if (check_myrtle(static_cast<const nk_myrtle_cfg*>(cfg), &net)) return 0;
      const int64_t np = std::max<int64_t>(1, nk::pair_count(n1, n2, 0));
      return plan_ntk(net, n1, n2, false, std::min(np, kDefaultChunk)).total + 256 * NK_MAX_STAGES;
    }
    case NK_OP_MYRTLE_BATCHED: {
      NetDesc net;
      if (check_myrtle(static_cast<const nk_myrtle_cfg*>(cfg), &net)) return 0;
      return plan_batched(net, n1, std::max<int64_t>(n2, 1), kDefaultChunk).total + 256 * NK_MAX_STAGES;
    }
    case NK_OP_PCG: {
      const nk_pcg_cfg* c = static_cast<const nk_pcg_cfg*>(cfg);
      if (!c || n1 <= 0 || c->rank < 0) return 0;
      return pcg_plan(n1, (int)std::min<int64_t>(c->rank, n1), 1).total;
    }
    case NK_OP_PIVOTED_CHOL:
      if (n1 <= 0) return 0;
      return pcg_plan(n1, (int)std::min<int64_t>(n2, n1), 0).total;
    case NK_OP_GRAM_MATVEC:
      if (n1 <= 0) return 0;
      return pcg_plan(n1, 0, 2).total;
    case NK_OP_APPROX: {
      const nk_approx_dims* d = static_cast<const nk_approx_dims*>(cfg);
      if (!d || d->n <= 0 || d->m <= 0 || d->c <= 0 || d->r < 0 || d->max_block < 0) return 0;
      return approx_plan(*d).total;
    }
    case NK_OP_CV: {
      const nk_cv_cfg* c = static_cast<const nk_cv_cfg*>(cfg);
      if (check_cv(c) || n1 <= 0 || n2 < 0) return 0;
      return cv_plan(c, n1, n2, n2 == 0).total;
    }
    default:
      return 0;
  }
}

int nk_fc_nngp(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_fc_cfg* cfg, float* K,
               int64_t ldk, void* ws, size_t ws_bytes, void* stream) {
  if (!cfg || !x1 || !x2 || !K) return fail(NK_EINVAL, "null pointer argument");
  if (n1 <= 0 || n2 <= 0 || cfg->d <= 0 || cfg->depth < 0) return fail(NK_EINVAL, "sizes must be positive");
  if (ldk < n2) return fail(NK_EINVAL, "ldk < n2");
  if (!(cfg->sigma_w2 > 0.f) || !(cfg->sigma_b2 >= 0.f)) return fail(NK_EINVAL, "need sigma_w2 > 0, sigma_b2 >= 0");
  const size_t need = nk_workspace_size(NK_OP_FC, cfg, n1, n2);
  if (!ws || ws_bytes < need) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", need);
  Bump b;
  float* d1 = at<float>(ws, b.take(sizeof(float) * n1));
  float* d2 = at<float>(ws, b.take(sizeof(float) * n2));
  nk::FcArgs a;
  a.x1 = x1;
  a.x2 = x2;
  a.n1 = n1;
  a.n2 = n2;
  a.d = cfg->d;
  a.depth = cfg->depth;
  a.sw2 = cfg->sigma_w2;
  a.sb2 = cfg->sigma_b2;
  a.d1 = d1;
  a.d2 = d2;
  a.K = K;
  a.ldk = ldk;
  a.sym = (x1 == x2 && n1 == n2) ? 1 : 0;
  ProfScope ps("fc_nngp", (hipStream_t)stream);
  if (nk::launch_fc(a, d1, d2, (hipStream_t)stream)) return hip_fail("fc kernel");
  return ok();
}

int nk_fc_nngp_static(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_fc_cfg* cfg, float* K,
                      int64_t ldk, void* stream) {
  if (!cfg || !x1 || !x2 || !K) return fail(NK_EINVAL, "null pointer argument");
  if (n1 <= 0 || n2 <= 0 || cfg->d <= 0 || cfg->depth < 0) return fail(NK_EINVAL, "sizes must be positive");
  if (ldk < n2) return fail(NK_EINVAL, "ldk < n2");
  if (!(cfg->sigma_w2 > 0.f) || !(cfg->sigma_b2 >= 0.f)) return fail(NK_EINVAL, "need sigma_w2 > 0, sigma_b2 >= 0");
  if (n1 + n2 > kFcStaticFloats)
    return fail(NK_EINVAL, "n1 + n2 = %lld exceeds the static scratch (%lld rows)", (long long)(n1 + n2),
                (long long)kFcStaticFloats);
  float* d = nullptr;
  int rc = fc_static_scratch(&d);
  if (rc) return rc;
  nk::FcArgs a;
  a.x1 = x1;
  a.x2 = x2;
  a.n1 = n1;
  a.n2 = n2;
  a.d = cfg->d;
  a.depth = cfg->depth;
  a.sw2 = cfg->sigma_w2;
  a.sb2 = cfg->sigma_b2;
  a.d1 = d;
  a.d2 = d + n1;
  a.K = K;
  a.ldk = ldk;
  a.sym = (x1 == x2 && n1 == n2) ? 1 : 0;
  if (nk::launch_fc(a, d, d + n1, (hipStream_t)stream)) return hip_fail("fc kernel");
  return ok();
}

int nk_myrtle_nngp(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_myrtle_cfg* cfg, float* K,
                   int64_t ldk, void* ws, size_t ws_bytes, void* stream) {
  NetDesc net;
  int rc = check_myrtle(cfg, &net, true);
  if (rc) return rc;
  if (!x1 || !x2 || !K) return fail(NK_EINVAL, "null pointer argument");
  if (n1 <= 0 || n2 <= 0) return fail(NK_EINVAL, "n1 and n2 must be positive");
  if (ldk < n2) return fail(NK_EINVAL, "ldk < n2");
  if (!ws) return fail(NK_EINVAL, "workspace is NULL");
  const bool sym = (x1 == x2) && (n1 == n2);
  const int64_t npairs = nk::pair_count(n1, n2, sym);
  int64_t chunk = max_chunk(net, n1, n2, sym, ws_bytes, npairs);
  if (chunk < 1) {
    return fail(NK_EINVAL, "workspace too small (need at least %zu bytes)",
                plan_myrtle(net, n1, n2, sym, 1).total + 256 * NK_MAX_STAGES);
  }
  // Passes are not lengthened beyond the default by a larger workspace: the
  // default fills whole rounds of resident workgroups, an arbitrary length
  // leaves a partly filled last round.  The 64x64 first stage runs one pair
  // per workgroup and one workgroup per CU: its passes are also rounded down
  // to a multiple of the CU count.
  chunk = std::min(chunk, net.hw > 32 ? kDefaultChunk64 : kDefaultChunk);
  if (net.hw > 32) {
    const int cus = cu_count();
    if (cus > 0 && chunk > cus) chunk -= chunk % cus;
  }
  const MyrtlePlan p = plan_myrtle(net, n1, n2, sym, chunk);
  hipStream_t s = (hipStream_t)stream;
  float2* tab1 = at<float2>(ws, p.tab1);
  float2* tab2 = at<float2>(ws, p.tab2);
  double* scratch = at<double>(ws, p.scratch);
  {
    ProfScope ps("myrtle_prepare", s);
    if (nk::launch_prepare(x1, n1, net, tab1, scratch, kPrepBlocks, s)) return hip_fail("prepare kernel");
    if (!sym && nk::launch_prepare(x2, n2, net, tab2, scratch, kPrepBlocks, s)) return hip_fail("prepare kernel");
  }
  float* bufs[NK_MAX_STAGES] = {nullptr, nullptr, nullptr, nullptr};
  for (int st = 1; st < net.S; ++st) bufs[st] = at<float>(ws, p.buf[st]);
  rc = run_myrtle_pairs(net, x1, n1, x2, n2, sym, tab1, tab2, K, ldk, bufs, chunk, s);
  if (rc) return rc;
  return ok();
}

int nk_myrtle_ntk(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_myrtle_cfg* cfg, float* K_ntk,
                  float* K_nngp, int64_t ldk, void* ws, size_t ws_bytes, void* stream) {
  NetDesc net;
  int rc = check_myrtle(cfg, &net);
  if (rc) return rc;
  if (!x1 || !x2 || !K_ntk) return fail(NK_EINVAL, "null pointer argument");
  if (n1 <= 0 || n2 <= 0) return fail(NK_EINVAL, "n1 and n2 must be positive");
  if (ldk < n2) return fail(NK_EINVAL, "ldk < n2");
  if (!ws) return fail(NK_EINVAL, "workspace is NULL");
  for (int st = 0; st < net.S; ++st)
    if (nk::stage_ntk_lds_bytes(net.hw >> st, net.depth[st], st + 1 < net.S, st == 0) > kLdsDynamicMax)
      return fail(NK_EUNSUPPORTED, "tangent-kernel stage %d needs more than 160 KiB of LDS", st);
  const bool sym = (x1 == x2) && (n1 == n2);
  const int64_t npairs = nk::pair_count(n1, n2, sym);
  int64_t chunk = max_chunk_ntk(net, n1, n2, sym, ws_bytes, npairs);
  if (chunk < 1)
    return fail(NK_EINVAL, "workspace too small (need at least %zu bytes)",
                plan_ntk(net, n1, n2, sym, 1).total + 256 * NK_MAX_STAGES);
  chunk = std::min(chunk, kDefaultChunk);  // whole rounds of workgroups, as for the NNGP
  const MyrtlePlan p = plan_ntk(net, n1, n2, sym, chunk);
  hipStream_t s = (hipStream_t)stream;
  float2* tab1 = at<float2>(ws, p.tab1);
  float2* tab2 = at<float2>(ws, p.tab2);
  double* scratch = at<double>(ws, p.scratch);
  {
    ProfScope ps("myrtle_prepare", s);
    if (nk::launch_prepare(x1, n1, net, tab1, scratch, kPrepBlocks, s)) return hip_fail("prepare kernel");
    if (!sym && nk::launch_prepare(x2, n2, net, tab2, scratch, kPrepBlocks, s)) return hip_fail("prepare kernel");
  }
  float* bufA[NK_MAX_STAGES] = {nullptr, nullptr, nullptr, nullptr};
  float* bufC[NK_MAX_STAGES] = {nullptr, nullptr, nullptr, nullptr};
  for (int st = 1; st < net.S; ++st) {
    const size_t n = (size_t)(net.hw >> st);
    bufA[st] = at<float>(ws, p.buf[st]);
    bufC[st] = bufA[st] + n * n * n * n * (size_t)chunk;
  }
  for (int64_t p0 = 0; p0 < npairs; p0 += chunk) {
    const int64_t np = std::min(chunk, npairs - p0);
    for (int st = 0; st < net.S; ++st) {
      nk::StageArgs a;
      memset(&a, 0, sizeof a);
      a.n1 = n1; a.n2 = n2; a.sym = sym ? 1 : 0; a.T = kPairTile; a.p0 = p0; a.np = np;
      a.x1 = x1; a.x2 = x2; a.tab1 = tab1; a.tab2 = tab2;
      a.tablen = nk::table_len(net); a.taboff = nk::table_off(net, st);
      a.C = net.C; a.D = net.depth[st]; a.sb2 = net.sb2; a.seed_scale = net.sw2 / 9.0f / (float)net.C;
      a.img_floats = (int64_t)net.hw * net.hw * net.C;
      const bool pool = st + 1 < net.S;
      a.in = st > 0 ? bufA[st] : nullptr;
      a.in2 = st > 0 ? bufC[st] : nullptr;
      a.out = pool ? bufA[st + 1] : nullptr;
      a.out2 = pool ? bufC[st + 1] : nullptr;
      a.K = K_nngp;
      a.K2 = K_ntk;
      a.ldk = ldk;
      for (int l = 0; l < net.depth[st]; ++l) a.kh[l] = (float)(0.5 * layer_kappa(net, st, l));
      char nm[48];
      snprintf(nm, sizeof nm, "myrtle_ntk_stage%d_n%d", st + 1, net.hw >> st);
      ProfScope ps(nm, s);
      if (nk::launch_stage_ntk(net.hw >> st, a, st == 0, pool, net.sb2 != 0.f, s))
        return hip_fail("tangent-kernel stage kernel");
    }
  }
  return ok();
}

int nk_myrtle_nngp_backward(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_myrtle_cfg* cfg,
                            const float* dK, int64_t lddk, float* dx1, float* dx2, float* dsigma, void* ws,
                            size_t ws_bytes, void* stream) {
  NetDesc net;
  int rc = check_myrtle(cfg, &net);
  if (rc) return rc;
  if (!x1 || !x2 || !dK) return fail(NK_EINVAL, "null pointer argument");
  if (n1 <= 0 || n2 <= 0) return fail(NK_EINVAL, "n1 and n2 must be positive");
  if (lddk < n2) return fail(NK_EINVAL, "lddk < n2");
  if (!ws) return fail(NK_EINVAL, "workspace is NULL");
  const bool sym = (x1 == x2) && (n1 == n2);
  if (sym && dx2 && dx2 != dx1) return fail(NK_EINVAL, "symmetric block: dx2 must be NULL or equal to dx1");
  if ((rc = check_bwd_lds(net))) return rc;
  const int64_t npairs = nk::pair_count(n1, n2, sym);
  const int64_t chunk = max_chunk_bwd(net, n1, n2, sym, ws_bytes, npairs);
  if (chunk < 1)
    return fail(NK_EINVAL, "workspace too small (need at least %zu bytes)",
                plan_bwd(net, n1, n2, sym, 1).total + 512 * NK_MAX_STAGES);
  const BwdPlan p = plan_bwd(net, n1, n2, sym, chunk);
  hipStream_t s = (hipStream_t)stream;
  float2* tab1 = at<float2>(ws, p.tab1);
  float2* tab2 = at<float2>(ws, p.tab2);
  double* W1 = at<double>(ws, p.W1);
  double* W2 = at<double>(ws, p.W2);
  double* xb1 = at<double>(ws, p.xb1);
  double* xb2 = at<double>(ws, p.xb2);
  double* sums = at<double>(ws, p.sums);
  const int tl = nk::table_len(net);
  const int64_t img = (int64_t)net.hw * net.hw * net.C;
  {
    ProfScope ps("myrtle_prepare", s);
    if (nk::launch_prepare(x1, n1, net, tab1, at<double>(ws, p.scratch), kPrepBlocks, s))
      return hip_fail("prepare kernel");
    if (!sym && nk::launch_prepare(x2, n2, net, tab2, at<double>(ws, p.scratch), kPrepBlocks, s))
      return hip_fail("prepare kernel");
  }
  if (nk::launch_zero_f64(W1, n1 * tl, s) || nk::launch_zero_f64(xb1, n1 * img, s) || nk::launch_zero_f64(sums, 4, s))
    return hip_fail("zero");
  if (!sym && (nk::launch_zero_f64(W2, n2 * tl, s) || nk::launch_zero_f64(xb2, n2 * img, s))) return hip_fail("zero");
  float* bufs[NK_MAX_STAGES] = {nullptr, nullptr, nullptr, nullptr};
  float* gbufs[NK_MAX_STAGES] = {nullptr, nullptr, nullptr, nullptr};
  for (int st = 1; st < net.S; ++st) {
    bufs[st] = at<float>(ws, p.buf[st]);
    gbufs[st] = at<float>(ws, p.gbuf[st]);
  }
  // x2's seed gradients only when asked for (a symmetric block's two sides
  // are the same images)
  if ((rc = bwd_block(net, x1, n1, x2, n2, sym, dK, lddk, tab1, tab2, W1, W2, xb1, xb2, sums, bufs, gbufs, chunk, s,
                      sym || dx2 != nullptr)))
    return rc;
  {
    ProfScope ps("myrtle_self_bwd", s);
    double* bs = at<double>(ws, p.bscratch);
    if (nk::launch_prepare_bwd(x1, n1, net, W1, tl, xb1, sums, bs, kPrepBwdBlocks, s)) return hip_fail("self adjoint");
    if (!sym && nk::launch_prepare_bwd(x2, n2, net, W2, tl, xb2, sums, bs, kPrepBwdBlocks, s))
      return hip_fail("self adjoint");
  }
  if (dx1 && nk::launch_cast_grad(xb1, dx1, n1 * img, s)) return hip_fail("cast");
  if (!sym && dx2 && nk::launch_cast_grad(xb2, dx2, n2 * img, s)) return hip_fail("cast");
  if (dsigma && nk::launch_finish_sigma(sums, (double)net.sw2, dsigma, s)) return hip_fail("sigma");
  return ok();
}

int nk_krr_predict(const float* K_train, int64_t n, const float* K_test, int64_t m, const float* Y, int64_t c,
                   double ridge_rel, float* pred, void* ws, size_t ws_bytes, void* stream) {
  if (!K_train || !Y || (m > 0 && (!K_test || !pred))) return fail(NK_EINVAL, "null pointer argument");
  if (n <= 0 || m < 0 || c <= 0) return fail(NK_EINVAL, "need n > 0, m >= 0, c > 0");
  if (!(ridge_rel >= 0.0)) return fail(NK_EINVAL, "ridge_rel must be >= 0");
  if (n > 16384) return fail(NK_EUNSUPPORTED, "n > 16384");
  const size_t need = nk_workspace_size(NK_OP_KRR, nullptr, n, std::max(m, c));
  if (!ws || ws_bytes < need) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", need);
  const KrrPlan kp = krr_plan(n, std::max(m, c));
  double* A = at<double>(ws, kp.A);
  double* mean = at<double>(ws, kp.mean);
  int* info = at<int>(ws, kp.info);
  double* X = at<double>(ws, kp.X);
  hipStream_t s = (hipStream_t)stream;
  if (nk::launch_krr_build(K_train, n, ridge_rel, 0.0, mean, A, info, s)) return hip_fail("krr build");
  if (nk::launch_cholesky(A, n, info, s)) return hip_fail("cholesky");
  if (nk::launch_chol_solve(A, n, Y, nullptr, c, X, s)) return hip_fail("cholesky solve");
  if (m > 0 && nk::launch_krr_matmul(K_test, m, n, n, X, c, pred, s)) return hip_fail("krr predict");
  int h_info = 0;
  if (hipMemcpyAsync(&h_info, info, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return hip_fail("krr");
  if (hipStreamSynchronize(s) != hipSuccess) return hip_fail("krr sync");
  if (h_info) return fail(NK_ENOTPD, "K_train + lambda I is not positive definite");
  return ok();
}

int nk_krr_mse_backward(const float* K_ss, int64_t n, const float* K_ts, int64_t m, const float* Y_s,
                        const float* Y_t, int64_t c, double ridge, int ridge_is_relative, float* dK_ss,
                        float* dK_ts, double* loss, double* lambda_used, void* ws, size_t ws_bytes, void* stream) {
  if (!K_ss || !K_ts || !Y_s || !Y_t || !dK_ss || !dK_ts || !loss) return fail(NK_EINVAL, "null pointer argument");
  if (n <= 0 || m <= 0 || c <= 0) return fail(NK_EINVAL, "need n, m, c > 0");
  if (!(ridge >= 0.0)) return fail(NK_EINVAL, "ridge must be >= 0");
  if (n > 16384) return fail(NK_EUNSUPPORTED, "n > 16384");
  const KrrPlan kp = krr_plan(n, std::max(m, c));
  if (!ws || ws_bytes < kp.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", kp.total);
  double* A = at<double>(ws, kp.A);
  double* mean = at<double>(ws, kp.mean);
  int* info = at<int>(ws, kp.info);
  double* X = at<double>(ws, kp.X);
  double* B = at<double>(ws, kp.B);
  double* Z = at<double>(ws, kp.Z);
  double* G = at<double>(ws, kp.G);
  double* sq = at<double>(ws, kp.sq);
  double* dloss = at<double>(ws, kp.loss);
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps("krr_mse_backward", s);
  if (nk::launch_krr_build(K_ss, n, ridge_is_relative ? ridge : -1.0, ridge, mean, A, info, s))
    return hip_fail("krr build");
  if (nk::launch_cholesky(A, n, info, s)) return hip_fail("cholesky");
  if (nk::launch_chol_solve(A, n, Y_s, nullptr, c, X, s)) return hip_fail("cholesky solve");
  if (nk::launch_krr_mse_bwd(K_ts, m, n, X, c, Y_t, G, sq, dloss, B, s)) return hip_fail("krr cotangent");
  if (nk::launch_chol_solve(A, n, nullptr, B, c, Z, s)) return hip_fail("cholesky solve");
  if (nk::launch_krr_outer(G, m, X, n, c, 1.0, dK_ts, s)) return hip_fail("krr outer");
  if (nk::launch_krr_outer(Z, n, X, n, c, -1.0, dK_ss, s)) return hip_fail("krr outer");
  int h_info = 0;
  if (hipMemcpyAsync(&h_info, info, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return hip_fail("krr");
  double h_mean = 0.0;
  if (hipMemcpyAsync(loss, dloss, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return hip_fail("krr");
  if (ridge_is_relative && hipMemcpyAsync(&h_mean, mean, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return hip_fail("krr");
  if (hipStreamSynchronize(s) != hipSuccess) return hip_fail("krr sync");
  if (lambda_used) *lambda_used = ridge_is_relative ? ridge * h_mean : ridge;
  if (h_info) return fail(NK_ENOTPD, "K_ss + lambda I is not positive definite");
  return ok();
}



size_t nk_krr_mse_grad_workspace(const nk_myrtle_cfg* cfg, int64_t n, int64_t m, int64_t c) {
  NetDesc net;
  if (n <= 0 || m <= 0 || c <= 0 || check_myrtle(cfg, &net)) return 0;
  const int64_t np = std::max(nk::pair_count(n, n, 1), nk::pair_count(m, n, 0));
  return plan_krr_grad(net, n, m, c, std::min(np, kDefaultChunk)).total;
}

size_t nk_krr_mse_grad_workspace_keep(const nk_myrtle_cfg* cfg, int64_t n, int64_t m, int64_t c) {
  NetDesc net;
  if (n <= 0 || m <= 0 || c <= 0 || check_myrtle(cfg, &net)) return 0;
  const int64_t np = std::max(nk::pair_count(n, n, 1), nk::pair_count(m, n, 0));
  return plan_krr_grad(net, n, m, c, std::min(np, kDefaultChunk), true).total;
}

// keep: the first-stage outputs of both blocks stay in the workspace between
// the passes (nk_krr_mse_grad_kept); otherwise the adjoint pass re-runs the
// first stage per chunk.
static int krr_mse_grad_impl(const float* x_s, int64_t n, const float* x_t, int64_t m, const float* Y_s,
                             const float* Y_t, int64_t c, const nk_myrtle_cfg* cfg, double ridge,
                             int ridge_is_relative, float* dx_s, float* dsigma, double* loss, double* lambda_used,
                             void* ws, size_t ws_bytes, void* stream, bool keep) {
  NetDesc net;
  int rc = check_myrtle(cfg, &net);
  if (rc) return rc;
  if (!x_s || !x_t || !Y_s || !Y_t || !loss) return fail(NK_EINVAL, "null pointer argument");
  if (n <= 0 || m <= 0 || c <= 0) return fail(NK_EINVAL, "need n, m, c > 0");
  if (x_s == x_t) return fail(NK_EINVAL, "x_s and x_t must be different arrays");
  if (!(ridge >= 0.0)) return fail(NK_EINVAL, "ridge must be >= 0");
  if (n > 16384) return fail(NK_EUNSUPPORTED, "n > 16384");
  if ((rc = check_bwd_lds(net))) return rc;
  if (!ws) return fail(NK_EINVAL, "workspace is NULL");
  const int64_t np = std::max(nk::pair_count(n, n, 1), nk::pair_count(m, n, 0));
  int64_t chunk = std::min(np, kDefaultChunk);
  KrrGradPlan p = plan_krr_grad(net, n, m, c, chunk, keep);
  if (p.keep && ws_bytes < p.total)
    return fail(NK_EINVAL, "workspace too small to keep the first-stage outputs (need %zu bytes)", p.total);
  if (ws_bytes < p.total) {
    // fewer pairs per pass if the workspace is short of the default
    const size_t fixed = plan_krr_grad(net, n, m, c, 0).total;
    size_t per = 0;
    for (int s = 1; s < net.S; ++s) {
      const size_t q = (size_t)(net.hw >> s);
      per += 2 * q * q * q * q * sizeof(float);
    }
    if (ws_bytes < fixed + 256 * 2 * NK_MAX_STAGES + per)
      return fail(NK_EINVAL, "workspace too small (need %zu bytes)", nk_krr_mse_grad_workspace(cfg, n, m, c));
    chunk = std::min<int64_t>(chunk, (int64_t)((ws_bytes - fixed - 256 * 2 * NK_MAX_STAGES) / per));
    p = plan_krr_grad(net, n, m, c, chunk);
  }
  hipStream_t s = (hipStream_t)stream;
  float* kss = at<float>(ws, p.kss);
  float* kts = at<float>(ws, p.kts);
  float* dss = at<float>(ws, p.dss);
  float* dts = at<float>(ws, p.dts);
  float2* tab_s = at<float2>(ws, p.tab_s);
  float2* tab_t = at<float2>(ws, p.tab_t);
  double* W_s = at<double>(ws, p.W_s);
  double* W_t = at<double>(ws, p.W_t);
  double* xb_s = at<double>(ws, p.xb_s);
  double* xb_t = at<double>(ws, p.xb_t);
  double* sums = at<double>(ws, p.sums);
  const int tl = nk::table_len(net);
  const int64_t img = (int64_t)net.hw * net.hw * net.C;
  float* bufs[NK_MAX_STAGES] = {nullptr, nullptr, nullptr, nullptr};
  float* gbufs[NK_MAX_STAGES] = {nullptr, nullptr, nullptr, nullptr};
  for (int st = 1; st < net.S; ++st) {
    bufs[st] = p.buf[st] ? at<float>(ws, p.buf[st]) : nullptr;
    gbufs[st] = at<float>(ws, p.gbuf[st]);
  }
  // kept first-stage outputs: the symmetric block's pairs, then the cross
  // block's as (support, targets), the order its adjoint runs in
  float* keep_ss = p.keep ? at<float>(ws, p.keep1) : nullptr;
  float* keep_st = p.keep ? keep_ss + nk::pair_count(n, n, 1) * stage1_out_floats(net) : nullptr;
  {
    ProfScope ps("myrtle_prepare", s);
    if (nk::launch_prepare(x_s, n, net, tab_s, at<double>(ws, p.scratch), kPrepBlocks, s) ||
        nk::launch_prepare(x_t, m, net, tab_t, at<double>(ws, p.scratch), kPrepBlocks, s))
      return hip_fail("prepare kernel");
  }
  // forward: K_ss (symmetric) and K_ts
  if ((rc = run_myrtle_pairs(net, x_s, n, x_s, n, true, tab_s, tab_s, kss, n, bufs, chunk, s, keep_ss))) return rc;
  if (p.keep) {
    // the cross block as (support, targets), its Gram block (n x m) in the
    // cotangent's place until it is transposed into K_ts
    if ((rc = run_myrtle_pairs(net, x_s, n, x_t, m, false, tab_s, tab_t, dts, m, bufs, chunk, s, keep_st))) return rc;
    if (nk::launch_transpose_f32(dts, n, m, kts, s)) return hip_fail("transpose");
  } else if ((rc = run_myrtle_pairs(net, x_t, m, x_s, n, false, tab_t, tab_s, kts, n, bufs, chunk, s))) {
    return rc;
  }
  // ridge solve, loss and the cotangents of both blocks (synchronises)
  if ((rc = nk_krr_mse_backward(kss, n, kts, m, Y_s, Y_t, c, ridge, ridge_is_relative, dss, dts, loss, lambda_used,
                                at<char>(ws, p.krr), p.krr_bytes, stream)))
    return rc;
  // both adjoints into one set of sums for the support images (x_s is x1 of
  // the symmetric block and x2 of the cross block)
  if (nk::launch_zero_f64(W_s, n * tl, s) || nk::launch_zero_f64(xb_s, n * img, s) ||
      nk::launch_zero_f64(W_t, m * tl, s) || nk::launch_zero_f64(xb_t, m * img, s) || nk::launch_zero_f64(sums, 4, s))
    return hip_fail("zero");
  if ((rc = bwd_block(net, x_s, n, x_s, n, true, dss, n, tab_s, tab_s, W_s, W_s, xb_s, xb_s, sums, bufs, gbufs, chunk,
                      s, true, false, keep_ss)))
    return rc;
  // the cross block as (support, targets) with its cotangent read transposed:
  // the support images' seed gradients are then the fixed-frame (i-side)
  // sums, and the targets' (not wanted) are not accumulated at 32x32
  if ((rc = bwd_block(net, x_s, n, x_t, m, false, dts, n, tab_s, tab_t, W_s, W_t, xb_s, xb_t, sums, bufs, gbufs, chunk,
                      s, /*xj=*/false, /*dk_t=*/true, keep_st)))
    return rc;
  {
    // the self-chain reverse is linear in W: once per image set on the summed
    // sums.  The targets' chain is run too: their variance maps depend on
    // both sigmas (their image gradient is not returned).
    ProfScope ps("myrtle_self_bwd", s);
    if (nk::launch_prepare_bwd(x_s, n, net, W_s, tl, xb_s, sums, at<double>(ws, p.bscratch), kPrepBwdBlocks, s) ||
        nk::launch_prepare_bwd(x_t, m, net, W_t, tl, xb_t, sums, at<double>(ws, p.bscratch), kPrepBwdBlocks, s))
      return hip_fail("self adjoint");
  }
  if (dx_s && nk::launch_cast_grad(xb_s, dx_s, n * img, s)) return hip_fail("cast");
  if (dsigma && nk::launch_finish_sigma(sums, (double)net.sw2, dsigma, s)) return hip_fail("sigma");
  return ok();
}

int nk_krr_mse_grad(const float* x_s, int64_t n, const float* x_t, int64_t m, const float* Y_s, const float* Y_t,
                    int64_t c, const nk_myrtle_cfg* cfg, double ridge, int ridge_is_relative, float* dx_s,
                    float* dsigma, double* loss, double* lambda_used, void* ws, size_t ws_bytes, void* stream) {
  return krr_mse_grad_impl(x_s, n, x_t, m, Y_s, Y_t, c, cfg, ridge, ridge_is_relative, dx_s, dsigma, loss,
                           lambda_used, ws, ws_bytes, stream, false);
}

int nk_krr_mse_grad_kept(const float* x_s, int64_t n, const float* x_t, int64_t m, const float* Y_s,
                         const float* Y_t, int64_t c, const nk_myrtle_cfg* cfg, double ridge, int ridge_is_relative,
                         float* dx_s, float* dsigma, double* loss, double* lambda_used, void* ws, size_t ws_bytes,
                         void* stream) {
  return krr_mse_grad_impl(x_s, n, x_t, m, Y_s, Y_t, c, cfg, ridge, ridge_is_relative, dx_s, dsigma, loss,
                           lambda_used, ws, ws_bytes, stream, true);
}

int nk_krr_nystrom(const float* K_nr, int64_t n, int64_t r, int64_t ld_nr, const float* K_rr, int64_t ld_rr,
                   const float* K_mn, int64_t m, int64_t ld_mn, const float* Y, int64_t c, double lambda,
                   double jitter, float* pred, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_approx_common(n, m, c, lambda, jitter, Y, pred);
  if (rc) return rc;
  if (!K_nr || !K_rr || !K_mn) return fail(NK_EINVAL, "null pointer argument");
  if (r <= 0 || r > n || ld_nr < r || ld_rr < r || ld_mn < n) return fail(NK_EINVAL, "bad r or leading dimension");
  if (r > kApproxMaxSolve) return fail(NK_EUNSUPPORTED, "r > %lld", (long long)kApproxMaxSolve);
  const nk_approx_dims d{n, r, m, c, 0};
  const ApproxPlan ap = approx_plan(d);
  if (!ws || ws_bytes < ap.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", ap.total);
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps("krr_nystrom", s);
  double* alpha = at<double>(ws, ap.alpha);
  double* P = at<double>(ws, ap.P);
  if (approx_low_rank_v(K_nr, n, r, ld_nr, K_rr, ld_rr, Y, c, lambda, jitter, ws, ap, s) ||
      nk::dn_gemm_fd(K_nr, ld_nr, false, at<double>(ws, ap.v), c, alpha, c, n, c, r, 1.0, 0.0, true, s) ||
      nk::dn_residual_scale(Y, c, n, c, 1.0 / lambda, alpha, s) ||
      nk::dn_gemm_fd(K_mn, ld_mn, false, alpha, c, P, c, m, c, n, 1.0, 0.0, false, s) ||
      nk::dn_cast(P, m, c, pred, c, s))
    return hip_fail("nystrom");
  return approx_finish(s, at<int>(ws, ap.info), "nystrom");
}

int nk_krr_sor(const float* K_nr, int64_t n, int64_t r, int64_t ld_nr, const float* K_rr, int64_t ld_rr,
               const float* K_mr, int64_t m, int64_t ld_mr, const float* Y, int64_t c, double lambda, double jitter,
               float* pred, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_approx_common(n, m, c, lambda, jitter, Y, pred);
  if (rc) return rc;
  if (!K_nr || !K_rr || !K_mr) return fail(NK_EINVAL, "null pointer argument");
  if (r <= 0 || r > n || ld_nr < r || ld_rr < r || ld_mr < r) return fail(NK_EINVAL, "bad r or leading dimension");
  if (r > kApproxMaxSolve) return fail(NK_EUNSUPPORTED, "r > %lld", (long long)kApproxMaxSolve);
  const nk_approx_dims d{n, r, m, c, 0};
  const ApproxPlan ap = approx_plan(d);
  if (!ws || ws_bytes < ap.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", ap.total);
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps("krr_sor", s);
  double* P = at<double>(ws, ap.P);
  if (approx_low_rank_v(K_nr, n, r, ld_nr, K_rr, ld_rr, Y, c, lambda, jitter, ws, ap, s) ||
      nk::dn_gemm_fd(K_mr, ld_mr, false, at<double>(ws, ap.v), c, P, c, m, c, r, 1.0, 0.0, false, s) ||
      nk::dn_cast(P, m, c, pred, c, s))
    return hip_fail("sor");
  return approx_finish(s, at<int>(ws, ap.info), "sor");
}

int nk_krr_block_diag(int32_t p, const float* const* K_blocks, const int64_t* sizes, const float* K_mn, int64_t m,
                      int64_t ld_mn, const float* Y, int64_t c, double lambda, float* pred, void* ws,
                      size_t ws_bytes, void* stream) {
  int64_t n = 0, maxb = 0;
  int rc = check_blocks(p, K_blocks, sizes, &n, &maxb);
  if (rc) return rc;
  rc = check_approx_common(n, m, c, lambda, 0.0, Y, pred);
  if (rc) return rc;
  if (!K_mn || ld_mn < n) return fail(NK_EINVAL, "K_mn is NULL or ld_mn < n");
  const nk_approx_dims d{n, 0, m, c, maxb};
  const ApproxPlan ap = approx_plan(d);
  if (!ws || ws_bytes < ap.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", ap.total);
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps("krr_block_diag", s);
  double* D = at<double>(ws, ap.D);
  double* alpha = at<double>(ws, ap.alpha);
  double* P = at<double>(ws, ap.P);
  int* info = at<int>(ws, ap.info);
  int64_t off = 0;
  for (int32_t i = 0; i < p; ++i) {
    const int64_t b = sizes[i];
    if (nk::dn_load_shift(K_blocks[i], b, b, lambda, D, i == 0 ? info : nullptr, s) ||
        nk::launch_cholesky(D, b, info, s) ||
        nk::launch_chol_solve(D, b, Y + off * c, nullptr, c, alpha + off * c, s))
      return hip_fail("block diagonal");
    off += b;
  }
  if (nk::dn_gemm_fd(K_mn, ld_mn, false, alpha, c, P, c, m, c, n, 1.0, 0.0, false, s) ||
      nk::dn_cast(P, m, c, pred, c, s))
    return hip_fail("block diagonal");
  return approx_finish(s, info, "block diagonal");
}

int nk_krr_bcm(int32_t p, const float* const* K_blocks, const int64_t* sizes, const float* K_mn, int64_t m,
               int64_t ld_mn, const float* K_mm, int64_t ld_mm, const float* Y, int64_t c, double lambda,
               double jitter, float* pred, void* ws, size_t ws_bytes, void* stream) {
  int64_t n = 0, maxb = 0;
  int rc = check_blocks(p, K_blocks, sizes, &n, &maxb);
  if (rc) return rc;
  rc = check_approx_common(n, m, c, lambda, jitter, Y, pred);
  if (rc) return rc;
  if (!K_mn || ld_mn < n || !K_mm || ld_mm < m) return fail(NK_EINVAL, "bad K_mn or K_mm");
  if (m > kApproxMaxSolve) return fail(NK_EUNSUPPORTED, "m > %lld", (long long)kApproxMaxSolve);
  const nk_approx_dims d{n, 0, m, c, maxb};
  const ApproxPlan ap = approx_plan(d);
  if (!ws || ws_bytes < ap.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", ap.total);
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps("krr_bcm", s);
  double* D = at<double>(ws, ap.D);
  double* RHS = at<double>(ws, ap.rhs2);
  double* Z = at<double>(ws, ap.Z);
  double* mu = at<double>(ws, ap.mu);
  double* S = at<double>(ws, ap.S);
  double* Sinv = at<double>(ws, ap.Sinv);
  double* Kinv = at<double>(ws, ap.Kinv);
  double* I = at<double>(ws, ap.I);
  double* prec = at<double>(ws, ap.prec);
  double* acc = at<double>(ws, ap.acc);
  double* P = at<double>(ws, ap.P);
  int* info = at<int>(ws, ap.info);
  const int64_t w = c + m;
  // prior precision of the test values: (K_mm + jitter I)^{-1}; prec = -(p - 1) of it
  if (nk::dn_identity(I, m, s) || nk::dn_load_shift(K_mm, ld_mm, m, jitter, S, info, s) ||
      nk::launch_cholesky(S, m, info, s) || nk::launch_chol_solve(S, m, nullptr, I, m, Kinv, s) ||
      nk::dn_axpby(prec, Kinv, m * m, 0.0, -(double)(p - 1), s) || nk::launch_zero_f64(acc, m * c, s))
    return hip_fail("bcm");
  int64_t off = 0;
  for (int32_t i = 0; i < p; ++i) {
    const int64_t b = sizes[i];
    const float* kmi = K_mn + off;  // columns off .. off + b of K_mn
    if (nk::dn_load_shift(K_blocks[i], b, b, lambda, D, nullptr, s) || nk::launch_cholesky(D, b, info, s) ||
        nk::dn_copy_f(Y + off * c, c, b, c, false, RHS, w, s) ||
        nk::dn_copy_f(kmi, ld_mn, b, m, true, RHS + c, w, s) ||
        nk::launch_chol_solve(D, b, nullptr, RHS, w, Z, s) ||
        // mu_i = K_mi Z[:, :c];  S_i = K_mm - K_mi Z[:, c:] (a difference of nearly equal terms: compensated)
        nk::dn_gemm_fd(kmi, ld_mn, false, Z, w, mu, c, m, c, b, 1.0, 0.0, false, s) ||
        nk::dn_copy_f(K_mm, ld_mm, m, m, false, S, m, s) ||
        nk::dn_gemm_fd(kmi, ld_mn, false, Z + c, w, S, m, m, m, b, -1.0, 1.0, true, s) ||
        nk::dn_shift(S, m, jitter, nullptr, s) || nk::launch_cholesky(S, m, info, s) ||
        nk::launch_chol_solve(S, m, nullptr, I, m, Sinv, s) || nk::dn_axpby(prec, Sinv, m * m, 1.0, 1.0, s) ||
        nk::dn_gemm_dd(Sinv, m, false, mu, c, acc, c, m, c, m, 1.0, 1.0, false, s))
      return hip_fail("bcm");
    off += b;
  }
  if (nk::launch_cholesky(prec, m, info, s) || nk::launch_chol_solve(prec, m, nullptr, acc, c, P, s) ||
      nk::dn_cast(P, m, c, pred, c, s))
    return hip_fail("bcm");
  return approx_finish(s, info, "bcm");
}

int nk_cv_nngp(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_cv_cfg* cfg, float* K,
               int64_t ldk, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_cv(cfg);
  if (rc) return rc;
  if (!x1 || !x2 || !K) return fail(NK_EINVAL, "null pointer argument");
  if (n1 <= 0 || n2 <= 0) return fail(NK_EINVAL, "n1 and n2 must be positive");
  if (ldk < n2) return fail(NK_EINVAL, "ldk < n2");
  const bool sym = (x1 == x2) && (n1 == n2);
  const CvPlan cp = cv_plan(cfg, n1, n2, sym);
  if (!ws || ws_bytes < cp.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", cp.total);
  hipStream_t s = (hipStream_t)stream;
  const int N = cfg->H;
  float2* t1 = at<float2>(ws, cp.tab1);
  float2* t2 = sym ? t1 : at<float2>(ws, cp.tab2);
  {
    ProfScope ps("cv_prepare", s);
    if (nk::launch_cv_prepare(x1, n1, N, cfg->C, cfg->depth, cfg->sigma_w2, cfg->sigma_b2, t1,
                              at<float>(ws, cp.d1), s))
      return hip_fail("cv prepare");
    if (!sym && nk::launch_cv_prepare(x2, n2, N, cfg->C, cfg->depth, cfg->sigma_w2, cfg->sigma_b2, t2,
                                      at<float>(ws, cp.d2), s))
      return hip_fail("cv prepare");
  }
  const float seed_scale = (float)((double)cfg->sigma_w2 / (9.0 * cfg->C));
  char nm[32];
  snprintf(nm, sizeof nm, "cv_pairs_n%d", N);
  ProfScope ps(nm, s);
  if (nk::launch_cv_pairs(N, x1, x2, n1, n2, sym ? 1 : 0, kPairTile, cfg->C, cfg->depth, t1, t2, K, ldk,
                          cfg->sigma_b2, seed_scale, s))
    return hip_fail("cv pairs");
  return ok();
}

int nk_pivoted_cholesky(const float* K, int64_t n, int64_t ldk, int32_t rank, double pivot_tol, double* L,
                        int32_t* piv, int32_t* rank_used, void* ws, size_t ws_bytes, void* stream) {
  if (!K || (rank > 0 && (!L || !piv))) return fail(NK_EINVAL, "null pointer argument");
  if (n <= 0 || ldk < n) return fail(NK_EINVAL, "need n > 0 and ldk >= n");
  if (rank < 0 || rank > n) return fail(NK_EINVAL, "need 0 <= rank <= n");
  if (rank > kPcgMaxRank) return fail(NK_EUNSUPPORTED, "rank > %d", kPcgMaxRank);
  if (!(pivot_tol >= 0.0)) return fail(NK_EINVAL, "pivot_tol must be >= 0");
  if (rank_used) *rank_used = 0;
  if (rank == 0) return ok();
  const PcgPlan pp = pcg_plan(n, rank, 0);
  if (!ws || ws_bytes < pp.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", pp.total);
  hipStream_t s = (hipStream_t)stream;
  {
    ProfScope ps("pivoted_cholesky", s);
    if (nk::launch_pchol(K, n, ldk, rank, pivot_tol, L, piv, at<double>(ws, pp.d), at<double>(ws, pp.pv),
                         at<int>(ws, pp.pi), at<double>(ws, pp.dpiv), s))
      return hip_fail("pivoted cholesky");
  }
  std::vector<int32_t> hp(rank);
  if (hipMemcpyAsync(hp.data(), piv, sizeof(int32_t) * rank, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return hip_fail("pivoted cholesky");
  int32_t r = 0;
  while (r < rank && hp[r] >= 0) ++r;
  if (rank_used) *rank_used = r;
  return ok();
}

int nk_gram_matvec(const float* K, int64_t n, int64_t ldk, const double* P, int64_t c, double lambda, double* Q,
                   void* ws, size_t ws_bytes, void* stream) {
  if (!K || !P || !Q) return fail(NK_EINVAL, "null pointer argument");
  if (n <= 0 || ldk < n) return fail(NK_EINVAL, "need n > 0 and ldk >= n");
  if (c < 1 || c > kPcgGroup) return fail(NK_EUNSUPPORTED, "need 1 <= c <= %d", kPcgGroup);
  const PcgPlan pp = pcg_plan(n, 0, 2);
  if (!ws || ws_bytes < pp.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", pp.total);
  hipStream_t s = (hipStream_t)stream;
  ScopeHook hook("gram_matvec");
  if (nk::launch_kmv(K, n, ldk, P, (int)c, lambda, at<double>(ws, pp.kpart), Q, at<double>(ws, pp.part1), s,
                     &hook))
    return hip_fail("gram matvec");
  return ok();
}

int nk_krr_pcg(const float* K, int64_t n, int64_t ldk, const double* Y, int64_t c, double ridge,
               int ridge_is_relative, const nk_pcg_cfg* cfg, double* X, int32_t* iters, double* relres,
               nk_pcg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  if (!K || !Y || !X || !cfg) return fail(NK_EINVAL, "null pointer argument");
  if (n <= 0 || ldk < n || c <= 0) return fail(NK_EINVAL, "need n > 0, ldk >= n and c > 0");
  if (cfg->rank < 0 || cfg->max_iter < 1 || !(cfg->tol >= 0.0) || !(cfg->pivot_tol >= 0.0) || !(ridge >= 0.0))
    return fail(NK_EINVAL, "need rank >= 0, max_iter >= 1, tol >= 0, pivot_tol >= 0, ridge >= 0");
  const int rank = (int)std::min<int64_t>(cfg->rank, n);
  if (rank > kPcgMaxRank) return fail(NK_EUNSUPPORTED, "rank > %d", kPcgMaxRank);
  const PcgPlan pp = pcg_plan(n, rank, 1);
  if (!ws || ws_bytes < pp.total) return fail(NK_EINVAL, "workspace too small (need %zu bytes)", pp.total);
  hipStream_t s = (hipStream_t)stream;

  double lam = ridge;
  if (ridge_is_relative) {
    double mean = 0.0;
    if (nk::launch_diag_mean(K, n, ldk, at<double>(ws, pp.mean), s) ||
        hipMemcpyAsync(&mean, at<double>(ws, pp.mean), sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return hip_fail("pcg ridge");
    lam = ridge * mean;
  }
  if (!(lam > 0.0)) return fail(NK_EINVAL, "lambda must be > 0 (got %g)", lam);

  double* L = at<double>(ws, pp.L);
  int r = 0;
  if (rank > 0) {
    int* piv = at<int>(ws, pp.piv);
    {
      ProfScope ps("pivoted_cholesky", s);
      if (nk::launch_pchol(K, n, ldk, rank, cfg->pivot_tol, L, piv, at<double>(ws, pp.d), at<double>(ws, pp.pv),
                           at<int>(ws, pp.pi), at<double>(ws, pp.dpiv), s))
        return hip_fail("pivoted cholesky");
    }
    std::vector<int> hp(rank);
    if (hipMemcpyAsync(hp.data(), piv, sizeof(int) * rank, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return hip_fail("pivoted cholesky");
    while (r < rank && hp[r] >= 0) ++r;
  }
  if (r > 0) {
    int info = 0;
    {
      ProfScope ps("pcg_precond_setup", s);
      if (nk::launch_pc_setup(L, n, r, lam, at<double>(ws, pp.Lr), at<double>(ws, pp.M), at<int>(ws, pp.info), s))
        return hip_fail("preconditioner set-up");
    }
    if (hipMemcpyAsync(&info, at<int>(ws, pp.info), sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return hip_fail("preconditioner set-up");
    if (info) return fail(NK_ENOTPD, "lambda I + L^T L is not positive definite");
  }

  nk::PcgArgs a{};
  a.K = K;
  a.n = n;
  a.ldk = ldk;
  a.Y = Y;
  a.ldy = c;
  a.Xout = X;
  a.ldx = c;
  a.lam = lam;
  a.tol = cfg->tol;
  a.max_iter = cfg->max_iter;
  a.r = r;
  a.U = L;  // L R^{-T}, formed in place by the set-up
  a.Ur = at<double>(ws, pp.Lr);
  a.W = at<double>(ws, pp.W);
  a.wpart = at<double>(ws, pp.wpart);
  a.lt_splits = pp.lt_splits;
  a.R = at<double>(ws, pp.R);
  a.X = at<double>(ws, pp.X);
  a.Z = at<double>(ws, pp.Z);
  a.P = at<double>(ws, pp.P);
  a.Q = at<double>(ws, pp.Q);
  a.kpart = at<double>(ws, pp.kpart);
  a.part1 = at<double>(ws, pp.part1);
  a.part2 = at<double>(ws, pp.part2);
  double* st = at<double>(ws, pp.st);
  a.gamma = st;
  a.beta = st + kPcgGroup;
  a.ynorm = st + 2 * kPcgGroup;
  a.relres = st + 3 * kPcgGroup;
  a.active = reinterpret_cast<int*>(st + 4 * kPcgGroup);
  a.iters = reinterpret_cast<int*>(st + 5 * kPcgGroup);
  a.any = reinterpret_cast<int*>(st + 6 * kPcgGroup);
  int* host_any = nullptr;
  if (hipHostMalloc((void**)&host_any, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return hip_fail("pinned flags");
  struct PinnedFree {
    int* p;
    ~PinnedFree() { (void)hipHostFree(p); }
  } pinned_free{host_any};
  a.host_any = host_any;
  ScopeHook hook("pcg_matvec");
  a.hook = &hook;
  int max_it = 0;
  for (int64_t c0 = 0; c0 < c; c0 += kPcgGroup) {
    const int C = (int)std::min<int64_t>(kPcgGroup, c - c0);
    int rc;
    {
      ProfScope ps("pcg_solve", s);
      rc = nk::launch_pcg_group(a, c0, C, s);
    }
    if (rc) return hip_fail("pcg");
    int hit[kPcgGroup];
    double hrel[kPcgGroup];
    if (hipMemcpyAsync(hit, a.iters, sizeof(int) * C, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hrel, a.relres, sizeof(double) * C, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return hip_fail("pcg");
    for (int j = 0; j < C; ++j) {
      if (iters) iters[c0 + j] = hit[j];
      if (relres) relres[c0 + j] = hrel[j];
      max_it = std::max(max_it, hit[j]);
    }
  }
  if (stats) {
    stats->rank = r;
    stats->iterations = max_it;
    stats->lambda = lam;
  }
  return ok();
}

int nk_myrtle_nngp_batched(const nk_tile* tiles, int32_t ntiles, const nk_myrtle_cfg* cfg, void* ws,
                           size_t ws_bytes, void* stream, int32_t graph) {
  NetDesc net;
  int rc = check_myrtle(cfg, &net);
  if (rc) return rc;
  if (!tiles || ntiles <= 0) return fail(NK_EINVAL, "need at least one tile");
  if (!ws) return fail(NK_EINVAL, "workspace is NULL");
  BatchLayout L;
  if ((rc = batch_layout(tiles, ntiles, net, &L))) return rc;
  const BatchPlan p0 = plan_batched(net, L.rows, ntiles, 0);
  size_t per = 0;
  for (int s = 1; s < net.S; ++s) {
    const size_t n = (size_t)(net.hw >> s);
    per += n * n * n * n * sizeof(float);
  }
  const size_t slack = 256 * NK_MAX_STAGES;
  if (ws_bytes < p0.total + slack + per)
    return fail(NK_EINVAL, "workspace too small (need at least %zu bytes)", p0.total + slack + per);
  const int64_t max_chunk_ws =
      per == 0 ? (int64_t)1 << 40 : (int64_t)((ws_bytes - p0.total - slack) / per);
  hipStream_t s = (hipStream_t)stream;
  const std::string key = net_key(net);

  // tile table -> workspace (every call: the caller may reuse the workspace)
  BatchPlan pl = plan_batched(net, L.rows, ntiles, std::min<int64_t>(max_chunk_ws, 32768));
  nk::TileDesc* ddesc = at<nk::TileDesc>(ws, pl.desc);
  if (nk::launch_put_tiles(L.desc.data(), (int)L.desc.size(), ddesc, s)) return hip_fail("tile table upload");
  float2* tab = at<float2>(ws, pl.tab);
  double* scratch = at<double>(ws, pl.scratch);
  float* bufs[NK_MAX_STAGES] = {nullptr, nullptr, nullptr, nullptr};
  for (int st = 1; st < net.S; ++st) bufs[st] = at<float>(ws, pl.buf[st]);

  auto prepare_all = [&]() -> int {
    int64_t row = 0;
    for (auto& im : L.images) {
      if (nk::launch_prepare(im.first, im.second, net, tab + row * nk::table_len(net), scratch, kPrepBlocks, s))
        return hip_fail("prepare kernel");
      row += im.second;
    }
    return NK_OK;
  };

  // schedule: tuned once per network and process
  BatchParams bp;
  bool have = false;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      bp = it->second.best;
      have = true;
    }
  }
  for (int st = 0; st < net.S; ++st)
    if (nk::prime_stage(net.hw >> st, net.depth[st], st == 0, st + 1 < net.S, net.sb2 != 0.f, net.C, bp.ppm))
      return hip_fail("stage kernel attributes");
  if (!have) {
    {
      ProfScope ps("myrtle_prepare", s);
      if ((rc = prepare_all())) return rc;
    }
    TuneRecord rec;
    if ((rc = autotune(net, ddesc, ntiles, tab, bufs, L.npairs, max_chunk_ws, s, &rec))) return rc;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = rec;
    bp = rec.best;
  }
  bp.chunk = std::min(bp.chunk, max_chunk_ws);
  // (the tuned shape's kernel attributes, before any capture)
  for (int st = 0; st < net.S; ++st)
    if (nk::prime_stage(net.hw >> st, net.depth[st], st == 0, st + 1 < net.S, net.sb2 != 0.f, net.C, bp.ppm))
      return hip_fail("stage kernel attributes");

  if (!graph) {
    {
      ProfScope ps("myrtle_prepare", s);
      if ((rc = prepare_all())) return rc;
    }
    if ((rc = run_batched_stages(net, ddesc, ntiles, tab, bufs, bp, 0, L.npairs, -1, s))) return rc;
    return ok();
  }

  // graph: captured on a library stream the first time this exact pass is
  // seen (tiles, network, workspace, schedule), replayed afterwards
  char sigb[256];
  snprintf(sigb, sizeof sigb, "%s|ws%p:%zu|c%lld T%d p%d m%d|", key.c_str(), ws, ws_bytes, (long long)bp.chunk, bp.T,
           bp.persist, bp.ppm);
  std::string sig(sigb);
  sig.append(reinterpret_cast<const char*>(L.desc.data()), sizeof(nk::TileDesc) * L.desc.size());
  for (auto& im : L.images) sig.append(reinterpret_cast<const char*>(&im), sizeof im);
  std::lock_guard<std::mutex> g(g_graph_mu);
  GraphEntry* hit = nullptr;
  for (auto& e : g_graphs)
    if (e.sig == sig) hit = &e;
  if (!hit) {
    if (!g_cap_stream && hipStreamCreateWithFlags(&g_cap_stream, hipStreamNonBlocking) != hipSuccess)
      return hip_fail("capture stream");
    GraphEntry e;
    e.sig = sig;
    if (hipStreamBeginCapture(g_cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
      return hip_fail("begin capture");
    g_capturing = true;
    hipStream_t keep = s;
    s = g_cap_stream;
    rc = prepare_all();
    if (!rc) rc = run_batched_stages(net, ddesc, ntiles, tab, bufs, bp, 0, L.npairs, -1, s);
    s = keep;
    g_capturing = false;
    const hipError_t ec = hipStreamEndCapture(g_cap_stream, &e.graph);
    if (rc) {
      if (e.graph) hipGraphDestroy(e.graph);
      return rc;
    }
    if (ec != hipSuccess || !e.graph) return hip_fail("end capture");
    if (hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess) {
      hipGraphDestroy(e.graph);
      return hip_fail("graph instantiate");
    }
    if (g_graphs.size() >= 8) {
      drop_graph(g_graphs.front());
      g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back(e);
    hit = &g_graphs.back();
  }
  ProfScope ps("myrtle_batched_graph", s);
  if (hipGraphLaunch(hit->exec, s) != hipSuccess) return hip_fail("graph launch");
  return ok();
}

size_t nk_myrtle_nngp_batched_workspace(const nk_tile* tiles, int32_t ntiles, const nk_myrtle_cfg* cfg) {
  NetDesc net;
  if (!tiles || ntiles <= 0 || check_myrtle(cfg, &net)) return 0;
  BatchLayout L;
  if (batch_layout(tiles, ntiles, net, &L)) return 0;
  return plan_batched(net, L.rows, ntiles, std::min<int64_t>(std::max<int64_t>(L.npairs, 1), 32768)).total +
         256 * NK_MAX_STAGES;
}

int nk_myrtle_batched_set_schedule(const nk_myrtle_cfg* cfg, const nk_batched_candidate* choice) {
  NetDesc net;
  int rc = check_myrtle(cfg, &net);
  if (rc) return rc;
  if (!choice) return fail(NK_EINVAL, "choice is NULL");
  if (choice->chunk <= 0 || choice->chunk > 32768) return fail(NK_EINVAL, "chunk must be in [1, 32768]");
  if (choice->pair_tile < 1 || choice->pair_tile > 256) return fail(NK_EINVAL, "pair_tile must be in [1, 256]");
  if (choice->persistent != 0 && choice->persistent != 1) return fail(NK_EINVAL, "persistent must be 0 or 1");
  if (choice->wg_pairs_mult != 1 && choice->wg_pairs_mult != 2) return fail(NK_EINVAL, "wg_pairs_mult must be 1 or 2");
  BatchParams bp;
  bp.chunk = choice->chunk;
  bp.T = choice->pair_tile;
  bp.persist = choice->persistent;
  bp.ppm = choice->wg_pairs_mult;
  std::lock_guard<std::mutex> g(g_tune_mu);
  TuneRecord& r = g_tune[net_key(net)];
  r.best = bp;
  r.cands.clear();
  return ok();
}

int nk_myrtle_batched_tuning(const nk_myrtle_cfg* cfg, nk_batched_candidate* out, int max_entries,
                             nk_batched_candidate* chosen) {
  NetDesc net;
  int rc = check_myrtle(cfg, &net);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(net_key(net));
  if (it == g_tune.end()) return fail(NK_EINVAL, "no batched pass has been tuned for this network yet");
  const TuneRecord& r = it->second;
  int n = 0;
  for (auto& c : r.cands) {
    if (out && n < max_entries) out[n] = c;
    ++n;
  }
  if (chosen) {
    memset(chosen, 0, sizeof *chosen);
    chosen->chunk = r.best.chunk;
    chosen->pair_tile = r.best.T;
    chosen->persistent = r.best.persist;
    chosen->kind = 0;
    chosen->wg_pairs_mult = r.best.ppm;
    for (auto& c : r.cands)
      if (c.kind == 0 && c.chunk == r.best.chunk && c.pair_tile == r.best.T && c.persistent == r.best.persist)
        chosen->us_per_pair = c.us_per_pair;
  }
  ok();
  return n;
}

}  // extern "C"
