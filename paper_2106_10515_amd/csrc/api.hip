// extern "C" entry points of libgeek.so: argument validation, workspace
// sizing and dispatch to the kernels of hash.hip, bucketize.hip, silk.hip,
// assign.hip, regroup.hip and quantile.hip.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace geek {

size_t hash_ws(const geek_hash_job& J);
int32_t hash_run(const geek_hash_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s);
size_t bucketize_ws(const geek_bucketize_job& J);
int32_t bucketize_run(const geek_bucketize_job& J, void* ws, size_t ws_bytes, int32_t* st,
                      hipStream_t s);
size_t silk_ws(const geek_silk_job& J);
int32_t silk_check(const geek_silk_job& J);
int32_t silk_run(const geek_silk_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s);
size_t assign_euclid_ws(const geek_assign_job& J);
int32_t assign_euclid(const geek_assign_job& J, void* ws, size_t ws_bytes, int32_t* st,
                      hipStream_t s);
size_t assign_sig_ws(const geek_assign_job& J);
bool assign_batchable(const geek_assign_job* jobs, int njobs);
size_t assign_batch_ws(const geek_assign_job* jobs, int njobs);
struct ScanTiles {
  int ncb, nbuf, blocks_per_cu;
};
ScanTiles scan_tiles_get(int precision, int dp);
int32_t scan_tiles_set(int precision, int dp, ScanTiles t);
int32_t assign_euclid_batch(const geek_assign_job* jobs, int njobs, void* ws, size_t ws_bytes, int32_t* st,
                            hipStream_t s);
int32_t assign_sig(const geek_assign_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s);
size_t regroup_ws(const geek_regroup_job& J);
int32_t regroup_run(const geek_regroup_job& J, void* ws, int32_t* st, hipStream_t s);
size_t quantile_ws(const geek_quantile_job& J);
int32_t quantile_run(const geek_quantile_job& J, void* ws, int32_t* st, hipStream_t s);

static thread_local std::string g_last_err;

struct ProfRec {
  int id;
  hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;
static thread_local int g_open[GEEK_PROF_COUNT] = {-1, -1, -1, -1, -1, -1, -1, -1};

void prof_begin(int id, hipStream_t s) {
  if (!g_prof_on || id < 0 || id >= GEEK_PROF_COUNT) return;
  ProfRec r{id, nullptr, nullptr};
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
  hipEventRecord(r.a, s);
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_open[id] = (int)g_prof.size();
  g_prof.push_back(r);
}

void prof_end(int id, hipStream_t s) {
  if (!g_prof_on || id < 0 || id >= GEEK_PROF_COUNT) return;
  std::lock_guard<std::mutex> g(g_prof_mu);
  const int k = g_open[id];
  if (k < 0 || k >= (int)g_prof.size()) return;
  hipEventRecord(g_prof[k].b, s);
  g_open[id] = -1;
}

namespace {
constexpr int FAN_DEVS = 64;
std::mutex g_fan_mu;
struct FanDev {
  bool tried = false, ok = false;
  hipStream_t side[FAN_LANES] = {};
  hipEvent_t fork = nullptr, join[FAN_LANES] = {};
};
FanDev g_fan[FAN_DEVS];
}  // namespace

Fan::Fan(hipStream_t main, int jobs) : main_(main) {
  if (jobs < 2 || hipGetDevice(&dev_) != hipSuccess || dev_ < 0 || dev_ >= FAN_DEVS) return;
  g_fan_mu.lock();
  FanDev& F = g_fan[dev_];
  if (!F.tried) {
    F.tried = true;
    bool ok = hipEventCreateWithFlags(&F.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < FAN_LANES; ++i)
      ok = hipStreamCreateWithFlags(&F.side[i], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&F.join[i], hipEventDisableTiming) == hipSuccess;
    F.ok = ok;
    if (!ok) (void)hipGetLastError();
  }
  if (!F.ok) {
    g_fan_mu.unlock();
    return;
  }
  n_ = jobs < FAN_LANES ? jobs : FAN_LANES;
  hipEventRecord(F.fork, main_);
  for (int i = 0; i < n_; ++i) {
    side_[i] = F.side[i];
    hipStreamWaitEvent(side_[i], F.fork, 0);
  }
}

Fan::~Fan() {
  if (n_ <= 1) return;
  FanDev& F = g_fan[dev_];
  for (int i = 0; i < n_; ++i) {
    hipEventRecord(F.join[i], side_[i]);
    hipStreamWaitEvent(main_, F.join[i], 0);
  }
  g_fan_mu.unlock();
}

size_t ws_slice(size_t bytes) { return (bytes + 255) / 256 * 256; }

int32_t hip_fail(hipError_t e) {
  g_last_err = hipGetErrorString(e);
  return GEEK_ERR_HIP;
}

static bool al16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
static bool al4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

static int32_t check_hash(const geek_hash_job& J) {
  if (J.n < 0 || J.n >= (1ll << 31)) return GEEK_ERR_ARG;
  if (J.kind == GEEK_HASH_DENSE || J.kind == GEEK_HASH_HETERO) {
    if (J.n > 0 && (!J.X || !al4(J.X))) return GEEK_ERR_ARG;
    if (!J.A || !J.b || J.d < 1 || J.ldx < J.d || J.m < 1 || J.L < 1 || !(J.w > 0.f))
      return GEEK_ERR_ARG;
    if (J.d > 256) return GEEK_ERR_UNSUPPORTED;
    if (J.m > 64) return GEEK_ERR_UNSUPPORTED;
    if ((int64_t)J.m * J.L > 65535) return GEEK_ERR_UNSUPPORTED;
  }
  if (J.kind == GEEK_HASH_DENSE) {
    if (J.m > 32) return GEEK_ERR_UNSUPPORTED;  // at least 4 bits per packed code
    if (J.n > 0 && (!J.keys || !al16(J.keys))) return GEEK_ERR_ARG;
  } else if (J.kind == GEEK_HASH_DOPH) {
    if (J.F < 1 || !J.mh_keys) return GEEK_ERR_ARG;
    if (J.F > 4096) return GEEK_ERR_UNSUPPORTED;
    if (J.n > 0 && (!J.sig || !J.offsets || !J.tokens)) return GEEK_ERR_ARG;
  } else if (J.kind == GEEK_HASH_SETS || J.kind == GEEK_HASH_HETERO) {
    if (J.F < 1 || !J.mh_keys) return GEEK_ERR_ARG;
    if (J.F > 512) return GEEK_ERR_UNSUPPORTED;
    if (J.n > 0 && !J.sig) return GEEK_ERR_ARG;
    if (J.kind == GEEK_HASH_SETS && J.n > 0 && (!J.offsets || !J.tokens)) return GEEK_ERR_ARG;
    if (J.kind == GEEK_HASH_HETERO) {
      if (J.n_cat < 0 || (J.n_cat > 0 && !J.cat)) return GEEK_ERR_ARG;
      if (J.n_cat >= 32768 || J.m * J.L >= 32768) return GEEK_ERR_UNSUPPORTED;
    }
  } else {
    return GEEK_ERR_ARG;
  }
  return GEEK_OK;
}

int32_t hash_check(const geek_hash_job& J) { return check_hash(J); }

static int32_t check_bz(const geek_bucketize_job& J) {
  if (J.n < 1 || J.n >= (1ll << 31) || J.T < 1 || J.T > 65535) return GEEK_ERR_ARG;
  if (J.key_words < 1 || J.key_words > 4) return GEEK_ERR_ARG;
  if (!J.keys || !al4(J.keys) || !J.members || !J.offsets || !J.nbuckets) return GEEK_ERR_ARG;
  if (J.table_stride < 0 || J.row_stride < J.key_words) return GEEK_ERR_ARG;
  return GEEK_OK;
}

static int32_t check_assign(const geek_assign_job& J) {
  if (J.n < 1 || J.n >= (1ll << 31) || J.k < 1) return GEEK_ERR_ARG;
  if (!J.seed_offsets || !J.seed_members || !J.assign || !J.sse) return GEEK_ERR_ARG;
  if (J.k_dev && J.metric != GEEK_METRIC_EUCLID) return GEEK_ERR_ARG;
  if (J.metric == GEEK_METRIC_EUCLID || J.metric == GEEK_METRIC_HETERO) {
    if (!J.X || !al4(J.X) || J.d < 1 || J.ldx < J.d || !J.centroids) return GEEK_ERR_ARG;
    if (J.d > 256) return GEEK_ERR_UNSUPPORTED;
    if (J.precision != GEEK_PREC_FP32 && J.precision != GEEK_PREC_BF16 && J.precision != GEEK_PREC_FP8)
      return GEEK_ERR_UNSUPPORTED;
    if (J.metric == GEEK_METRIC_HETERO) {
      if (!J.cat || J.n_cat < 1 || !J.modes || J.n_members < J.k) return GEEK_ERR_ARG;
      if (J.n_cat > 16) return GEEK_ERR_UNSUPPORTED;
      // gamma must be finite, non-negative and exact in float32
      if (!(J.gamma >= 0.0) || !(J.gamma < 1e30) || (double)(float)J.gamma != J.gamma) return GEEK_ERR_ARG;
    }
  } else if (J.metric == GEEK_METRIC_SIG) {
    if (!J.sig || J.F < 1 || !J.modes || J.n_members < J.k) return GEEK_ERR_ARG;
    if (J.F > 1024) return GEEK_ERR_UNSUPPORTED;
  } else {
    return GEEK_ERR_ARG;
  }
  return GEEK_OK;
}

static int32_t check_regroup(const geek_regroup_job& J) {
  if (J.n < 0 || J.n >= (1ll << 31) || J.k < 1) return GEEK_ERR_ARG;
  if (!J.seed_offsets || !J.k_out) return GEEK_ERR_ARG;
  if (J.n > 0 && (!J.assign || !J.seed_members)) return GEEK_ERR_ARG;
  return GEEK_OK;
}

static int32_t check_quantile(const geek_quantile_job& J) {
  if (J.n < 1 || J.n >= (1ll << 31) || J.m < 1 || J.t < 1 || (int64_t)J.t > J.n || J.d < 1) return GEEK_ERR_ARG;
  if (!J.X || !J.A || !J.members || !J.offsets || J.ldx < J.d) return GEEK_ERR_ARG;
  if (J.d > 256) return GEEK_ERR_UNSUPPORTED;
  return GEEK_OK;
}

}  // namespace geek

using namespace geek;

extern "C" {

const char* geek_status_string(int32_t s) {
  switch (s) {
    case GEEK_OK: return "ok";
    case GEEK_ERR_ARG: return "invalid argument";
    case GEEK_ERR_WORKSPACE: return "workspace too small";
    case GEEK_ERR_UNSUPPORTED: return "unsupported size";
    case GEEK_ERR_HIP: return "HIP error";
    case GEEK_ERR_NONFINITE: return "non-finite input";
    case GEEK_ERR_RANGE: return "value outside the packable range";
    case GEEK_ERR_CAPACITY: return "output capacity too small";
    case GEEK_ERR_NO_SEEDS: return "no seeds";
    case GEEK_ERR_EMPTY_SET: return "empty set";
    case GEEK_ERR_KEYS: return "too many distinct keys collide in one bucketize bin";
    default: return "unknown status";
  }
}

const char* geek_version(void) { return "geek 0.1.0 gfx950"; }

int32_t geek_set_scan_tiles(int32_t precision, int32_t dp, int32_t ncb, int32_t nbuf, int32_t blocks_per_cu) {
  return geek::scan_tiles_set(precision, dp, geek::ScanTiles{ncb, nbuf, blocks_per_cu});
}

int32_t geek_get_scan_tiles(int32_t precision, int32_t dp, int32_t* ncb, int32_t* nbuf, int32_t* blocks_per_cu) {
  if (!ncb || !nbuf || !blocks_per_cu) return GEEK_ERR_ARG;
  if (!(precision >= 0 && precision <= 2) || !(dp == 32 || dp == 64 || dp == 128 || dp == 256)) return GEEK_ERR_ARG;
  const geek::ScanTiles t = geek::scan_tiles_get(precision, dp);
  *ncb = t.ncb;
  *nbuf = t.nbuf;
  *blocks_per_cu = t.blocks_per_cu;
  return GEEK_OK;
}

int64_t geek_wallclock_hz(void) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
  return (int64_t)khz * 1000;
}

int32_t geek_profile(int32_t enable) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (enable) {
    for (auto& r : g_prof) {
      hipEventSynchronize(r.b);
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
    g_prof.clear();
    for (int i = 0; i < GEEK_PROF_COUNT; ++i) g_open[i] = -1;
  }
  g_prof_on = enable != 0;
  return GEEK_OK;
}

int32_t geek_profile_read(int32_t id, double* total_ms, int64_t* launches) {
  if (!total_ms || !launches) return GEEK_ERR_ARG;
  std::lock_guard<std::mutex> g(g_prof_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : g_prof) {
    if (r.id != id) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return hip_fail(hipGetLastError());
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return hip_fail(hipGetLastError());
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return GEEK_OK;
}

const char* geek_last_hip_error(void) { return g_last_err.c_str(); }

int32_t geek_workspace_size(int32_t op, const void* jobs, int32_t njobs, size_t* bytes) {
  if (!jobs || njobs < 1 || !bytes) return GEEK_ERR_ARG;
  size_t tot = 0;
  for (int j = 0; j < njobs; ++j) {
    size_t b = 0;
    switch (op) {
      case GEEK_OP_HASH: {
        const geek_hash_job& J = static_cast<const geek_hash_job*>(jobs)[j];
        if (int32_t rc = check_hash(J)) return rc;
        b = hash_ws(J);
        break;
      }
      case GEEK_OP_BUCKETIZE: {
        const geek_bucketize_job& J = static_cast<const geek_bucketize_job*>(jobs)[j];
        if (int32_t rc = check_bz(J)) return rc;
        b = bucketize_ws(J);
        break;
      }
      case GEEK_OP_SILK: {
        const geek_silk_job& J = static_cast<const geek_silk_job*>(jobs)[j];
        if (int32_t rc = silk_check(J)) return rc;
        b = silk_ws(J);
        break;
      }
      case GEEK_OP_ASSIGN: {
        const geek_assign_job& J = static_cast<const geek_assign_job*>(jobs)[j];
        if (int32_t rc = check_assign(J)) return rc;
        b = J.metric == GEEK_METRIC_SIG ? assign_sig_ws(J) : assign_euclid_ws(J);
        break;
      }
      case GEEK_OP_QUANTILE: {
        const geek_quantile_job& J = static_cast<const geek_quantile_job*>(jobs)[j];
        if (int32_t rc = check_quantile(J)) return rc;
        b = quantile_ws(J);
        break;
      }
      case GEEK_OP_REGROUP: {
        const geek_regroup_job& J = static_cast<const geek_regroup_job*>(jobs)[j];
        if (int32_t rc = check_regroup(J)) return rc;
        b = regroup_ws(J);
        break;
      }
      default:
        return GEEK_ERR_ARG;
    }
    tot = b > tot ? b : tot;
  }
  // hash and bucketize jobs run on up to FAN_LANES streams at once, each lane
  // reusing its own slice of the workspace for its jobs in turn
  if (op == GEEK_OP_HASH || op == GEEK_OP_BUCKETIZE)
    tot = ws_slice(tot) * (size_t)(njobs < FAN_LANES ? njobs : FAN_LANES);
  if (op == GEEK_OP_ASSIGN && assign_batchable(static_cast<const geek_assign_job*>(jobs), njobs))
    tot = assign_batch_ws(static_cast<const geek_assign_job*>(jobs), njobs);  // one slice per job
  *bytes = tot;
  return GEEK_OK;
}

int32_t geek_hash(const geek_hash_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                  int32_t* d_status, void* stream) {
  if (!jobs || njobs < 1) return GEEK_ERR_ARG;
  size_t slice = 0;
  for (int j = 0; j < njobs; ++j) {
    if (int32_t rc = check_hash(jobs[j])) return rc;
    slice = std::max(slice, ws_slice(hash_ws(jobs[j])));
  }
  if (ws_bytes < slice) return GEEK_ERR_WORKSPACE;
  // as many lanes as the workspace holds slices for
  Fan fan((hipStream_t)stream, (int)std::min<size_t>((size_t)njobs, ws_bytes / slice));
  for (int j = 0; j < njobs; ++j) {
    const int l = fan.lanes() > 1 ? j % fan.lanes() : 0;
    int32_t rc = hash_run(jobs[j], static_cast<char*>(ws) + (size_t)l * slice, slice, d_status, fan.lane(j));
    if (rc) return rc;
  }
  return GEEK_OK;
}

int32_t geek_bucketize(const geek_bucketize_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                       int32_t* d_status, void* stream) {
  if (!jobs || njobs < 1) return GEEK_ERR_ARG;
  size_t slice = 0;
  for (int j = 0; j < njobs; ++j) {
    if (int32_t rc = check_bz(jobs[j])) return rc;
    slice = std::max(slice, ws_slice(bucketize_ws(jobs[j])));
  }
  if (!ws) return GEEK_ERR_ARG;
  if (ws_bytes < slice) return GEEK_ERR_WORKSPACE;
  Fan fan((hipStream_t)stream, (int)std::min<size_t>((size_t)njobs, ws_bytes / slice));
  for (int j = 0; j < njobs; ++j) {
    const int l = fan.lanes() > 1 ? j % fan.lanes() : 0;
    int32_t rc = bucketize_run(jobs[j], static_cast<char*>(ws) + (size_t)l * slice, slice, d_status, fan.lane(j));
    if (rc) return rc;
  }
  return GEEK_OK;
}

int32_t geek_silk_seeds(const geek_silk_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                        int32_t* d_status, void* stream) {
  if (!jobs || njobs < 1) return GEEK_ERR_ARG;
  for (int j = 0; j < njobs; ++j) {
    int32_t rc = silk_run(jobs[j], ws, ws_bytes, d_status, (hipStream_t)stream);
    if (rc) return rc;
  }
  return GEEK_OK;
}

int32_t geek_assign(const geek_assign_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                    int32_t* d_status, void* stream) {
  if (!jobs || njobs < 1) return GEEK_ERR_ARG;
  for (int j = 0; j < njobs; ++j) {
    if (int32_t rc = check_assign(jobs[j])) return rc;
    if (njobs > 1 && jobs[j].k_dev) return GEEK_ERR_ARG;  // a device seed count: one job per call
  }
  if (!ws) return GEEK_ERR_ARG;
  if (assign_batchable(jobs, njobs)) {
    if (ws_bytes < assign_batch_ws(jobs, njobs)) return GEEK_ERR_WORKSPACE;
    return assign_euclid_batch(jobs, njobs, ws, ws_bytes, d_status, (hipStream_t)stream);
  }
  for (int j = 0; j < njobs; ++j) {
    const size_t need = jobs[j].metric == GEEK_METRIC_SIG ? assign_sig_ws(jobs[j])
                                                          : assign_euclid_ws(jobs[j]);
    if (ws_bytes < need) return GEEK_ERR_WORKSPACE;
  }
  for (int j = 0; j < njobs; ++j) {
    const geek_assign_job& J = jobs[j];
    int32_t rc = J.metric == GEEK_METRIC_SIG
                     ? assign_sig(J, ws, ws_bytes, d_status, (hipStream_t)stream)
                     : assign_euclid(J, ws, ws_bytes, d_status, (hipStream_t)stream);
    if (rc) return rc;
  }
  return GEEK_OK;
}

int32_t geek_regroup(const geek_regroup_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                     int32_t* d_status, void* stream) {
  if (!jobs || njobs < 1) return GEEK_ERR_ARG;
  for (int j = 0; j < njobs; ++j) {
    if (int32_t rc = check_regroup(jobs[j])) return rc;
    if (ws_bytes < regroup_ws(jobs[j])) return GEEK_ERR_WORKSPACE;
  }
  if (!ws) return GEEK_ERR_ARG;
  for (int j = 0; j < njobs; ++j)
    if (int32_t rc = regroup_run(jobs[j], ws, d_status, (hipStream_t)stream)) return rc;
  return GEEK_OK;
}

int32_t geek_quantile_buckets(const geek_quantile_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                              int32_t* d_status, void* stream) {
  if (!jobs || njobs < 1) return GEEK_ERR_ARG;
  for (int j = 0; j < njobs; ++j) {
    if (int32_t rc = check_quantile(jobs[j])) return rc;
    if (ws_bytes < quantile_ws(jobs[j])) return GEEK_ERR_WORKSPACE;
  }
  if (!ws) return GEEK_ERR_ARG;
  for (int j = 0; j < njobs; ++j)
    if (int32_t rc = quantile_run(jobs[j], ws, d_status, (hipStream_t)stream)) return rc;
  return GEEK_OK;
}

}  // extern "C"
