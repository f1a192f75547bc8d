// C ABI of the library: argument checks (host only, before any HIP call),
// context state (stencil tables, descriptor/work-list caches, captured
// graphs, tuning choices) and dispatch to the kernels.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.h"
#include "m2l_mfma.h"

using namespace fmm;

// Device memory of fmm_m2l_noalloc: descriptors, work list and work counter of
// one call, at most FMM_NOALLOC_MAX_SUBGRIDS sub-grids. One copy per device,
// held until the process ends; every call on a device shares it. Host code
// never passes this name to a kernel or a copy: fmm_create looks up each
// device's address of it (fmm_ctx::noalloc_dev) and that address is used.
constexpr size_t kNoAllocDescBytes = sizeof(fmm_subgrid) * FMM_NOALLOC_MAX_SUBGRIDS;
constexpr size_t kNoAllocWorkOff = (kNoAllocDescBytes + 255) / 256 * 256;
constexpr size_t kNoAllocCounterOff = (kNoAllocWorkOff + sizeof(WorkItem) * FMM_NOALLOC_MAX_SUBGRIDS + 255) / 256 * 256;
constexpr size_t kNoAllocBytes = kNoAllocCounterOff + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

thread_local std::string g_create_error;

const char* kStatusStrings[] = {"FMM_OK", "FMM_EINVAL: invalid argument",
                                "FMM_ENOMEM: out of memory", "FMM_EHIP: HIP runtime error",
                                "FMM_EUNSUPPORTED: unsupported request"};

// Shell stencil 5 <= |d|^2 <= 36, dz slowest, then dy, then dx.
std::vector<int> make_stencil() {
  std::vector<int> s;
  for (int dz = -kRad; dz <= kRad; ++dz)
    for (int dy = -kRad; dy <= kRad; ++dy)
      for (int dx = -kRad; dx <= kRad; ++dx) {
        int q = dx * dx + dy * dy + dz * dz;
        if (q >= 5 && q <= 36) {
          s.push_back(dx);
          s.push_back(dy);
          s.push_back(dz);
        }
      }
  return s;
}

const std::vector<int>& stencil_host() {
  static const std::vector<int> s = make_stencil();
  return s;
}

// pairs (target cell, offset) whose source lies in each of the 27 blocks
const std::vector<int64_t>& block_pairs() {
  static const std::vector<int64_t> bp = [] {
    std::vector<int64_t> v(27, 0);
    const auto& s = stencil_host();
    for (int t = 0; t < kNTarget; ++t) {
      int jx = t % 8 + 8, jy = (t / 8) % 8 + 8, jz = t / 64 + 8;
      for (size_t i = 0; i < s.size(); i += 3) {
        int sx = jx + s[i], sy = jy + s[i + 1], sz = jz + s[i + 2];
        v[(sx / 8) + 3 * (sy / 8) + 9 * (sz / 8)]++;
      }
    }
    return v;
  }();
  return bp;
}

int64_t pairs_of_mask(uint32_t mask) {
  const auto& bp = block_pairs();
  int64_t n = 0;
  for (int b = 0; b < 27; ++b)
    if ((mask >> b) & 1u) n += bp[b];
  return n;
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

// Descriptor set uploaded to the device, plus everything derived from it.
struct DescEntry {
  std::vector<fmm_subgrid> host;
  uint64_t hash = 0;
  uint64_t id = 0;                // unique per upload (keys this set's graphs)
  uint64_t last_use = 0;
  void* dev = nullptr;            // one device allocation: descriptors, id lists, work list
  void* pinned = nullptr;         // pinned host copy of the same bytes
  size_t bytes = 0;
  DevDesc* d_desc = nullptr;
  int* d_ids[kMaxP + 1] = {};     // reference kernels: sub-grids per order
  int count[kMaxP + 1] = {};
  WorkList work;                  // matrix-core kernels, dense-form costs (C^2 per pair)
  WorkList work_h;                // the same items ordered by harmonic-form costs ((p+1)^4)
  // FMM_OPT_ROUND_SPLIT, per form (dense, harmonic): (sub-grid, round) list, the
  // first slot of each sub-grid, and the rounds' sums; one allocation each
  void* split_dev[2] = {};
  void* split_pinned[2] = {};     // host staging of the (sub-grid, round) list
  WorkList split[2];
  int* split_base[2] = {};
  double* split_part[2] = {};
  bool part_even = true;          // every part_off even: particle blocks 16-byte aligned
  int tuned[4] = {-1, -1, -1, -1};   // autotuned configuration per precision
  bool split_tuned[4] = {false, false, false, false};   // the autotuner chose the round split
  // FMM_EXACT_SLICE: the sub-grids' slice planes and exponents (one allocation)
  void* slice_dev = nullptr;
  size_t slice_bytes = 0;
  hipEvent_t ready = nullptr;     // upload finished
  hipEvent_t last_launch = nullptr;
};

struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;      // recorded after every launch of this graph
  uint64_t owner = 0;             // DescEntry::id of the descriptor set it was captured for
  uint64_t last_use = 0;
};

struct fmm_ctx {
  int device = -1;
  bool host_only = true;
  std::string last_error;
  hipStream_t internal = nullptr;
  int* d_stencil = nullptr;
  double* d_D = nullptr;                      // [892][165] derivatives up to order 8
  double* d_T[kMaxP + 1] = {};                // canonical [892][C][C] per order
  MfmaTables mfma;                            // packed tables for the matrix-core kernels
  SliceTables slice;                          // int8 table slices of FMM_EXACT_SLICE
  TreeTables tree;                            // interaction-list tables of the multi-level M2L
  std::vector<std::unique_ptr<DescEntry>> descs;
  std::unordered_map<uint64_t, GraphEntry> graphs;
  uint64_t clock = 0;
  uint64_t next_id = 0;
  int m2l_kernel = 0;                         // 0 auto, 1 reference, 2 matrix core
  int use_graph = 1;
  int tile_config = -1;
  int adjoint_form = 0;     // FMM_OPT_ADJOINT_FORM
  int p2m_window = 0;       // FMM_OPT_P2M_WINDOW
  int round_split = -1;     // FMM_OPT_ROUND_SPLIT: -1 the autotuner's choice, 0 never, 1 always
  int slices = 7;           // FMM_OPT_SLICES
  // fmm_m2l_noalloc: this device's address of the static array, a pinned host
  // copy of its descriptor and work-list part, and the event after its upload
  unsigned char* noalloc_dev = nullptr;
  unsigned char* noalloc_host = nullptr;
  hipEvent_t noalloc_uploaded = nullptr;
};

namespace {

fmm_status set_err(fmm_ctx* ctx, fmm_status st, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  else g_create_error = msg;
  return st;
}

fmm_status hip_err(fmm_ctx* ctx, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return set_err(ctx, e == hipErrorOutOfMemory ? FMM_ENOMEM : FMM_EHIP, msg);
}

#define HIP_TRY(ctx, call)                                   \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_err((ctx), e_, #call);  \
  } while (0)

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

fmm_status check_ctx(fmm_ctx* ctx) {
  if (!ctx) return set_err(nullptr, FMM_EINVAL, "context is NULL");
  return FMM_OK;
}

fmm_status check_desc(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub) {
  if (nsub < 0) return set_err(ctx, FMM_EINVAL, "nsub < 0");
  if (nsub > 0x7fffffff) return set_err(ctx, FMM_EINVAL, "nsub exceeds 2^31 - 1");
  if (nsub > 0 && !desc) return set_err(ctx, FMM_EINVAL, "desc is NULL");
  for (int64_t b = 0; b < nsub; ++b) {
    const fmm_subgrid& d = desc[b];
    char buf[160];
    if (d.p < 2 || d.p > kMaxP) {
      snprintf(buf, sizeof buf, "desc[%lld].p = %d not in {2,3,4}", (long long)b, d.p);
      return set_err(ctx, FMM_EINVAL, buf);
    }
    if (d.log2_inv_h < 0 || d.log2_inv_h > 2) {
      snprintf(buf, sizeof buf, "desc[%lld].log2_inv_h = %d not in [0,2]", (long long)b, d.log2_inv_h);
      return set_err(ctx, FMM_EINVAL, buf);
    }
    if (d.mask > kFullMask || !((d.mask >> kCentreBit) & 1u)) {
      snprintf(buf, sizeof buf, "desc[%lld].mask = 0x%x: needs bit 13 and no bit above 26", (long long)b, d.mask);
      return set_err(ctx, FMM_EINVAL, buf);
    }
    if (d.reserved != 0) {
      snprintf(buf, sizeof buf, "desc[%lld].reserved must be 0", (long long)b);
      return set_err(ctx, FMM_EINVAL, buf);
    }
    if (d.m_off < 0 || d.l_off < 0 || d.part_off < 0) {
      snprintf(buf, sizeof buf, "desc[%lld] has a negative offset", (long long)b);
      return set_err(ctx, FMM_EINVAL, buf);
    }
  }
  return FMM_OK;
}

fmm_status check_ptr(fmm_ctx* ctx, const void* p, const char* name, int64_t nsub) {
  if (nsub == 0) return FMM_OK;
  if (!p) return set_err(ctx, FMM_EINVAL, std::string(name) + " is NULL");
  if (!aligned8(p)) return set_err(ctx, FMM_EINVAL, std::string(name) + " is not 8-byte aligned");
  return FMM_OK;
}

fmm_status check_ppc(fmm_ctx* ctx, int32_t ppc) {
  if (ppc < 1 || ppc > 64) return set_err(ctx, FMM_EINVAL, "ppc not in [1, 64]");
  return FMM_OK;
}

fmm_status check_precision(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, fmm_precision prec) {
  if (prec != FMM_FP64 && prec != FMM_SPLIT_FP32 && prec != FMM_FP64_HARMONIC && prec != FMM_EXACT_SLICE)
    return set_err(ctx, FMM_EINVAL, "unknown precision");
  if (prec == FMM_EXACT_SLICE)
    for (int64_t b = 0; b < nsub; ++b)
      if (desc[b].p > 3) {
        char buf[120];
        snprintf(buf, sizeof buf, "FMM_EXACT_SLICE runs orders 2 and 3; desc[%lld].p = %d", (long long)b, desc[b].p);
        return set_err(ctx, FMM_EUNSUPPORTED, buf);
      }
  return FMM_OK;
}

#define CHECK_OK(expr)                    \
  do {                                    \
    fmm_status s_ = (expr);               \
    if (s_ != FMM_OK) return s_;          \
  } while (0)

// Set the context's device for the duration of a call, restore on exit.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) {
      err = hipSetDevice(dev);
      changed = err == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

void free_entry(DescEntry* e) {
  if (e->last_launch) (void)hipEventSynchronize(e->last_launch);
  if (e->ready) (void)hipEventSynchronize(e->ready);
  if (e->dev) (void)hipFree(e->dev);
  for (int f = 0; f < 2; ++f) {
    if (e->split_dev[f]) (void)hipFree(e->split_dev[f]);
    if (e->split_pinned[f]) (void)hipHostFree(e->split_pinned[f]);
  }
  if (e->pinned) (void)hipHostFree(e->pinned);
  if (e->slice_dev) (void)hipFree(e->slice_dev);
  if (e->ready) (void)hipEventDestroy(e->ready);
  if (e->last_launch) (void)hipEventDestroy(e->last_launch);
}

// Wait for the graph's last launch (on whatever stream it ran), then release it.
void destroy_graph(GraphEntry& g) {
  if (g.done) (void)hipEventSynchronize(g.done);
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  if (g.done) (void)hipEventDestroy(g.done);
  g = GraphEntry{};
}

constexpr size_t kMaxDescEntries = 8;
constexpr size_t kMaxGraphs = 16;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Find or upload the descriptor set; builds the id lists and the work list.
fmm_status get_desc(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, hipStream_t stream,
                    DescEntry** out) {
  const size_t nbytes = sizeof(fmm_subgrid) * (size_t)nsub;
  const uint64_t h = fnv1a(desc, nbytes, fnv1a(&nsub, sizeof nsub));
  for (auto& e : ctx->descs) {
    if (e->hash == h && e->host.size() == (size_t)nsub &&
        std::memcmp(e->host.data(), desc, nbytes) == 0) {
      e->last_use = ++ctx->clock;
      // order after the previous call on this set, whatever its stream: calls
      // share the set's work-list counters and round-split partials (the event
      // was first recorded after the upload, so this also covers the upload)
      HIP_TRY(ctx, hipStreamWaitEvent(stream, e->last_launch, 0));
      *out = e.get();
      return FMM_OK;
    }
  }
  if (ctx->descs.size() >= kMaxDescEntries) {
    auto it = std::min_element(ctx->descs.begin(), ctx->descs.end(),
                               [](const auto& a, const auto& b) { return a->last_use < b->last_use; });
    // the graphs captured for this set refer to its work list: drop those (each
    // waits for its own last launch); the other sets' graphs stay
    const uint64_t owner = (*it)->id;
    for (auto g = ctx->graphs.begin(); g != ctx->graphs.end();) {
      if (g->second.owner == owner) {
        destroy_graph(g->second);
        g = ctx->graphs.erase(g);
      } else {
        ++g;
      }
    }
    free_entry(it->get());
    ctx->descs.erase(it);
  }
  auto e = std::make_unique<DescEntry>();
  e->host.assign(desc, desc + nsub);
  e->hash = h;
  e->id = ++ctx->next_id;
  e->last_use = ++ctx->clock;
  // layout: descriptors | ids per order | work list
  std::vector<int> ids[kMaxP + 1];
  for (int64_t b = 0; b < nsub; ++b) {
    ids[desc[b].p].push_back((int)b);
    if (desc[b].part_off & 1) e->part_even = false;
  }
  std::vector<WorkItem> items = build_work_list(desc, nsub, false);
  std::vector<WorkItem> items_h = build_work_list(desc, nsub, true);
  size_t off_desc = 0;
  size_t off = align_up(nbytes, 256);
  size_t off_ids[kMaxP + 1] = {};
  for (int p = 2; p <= kMaxP; ++p) {
    off_ids[p] = off;
    off = align_up(off + sizeof(int) * ids[p].size(), 256);
  }
  size_t off_work = off;
  off = align_up(off + sizeof(WorkItem) * items.size(), 256);
  size_t off_work_h = off;
  off = align_up(off + sizeof(WorkItem) * items_h.size(), 256);
  size_t off_counter = off;
  off = align_up(off + 256, 256);
  size_t off_counter_h = off;
  off = align_up(off + 256, 256);
  e->bytes = off;
  HIP_TRY(ctx, hipMalloc(&e->dev, e->bytes));
  HIP_TRY(ctx, hipHostMalloc(&e->pinned, e->bytes, hipHostMallocDefault));
  char* hp = static_cast<char*>(e->pinned);
  std::memset(hp, 0, e->bytes);
  std::memcpy(hp + off_desc, desc, nbytes);
  for (int p = 2; p <= kMaxP; ++p) std::memcpy(hp + off_ids[p], ids[p].data(), sizeof(int) * ids[p].size());
  std::memcpy(hp + off_work, items.data(), sizeof(WorkItem) * items.size());
  std::memcpy(hp + off_work_h, items_h.data(), sizeof(WorkItem) * items_h.size());
  char* dp = static_cast<char*>(e->dev);
  e->d_desc = reinterpret_cast<DevDesc*>(dp + off_desc);
  for (int p = 2; p <= kMaxP; ++p) {
    e->d_ids[p] = reinterpret_cast<int*>(dp + off_ids[p]);
    e->count[p] = (int)ids[p].size();
  }
  e->work.items = reinterpret_cast<const WorkItem*>(dp + off_work);
  e->work.count = (int)items.size();
  e->work.counter = reinterpret_cast<unsigned*>(dp + off_counter);
  e->work.cost = 0;
  for (const auto& it : items) e->work.cost += it.cost;
  e->work_h.items = reinterpret_cast<const WorkItem*>(dp + off_work_h);
  e->work_h.count = (int)items_h.size();
  e->work_h.counter = reinterpret_cast<unsigned*>(dp + off_counter_h);
  e->work_h.cost = 0;
  for (const auto& it : items_h) e->work_h.cost += it.cost;
  HIP_TRY(ctx, hipEventCreateWithFlags(&e->ready, hipEventDisableTiming));
  HIP_TRY(ctx, hipEventCreateWithFlags(&e->last_launch, hipEventDisableTiming));
  HIP_TRY(ctx, hipMemcpyAsync(e->dev, e->pinned, e->bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(ctx, hipEventRecord(e->ready, stream));
  HIP_TRY(ctx, hipEventRecord(e->last_launch, stream));
  *out = e.get();
  ctx->descs.push_back(std::move(e));
  return FMM_OK;
}

// the work list ordered by the costs of the form that runs
const WorkList& work_for(const DescEntry* e, bool harmonic) { return harmonic ? e->work_h : e->work; }

fmm_status mark_used(fmm_ctx* ctx, DescEntry* e, hipStream_t stream) {
  HIP_TRY(ctx, hipEventRecord(e->last_launch, stream));
  return FMM_OK;
}

}  // namespace

extern "C" {

const char* fmm_status_string(fmm_status s) {
  if (s <= 0 && s >= -4) return kStatusStrings[-s];
  return "unknown fmm_status";
}

const char* fmm_last_error(const fmm_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

fmm_status fmm_stencil(int32_t* count, int32_t* offsets) {
  if (!count) return set_err(nullptr, FMM_EINVAL, "count is NULL");
  const auto& s = stencil_host();
  *count = (int32_t)(s.size() / 3);
  if (offsets) std::memcpy(offsets, s.data(), s.size() * sizeof(int32_t));
  return FMM_OK;
}

fmm_status fmm_pair_count(const fmm_subgrid* desc, int64_t nsub, int64_t* pairs) {
  if (!pairs) return set_err(nullptr, FMM_EINVAL, "pairs is NULL");
  CHECK_OK(check_desc(nullptr, desc, nsub));
  int64_t n = 0;
  for (int64_t b = 0; b < nsub; ++b) n += pairs_of_mask(desc[b].mask);
  *pairs = n;
  return FMM_OK;
}

fmm_status fmm_create(fmm_ctx** out, int32_t device) {
  if (!out) return set_err(nullptr, FMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (device < -1) return set_err(nullptr, FMM_EINVAL, "device < -1");
  auto ctx = std::make_unique<fmm_ctx>();
  if (device == -1) {
    *out = ctx.release();
    return FMM_OK;
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_err(nullptr, e, "hipGetDeviceCount");
  if (device >= ndev) return set_err(nullptr, FMM_EINVAL, "device index out of range");
  ctx->device = device;
  ctx->host_only = false;
  DeviceGuard guard(device);
  if (guard.err != hipSuccess) return hip_err(nullptr, guard.err, "hipSetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_err(nullptr, e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_err(nullptr, FMM_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
  fmm_ctx* c = ctx.get();
  auto fail = [&](hipError_t err, const char* what) {
    fmm_status st = hip_err(c, err, what);
    g_create_error = c->last_error;
    fmm_destroy(ctx.release());
    return st;
  };
#define CREATE_TRY(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) return fail(e_, #call); } while (0)
  CREATE_TRY(hipStreamCreateWithFlags(&c->internal, hipStreamNonBlocking));
  const auto& st = stencil_host();
  CREATE_TRY(hipMalloc(&c->d_stencil, st.size() * sizeof(int)));
  CREATE_TRY(hipMemcpyAsync(c->d_stencil, st.data(), st.size() * sizeof(int), hipMemcpyHostToDevice, c->internal));
  CREATE_TRY(hipMalloc(&c->d_D, sizeof(double) * kNStencil * ncomp(kMaxOrderD)));
  const std::vector<double> hD = host_derivative_tables(st.data(), kNStencil, kMaxOrderD);
  CREATE_TRY(hipMemcpyAsync(c->d_D, hD.data(), sizeof(double) * hD.size(), hipMemcpyHostToDevice, c->internal));
  for (int p = 2; p <= kMaxP; ++p) {
    const int C = ncomp(p);
    CREATE_TRY(hipMalloc(&c->d_T[p], sizeof(double) * kNStencil * C * C));
    CREATE_TRY(launch_build_tensors(c->d_D, kMaxOrderD, p, c->d_T[p], c->internal));
  }
  CREATE_TRY(mfma_tables_create(&c->mfma, c->d_T, c->d_stencil, c->internal));
  CREATE_TRY(slice_tables_create(&c->slice, c->d_T, c->internal));
  CREATE_TRY(tree_tables_create(&c->tree, c->d_T, st.data(), (int)(st.size() / 3), c->internal));
  // fmm_m2l_noalloc: the device's address of the static array (the device is current)
  CREATE_TRY(hipGetSymbolAddress(reinterpret_cast<void**>(&c->noalloc_dev), HIP_SYMBOL(scratch)));
  CREATE_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->noalloc_host), kNoAllocCounterOff, hipHostMallocDefault));
  CREATE_TRY(hipEventCreateWithFlags(&c->noalloc_uploaded, hipEventDisableTiming));
  fill_work_list(nullptr, 0, false, nullptr);   // the work-list builder's tables, set up once
  CREATE_TRY(hipStreamSynchronize(c->internal));
#undef CREATE_TRY
  *out = ctx.release();
  return FMM_OK;
}

fmm_status fmm_destroy(fmm_ctx* ctx) {
  if (!ctx) return FMM_OK;
  if (!ctx->host_only) {
    DeviceGuard guard(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& g : ctx->graphs) destroy_graph(g.second);
    for (auto& e : ctx->descs) free_entry(e.get());
    mfma_tables_destroy(&ctx->mfma);
    slice_tables_destroy(&ctx->slice);
    tree_tables_destroy(&ctx->tree);
    for (int p = 0; p <= kMaxP; ++p)
      if (ctx->d_T[p]) (void)hipFree(ctx->d_T[p]);
    if (ctx->d_D) (void)hipFree(ctx->d_D);
    if (ctx->d_stencil) (void)hipFree(ctx->d_stencil);
    if (ctx->noalloc_host) (void)hipHostFree(ctx->noalloc_host);
    if (ctx->noalloc_uploaded) (void)hipEventDestroy(ctx->noalloc_uploaded);
    if (ctx->internal) (void)hipStreamDestroy(ctx->internal);
  }
  delete ctx;
  return FMM_OK;
}

fmm_status fmm_set_option(fmm_ctx* ctx, int32_t option, int64_t value) {
  CHECK_OK(check_ctx(ctx));
  switch (option) {
    case FMM_OPT_M2L_KERNEL:
      if (value < 0 || value > 2) return set_err(ctx, FMM_EINVAL, "FMM_OPT_M2L_KERNEL value not in [0,2]");
      ctx->m2l_kernel = (int)value;
      return FMM_OK;
    case FMM_OPT_USE_GRAPH:
      if (value != 0 && value != 1) return set_err(ctx, FMM_EINVAL, "FMM_OPT_USE_GRAPH value not 0/1");
      ctx->use_graph = (int)value;
      return FMM_OK;
    case FMM_OPT_P2M_WINDOW:
      if (value != 0 && value != 1) return set_err(ctx, FMM_EINVAL, "FMM_OPT_P2M_WINDOW value not 0/1");
      ctx->p2m_window = (int)value;
      return FMM_OK;
    case FMM_OPT_ROUND_SPLIT:
      if (value < -1 || value > 1) return set_err(ctx, FMM_EINVAL, "FMM_OPT_ROUND_SPLIT value not -1/0/1");
      ctx->round_split = (int)value;
      return FMM_OK;
    case FMM_OPT_SLICES:
      if (value < kSliceMin || value > kSliceMax) return set_err(ctx, FMM_EINVAL, "FMM_OPT_SLICES value not in [6,8]");
      ctx->slices = (int)value;
      return FMM_OK;
    case FMM_OPT_ADJOINT_FORM:
      if (value != 0 && value != 1) return set_err(ctx, FMM_EINVAL, "FMM_OPT_ADJOINT_FORM value not 0/1");
      ctx->adjoint_form = (int)value;
      return FMM_OK;
    case FMM_OPT_TILE_CONFIG:
      if (value < -1 || value >= mfma_num_configs()) return set_err(ctx, FMM_EINVAL, "FMM_OPT_TILE_CONFIG out of range");
      ctx->tile_config = (int)value;
      return FMM_OK;
    default:
      return set_err(ctx, FMM_EINVAL, "unknown option");
  }
}

fmm_status fmm_p2m(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* pos,
                   const double* mass, int32_t ppc, double* M, void* stream) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ppc(ctx, ppc));
  CHECK_OK(check_ptr(ctx, pos, "pos", nsub));
  CHECK_OK(check_ptr(ctx, mass, "mass", nsub));
  CHECK_OK(check_ptr(ctx, M, "M", nsub));
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) return FMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  DescEntry* e = nullptr;
  CHECK_OK(get_desc(ctx, desc, nsub, s, &e));
  HIP_TRY(ctx, launch_p2m(e->d_desc, nsub, e->d_ids, e->count, pos, mass, ppc, M, e->part_even,
                          ctx->p2m_window != 0, s));
  return mark_used(ctx, e, s);
}

fmm_status fmm_p2m_backward(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* pos,
                            int32_t ppc, const double* dM, double* dmass, void* stream) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ppc(ctx, ppc));
  CHECK_OK(check_ptr(ctx, pos, "pos", nsub));
  CHECK_OK(check_ptr(ctx, dM, "dM", nsub));
  CHECK_OK(check_ptr(ctx, dmass, "dmass", nsub));
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) return FMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  DescEntry* e = nullptr;
  CHECK_OK(get_desc(ctx, desc, nsub, s, &e));
  HIP_TRY(ctx, launch_p2m_backward(e->d_desc, nsub, e->d_ids, e->count, pos, ppc, dM, dmass, e->part_even, s));
  return mark_used(ctx, e, s);
}

fmm_status fmm_evaluate(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* pos,
                        const double* mass, int32_t ppc, const double* L, double* out,
                        void* stream) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ppc(ctx, ppc));
  CHECK_OK(check_ptr(ctx, pos, "pos", nsub));
  CHECK_OK(check_ptr(ctx, mass, "mass", nsub));
  CHECK_OK(check_ptr(ctx, L, "L", nsub));
  CHECK_OK(check_ptr(ctx, out, "out", nsub));
  // one workgroup of 256 threads per target z-plane: the grid's thread count fits 32 bits
  if (nsub > (int64_t)1 << 21) return set_err(ctx, FMM_EINVAL, "nsub exceeds 2^21 for fmm_evaluate");
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) return FMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  DescEntry* e = nullptr;
  CHECK_OK(get_desc(ctx, desc, nsub, s, &e));
  HIP_TRY(ctx, launch_evaluate(e->d_desc, nsub, pos, mass, ppc, L, out, s));
  return mark_used(ctx, e, s);
}

// ---------------------------------------------------------------------------
// multi-level iteration on a uniform octree

static fmm_status check_tree(fmm_ctx* ctx, const fmm_tree* t) {
  if (!t) return set_err(ctx, FMM_EINVAL, "tree is NULL");
  if (t->p < 2 || t->p > kMaxP) return set_err(ctx, FMM_EINVAL, "tree.p not in {2,3,4}");
  if (t->n < 8 || t->n > 128 || (t->n & (t->n - 1)))
    return set_err(ctx, FMM_EINVAL, "tree.n must be 8, 16, 32, 64 or 128");
  if (t->ppc < 1 || t->ppc > 64) return set_err(ctx, FMM_EINVAL, "tree.ppc not in [1, 64]");
  if (t->log2_h < -4 || t->log2_h > 4) return set_err(ctx, FMM_EINVAL, "tree.log2_h not in [-4, 4]");
  if (t->harmonic != 0 && t->harmonic != 1) return set_err(ctx, FMM_EINVAL, "tree.harmonic not 0/1");
  return FMM_OK;
}

static int tree_nlevels(int n) {
  int l = 1;
  for (int m = n; m > 4; m /= 2) ++l;
  return l;
}

// element offset of level l in a workspace
static int64_t tree_level_off(const fmm_tree* t, int l) {
  const int64_t C = ncomp(t->p);
  int64_t off = 0;
  for (int i = 0, m = t->n; i < l; ++i, m /= 2) off += C * m * m * m;
  return off;
}

static fmm_status tree_begin(fmm_ctx* ctx, const fmm_tree* t) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_tree(ctx, t));
  return FMM_OK;
}

static fmm_status tree_device(fmm_ctx* ctx) {
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  return FMM_OK;
}

fmm_status fmm_tree_size(const fmm_tree* tree, int32_t* levels, int64_t* elems) {
  CHECK_OK(check_tree(nullptr, tree));
  const int nl = tree_nlevels(tree->n);
  if (levels) *levels = nl;
  if (elems) *elems = tree_level_off(tree, nl);
  return FMM_OK;
}

static fmm_status tree_upward(fmm_ctx* ctx, const fmm_tree* t, const double* pos, const double* mass,
                              double* M, hipStream_t s) {
  HIP_TRY(ctx, launch_tree_p2m(t->p, pos, mass, t->ppc, t->n, ldexp(1.0, t->log2_h), M, s));
  const int nl = tree_nlevels(t->n);
  for (int l = 0, m = t->n; l + 1 < nl; ++l, m /= 2)
    HIP_TRY(ctx, launch_tree_m2m(t->p, M + tree_level_off(t, l), M + tree_level_off(t, l + 1), m,
                                 ldexp(1.0, t->log2_h + l), s));
  return FMM_OK;
}

static fmm_status tree_m2l(fmm_ctx* ctx, const fmm_tree* t, const double* M, double* L, hipStream_t s) {
  const int nl = tree_nlevels(t->n);
  int n[8], lg[8];
  int64_t off[8];
  for (int l = 0, m = t->n; l < nl; ++l, m /= 2) {
    n[l] = m;
    lg[l] = t->log2_h + l;
    off[l] = tree_level_off(t, l);
  }
  HIP_TRY(ctx, launch_tree_m2l(t->p, ctx->tree, ctx->mfma, t->harmonic != 0, M, L, nl, n, lg, off, s));
  return FMM_OK;
}

static fmm_status tree_downward(fmm_ctx* ctx, const fmm_tree* t, double* L, hipStream_t s) {
  const int nl = tree_nlevels(t->n);
  for (int l = nl - 2; l >= 0; --l)
    HIP_TRY(ctx, launch_tree_l2l(t->p, L + tree_level_off(t, l + 1), L + tree_level_off(t, l),
                                 t->n >> l, ldexp(1.0, t->log2_h + l), s));
  return FMM_OK;
}

fmm_status fmm_tree_upward(fmm_ctx* ctx, const fmm_tree* tree, const double* pos, const double* mass,
                           double* M, void* stream) {
  CHECK_OK(tree_begin(ctx, tree));
  CHECK_OK(check_ptr(ctx, pos, "pos", 1));
  CHECK_OK(check_ptr(ctx, mass, "mass", 1));
  CHECK_OK(check_ptr(ctx, M, "M", 1));
  CHECK_OK(tree_device(ctx));
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  return tree_upward(ctx, tree, pos, mass, M, static_cast<hipStream_t>(stream));
}

fmm_status fmm_tree_m2l(fmm_ctx* ctx, const fmm_tree* tree, const double* M, double* L, void* stream) {
  CHECK_OK(tree_begin(ctx, tree));
  CHECK_OK(check_ptr(ctx, M, "M", 1));
  CHECK_OK(check_ptr(ctx, L, "L", 1));
  CHECK_OK(tree_device(ctx));
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  return tree_m2l(ctx, tree, M, L, static_cast<hipStream_t>(stream));
}

fmm_status fmm_tree_downward(fmm_ctx* ctx, const fmm_tree* tree, double* L, void* stream) {
  CHECK_OK(tree_begin(ctx, tree));
  CHECK_OK(check_ptr(ctx, L, "L", 1));
  CHECK_OK(tree_device(ctx));
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  return tree_downward(ctx, tree, L, static_cast<hipStream_t>(stream));
}

fmm_status fmm_tree_evaluate(fmm_ctx* ctx, const fmm_tree* tree, const double* pos, const double* mass,
                             const double* L, double* out, void* stream) {
  CHECK_OK(tree_begin(ctx, tree));
  CHECK_OK(check_ptr(ctx, pos, "pos", 1));
  CHECK_OK(check_ptr(ctx, mass, "mass", 1));
  CHECK_OK(check_ptr(ctx, L, "L", 1));
  CHECK_OK(check_ptr(ctx, out, "out", 1));
  CHECK_OK(tree_device(ctx));
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  HIP_TRY(ctx, launch_evaluate_grid(tree->p, tree->n, ldexp(1.0, tree->log2_h), pos, mass, tree->ppc, L,
                                    out, static_cast<hipStream_t>(stream)));
  return FMM_OK;
}

fmm_status fmm_tree_solve(fmm_ctx* ctx, const fmm_tree* tree, const double* pos, const double* mass,
                          double* M, double* L, double* out, void* stream) {
  CHECK_OK(tree_begin(ctx, tree));
  CHECK_OK(check_ptr(ctx, pos, "pos", 1));
  CHECK_OK(check_ptr(ctx, mass, "mass", 1));
  CHECK_OK(check_ptr(ctx, M, "M", 1));
  CHECK_OK(check_ptr(ctx, L, "L", 1));
  CHECK_OK(check_ptr(ctx, out, "out", 1));
  CHECK_OK(tree_device(ctx));
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  hipStream_t s = static_cast<hipStream_t>(stream);
  CHECK_OK(tree_upward(ctx, tree, pos, mass, M, s));
  CHECK_OK(tree_m2l(ctx, tree, M, L, s));
  CHECK_OK(tree_downward(ctx, tree, L, s));
  HIP_TRY(ctx, launch_evaluate_grid(tree->p, tree->n, ldexp(1.0, tree->log2_h), pos, mass, tree->ppc, L,
                                    out, s));
  return FMM_OK;
}

static fmm_status run_ref(fmm_ctx* ctx, DescEntry* e, bool backward, const double* src, double* out,
                          hipStream_t s) {
  for (int p = 2; p <= kMaxP; ++p)
    HIP_TRY(ctx, launch_m2l_ref(p, backward, e->d_desc, e->d_ids[p], e->count[p], ctx->d_stencil,
                                ctx->d_T[p], src, out, s));
  return FMM_OK;
}

// Launch the persistent matrix-core kernel, through a cached graph if enabled.
// pos, mass, Mw non-null: the fused P2M + M2L launch (launch_m2l_mfma's fused
// form; Mw is M, writable).
static fmm_status run_mfma(fmm_ctx* ctx, DescEntry* e, const double* M, double* L,
                           fmm_precision prec, int cfg, hipStream_t s,
                           const double* pos = nullptr, const double* mass = nullptr,
                           double* Mw = nullptr) {
  const WorkList& wl = work_for(e, prec == FMM_FP64_HARMONIC);
  if (!ctx->use_graph) {
    HIP_TRY(ctx, launch_m2l_mfma(ctx->mfma, wl, e->d_desc, M, L, prec, cfg, s, pos, mass, Mw));
    return FMM_OK;
  }
  uint64_t key = fnv1a(&e->id, sizeof e->id);
  key = fnv1a(&M, sizeof M, key);
  key = fnv1a(&L, sizeof L, key);
  key = fnv1a(&prec, sizeof prec, key);
  key = fnv1a(&cfg, sizeof cfg, key);
  key = fnv1a(&pos, sizeof pos, key);
  key = fnv1a(&mass, sizeof mass, key);
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (ctx->graphs.size() >= kMaxGraphs) {
      // the least recently used graph; its own last launch (on any stream) is
      // waited for before it is released
      auto victim = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                     [](const auto& a, const auto& b) { return a.second.last_use < b.second.last_use; });
      destroy_graph(victim->second);
      ctx->graphs.erase(victim);
    }
    GraphEntry g;
    g.owner = e->id;
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->internal, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_m2l_mfma(ctx->mfma, wl, e->d_desc, M, L, prec, cfg, ctx->internal, pos, mass, Mw);
    hipError_t ce = hipStreamEndCapture(ctx->internal, &g.graph);
    if (le != hipSuccess || ce != hipSuccess) {
      if (g.graph) (void)hipGraphDestroy(g.graph);
      return le != hipSuccess ? hip_err(ctx, le, "launch_m2l_mfma (capture)")
                              : hip_err(ctx, ce, "hipStreamEndCapture");
    }
    hipError_t ie = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (ie == hipSuccess) ie = hipEventCreateWithFlags(&g.done, hipEventDisableTiming);
    if (ie != hipSuccess) {
      destroy_graph(g);
      return hip_err(ctx, ie, "hipGraphInstantiate");
    }
    it = ctx->graphs.emplace(key, g).first;
  }
  it->second.last_use = ++ctx->clock;
  HIP_TRY(ctx, hipGraphLaunch(it->second.exec, s));
  HIP_TRY(ctx, hipEventRecord(it->second.done, s));
  return FMM_OK;
}

// FMM_OPT_ROUND_SPLIT: the (sub-grid, round) list of the entry for this form,
// built on first use, then the two launches
static fmm_status run_split(fmm_ctx* ctx, DescEntry* e, const double* M, double* L, fmm_precision prec,
                            int cfg, hipStream_t s) {
  const int f = prec == FMM_FP64_HARMONIC ? 1 : 0;
  const int64_t nsub = (int64_t)e->host.size();
  if (!e->split_dev[f]) {
    std::vector<WorkItem> items;
    std::vector<int> base((size_t)nsub);
    for (int64_t b = 0; b < nsub; ++b) {
      base[(size_t)b] = (int)items.size();
      for (int r = 0; r < m2l_rounds(e->host[(size_t)b].p, f == 1); ++r) items.push_back(WorkItem{(int32_t)b, r});
    }
    const size_t off_base = align_up(sizeof(WorkItem) * items.size(), 256);
    const size_t off_counter = align_up(off_base + sizeof(int) * base.size(), 256);
    const size_t off_part = align_up(off_counter + 256, 256);
    const size_t bytes = off_part + sizeof(double) * items.size() * 35 * kNTarget;
    // the list goes through pinned host memory, copied on the caller's stream
    // (both allocations are held with the descriptor set)
    void* dev = nullptr;
    void* pin = nullptr;
    HIP_TRY(ctx, hipMalloc(&dev, bytes));
    hipError_t ae = hipHostMalloc(&pin, off_counter, hipHostMallocDefault);
    if (ae != hipSuccess) {
      (void)hipFree(dev);
      return hip_err(ctx, ae, "hipHostMalloc (round split list)");
    }
    char* hp = static_cast<char*>(pin);
    std::memcpy(hp, items.data(), sizeof(WorkItem) * items.size());
    std::memcpy(hp + off_base, base.data(), sizeof(int) * base.size());
    char* dp = static_cast<char*>(dev);
    hipError_t ce = hipMemcpyAsync(dp, hp, off_counter, hipMemcpyHostToDevice, s);
    if (ce != hipSuccess) {
      (void)hipFree(dev);
      (void)hipHostFree(pin);
      return hip_err(ctx, ce, "hipMemcpyAsync (round split list)");
    }
    e->split_dev[f] = dev;
    e->split_pinned[f] = pin;
    e->split[f].items = reinterpret_cast<const WorkItem*>(dp);
    e->split[f].count = (int)items.size();
    e->split[f].counter = reinterpret_cast<unsigned*>(dp + off_counter);
    e->split_base[f] = reinterpret_cast<int*>(dp + off_base);
    e->split_part[f] = reinterpret_cast<double*>(dp + off_part);
  }
  HIP_TRY(ctx, launch_m2l_round_split(ctx->mfma, e->split[f], e->d_desc, nsub, e->split_base[f], M, L,
                                      e->split_part[f], prec, cfg, s));
  return FMM_OK;
}

// FMM_EXACT_SLICE: the slice planes and exponents of the set (allocated on first
// use, and again if more slices are asked for), then the two kernels
static fmm_status run_slice(fmm_ctx* ctx, DescEntry* e, const double* M, double* L, hipStream_t s) {
  const int64_t nsub = (int64_t)e->host.size();
  const size_t planes = align_up((size_t)nsub * ctx->slices * kSlicePlane, 256);
  const size_t bytes = planes + sizeof(int32_t) * (size_t)nsub;
  if (e->slice_bytes < bytes) {
    if (e->slice_dev) {
      // the previous launches on this set read the old buffer
      HIP_TRY(ctx, hipEventSynchronize(e->last_launch));
      (void)hipFree(e->slice_dev);
      e->slice_dev = nullptr;
      e->slice_bytes = 0;
    }
    HIP_TRY(ctx, hipMalloc(&e->slice_dev, bytes));
    e->slice_bytes = bytes;
  }
  int8_t* pl = static_cast<int8_t*>(e->slice_dev);
  int32_t* ex = reinterpret_cast<int32_t*>(pl + planes);
  HIP_TRY(ctx, launch_m2l_slice(ctx->mfma, ctx->slice, e->work_h, e->d_desc, nsub, M, L, ctx->slices, pl, ex, s));
  return FMM_OK;
}

// The M2L of one call: reference kernel, exact slices, round split or the
// persistent matrix-core kernel.
static fmm_status run_m2l(fmm_ctx* ctx, DescEntry* e, const double* M, double* L, fmm_precision prec,
                          int cfg, hipStream_t s) {
  if (ctx->m2l_kernel == 1) return run_ref(ctx, e, false, M, L, s);
  if (prec == FMM_EXACT_SLICE) return run_slice(ctx, e, M, L, s);
  const bool split = ctx->round_split > 0 || (ctx->round_split < 0 && e->split_tuned[prec]);
  if (split && (int64_t)e->host.size() <= kMaxSplitSubgrids && mfma_config_fusable(cfg))
    return run_split(ctx, e, M, L, prec, cfg, s);
  return run_mfma(ctx, e, M, L, prec, cfg, s);
}

static int pick_config(const fmm_ctx* ctx, const DescEntry* e, fmm_precision prec) {
  if (ctx->tile_config >= 0) return ctx->tile_config;
  if (e && e->tuned[prec] >= 0) return e->tuned[prec];
  return mfma_default_config(prec);
}

fmm_status fmm_m2l(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* M, double* L,
                   fmm_precision prec, void* stream) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ptr(ctx, M, "M", nsub));
  CHECK_OK(check_ptr(ctx, L, "L", nsub));
  CHECK_OK(check_precision(ctx, desc, nsub, prec));
  if (prec != FMM_FP64 && ctx->m2l_kernel == 1)
    return set_err(ctx, FMM_EINVAL, "the reference kernel computes FMM_FP64 only");
  if (ctx->m2l_kernel != 1 && ctx->tile_config >= 0 && !mfma_config_supports(ctx->tile_config, prec))
    return set_err(ctx, FMM_EINVAL, "FMM_OPT_TILE_CONFIG selects a configuration of the other precision");
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) return FMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  DescEntry* e = nullptr;
  CHECK_OK(get_desc(ctx, desc, nsub, s, &e));
  CHECK_OK(run_m2l(ctx, e, M, L, prec, pick_config(ctx, e, prec), s));
  return mark_used(ctx, e, s);
}

fmm_status fmm_m2l_noalloc(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* M,
                           double* L, fmm_precision prec, void* stream) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ptr(ctx, M, "M", nsub));
  CHECK_OK(check_ptr(ctx, L, "L", nsub));
  CHECK_OK(check_precision(ctx, desc, nsub, prec));
  if (nsub > FMM_NOALLOC_MAX_SUBGRIDS)
    return set_err(ctx, FMM_EINVAL, "fmm_m2l_noalloc: nsub exceeds FMM_NOALLOC_MAX_SUBGRIDS (16384)");
  if (prec == FMM_EXACT_SLICE)
    return set_err(ctx, FMM_EUNSUPPORTED, "fmm_m2l_noalloc: FMM_EXACT_SLICE needs slice buffers (use fmm_m2l)");
  if (ctx->m2l_kernel == 1)
    return set_err(ctx, FMM_EUNSUPPORTED, "fmm_m2l_noalloc runs the matrix-core kernels only");
  if (ctx->tile_config >= 0 && !mfma_config_supports(ctx->tile_config, prec))
    return set_err(ctx, FMM_EINVAL, "FMM_OPT_TILE_CONFIG selects a configuration of the other precision");
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) return FMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  // the pinned copy is rewritten only after the previous call's upload out of it
  HIP_TRY(ctx, hipEventSynchronize(ctx->noalloc_uploaded));
  unsigned char* hp = ctx->noalloc_host;
  std::memcpy(hp, desc, sizeof(fmm_subgrid) * (size_t)nsub);
  fill_work_list(desc, nsub, prec == FMM_FP64_HARMONIC, reinterpret_cast<WorkItem*>(hp + kNoAllocWorkOff));
  const size_t used = kNoAllocWorkOff + sizeof(WorkItem) * (size_t)nsub;
  HIP_TRY(ctx, hipMemcpyAsync(ctx->noalloc_dev, hp, used, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipEventRecord(ctx->noalloc_uploaded, s));
  WorkList wl;
  wl.items = reinterpret_cast<const WorkItem*>(ctx->noalloc_dev + kNoAllocWorkOff);
  wl.count = (int)nsub;
  wl.counter = reinterpret_cast<unsigned*>(ctx->noalloc_dev + kNoAllocCounterOff);   // reset by the launch
  HIP_TRY(ctx, launch_m2l_mfma(ctx->mfma, wl, reinterpret_cast<const DevDesc*>(ctx->noalloc_dev), M, L, prec,
                               pick_config(ctx, nullptr, prec), s));
  return FMM_OK;
}

fmm_status fmm_p2m_m2l(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* pos,
                       const double* mass, int32_t ppc, double* M, double* L, fmm_precision prec,
                       void* stream) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ppc(ctx, ppc));
  CHECK_OK(check_ptr(ctx, pos, "pos", nsub));
  CHECK_OK(check_ptr(ctx, mass, "mass", nsub));
  CHECK_OK(check_ptr(ctx, M, "M", nsub));
  CHECK_OK(check_ptr(ctx, L, "L", nsub));
  CHECK_OK(check_precision(ctx, desc, nsub, prec));
  if (prec != FMM_FP64 && ctx->m2l_kernel == 1)
    return set_err(ctx, FMM_EINVAL, "the reference kernel computes FMM_FP64 only");
  if (ctx->m2l_kernel != 1 && ctx->tile_config >= 0 && !mfma_config_supports(ctx->tile_config, prec))
    return set_err(ctx, FMM_EINVAL, "FMM_OPT_TILE_CONFIG selects a configuration of the other precision");
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) return FMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  DescEntry* e = nullptr;
  CHECK_OK(get_desc(ctx, desc, nsub, s, &e));
  const int cfg = pick_config(ctx, e, prec);
  const bool aligned = ((reinterpret_cast<uintptr_t>(pos) | reinterpret_cast<uintptr_t>(mass)) & 15u) == 0;
  // one launch pays off once workgroups take several sub-grids (with at most one
  // each, every moment phase runs at the start, on one workgroup per sub-grid)
  if (ctx->m2l_kernel != 1 && ppc == 8 && e->part_even && aligned && mfma_config_fusable(cfg) &&
      nsub > ctx->mfma.num_cu) {
    CHECK_OK(run_mfma(ctx, e, M, L, prec, cfg, s, pos, mass, M));
  } else {
    HIP_TRY(ctx, launch_p2m(e->d_desc, nsub, e->d_ids, e->count, pos, mass, ppc, M, e->part_even, true, s));
    CHECK_OK(run_m2l(ctx, e, M, L, prec, cfg, s));
  }
  return mark_used(ctx, e, s);
}

fmm_status fmm_m2l_backward(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* dL,
                            double* dM, void* stream) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ptr(ctx, dL, "dL", nsub));
  CHECK_OK(check_ptr(ctx, dM, "dM", nsub));
  if (ctx->adjoint_form == 1 && ctx->m2l_kernel == 1)
    return set_err(ctx, FMM_EINVAL, "the reference kernel computes the dense adjoint only");
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) return FMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  DescEntry* e = nullptr;
  CHECK_OK(get_desc(ctx, desc, nsub, s, &e));
  if (ctx->m2l_kernel == 1) {
    CHECK_OK(run_ref(ctx, e, true, dL, dM, s));
  } else {
    HIP_TRY(ctx, launch_m2l_mfma_backward(ctx->mfma, work_for(e, ctx->adjoint_form == 1), e->d_desc, dL, dM,
                                          ctx->adjoint_form == 1, s));
  }
  return mark_used(ctx, e, s);
}

fmm_status fmm_m2l_p2m_backward(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* pos,
                                int32_t ppc, const double* dL, double* dM, double* dmass, void* stream) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ppc(ctx, ppc));
  CHECK_OK(check_ptr(ctx, pos, "pos", nsub));
  CHECK_OK(check_ptr(ctx, dL, "dL", nsub));
  CHECK_OK(check_ptr(ctx, dM, "dM", nsub));
  CHECK_OK(check_ptr(ctx, dmass, "dmass", nsub));
  if (ctx->adjoint_form == 1 && ctx->m2l_kernel == 1)
    return set_err(ctx, FMM_EINVAL, "the reference kernel computes the dense adjoint only");
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) return FMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  DescEntry* e = nullptr;
  CHECK_OK(get_desc(ctx, desc, nsub, s, &e));
  const bool aligned = ((reinterpret_cast<uintptr_t>(pos) | reinterpret_cast<uintptr_t>(dmass)) & 15u) == 0;
  if (ctx->m2l_kernel != 1 && ppc == 8 && e->part_even && aligned && nsub > ctx->mfma.num_cu) {
    HIP_TRY(ctx, launch_m2l_mfma_backward(ctx->mfma, work_for(e, ctx->adjoint_form == 1), e->d_desc, dL, dM,
                                          ctx->adjoint_form == 1, s, pos, dmass));
  } else {
    if (ctx->m2l_kernel == 1) CHECK_OK(run_ref(ctx, e, true, dL, dM, s));
    else HIP_TRY(ctx, launch_m2l_mfma_backward(ctx->mfma, work_for(e, ctx->adjoint_form == 1), e->d_desc, dL, dM,
                                               ctx->adjoint_form == 1, s));
    HIP_TRY(ctx, launch_p2m_backward(e->d_desc, nsub, e->d_ids, e->count, pos, ppc, dM, dmass, e->part_even, s));
  }
  return mark_used(ctx, e, s);
}

fmm_status fmm_stencil_tables(fmm_ctx* ctx, int32_t p, double* out, void* stream) {
  CHECK_OK(check_ctx(ctx));
  if (p < 2 || p > kMaxP) return set_err(ctx, FMM_EINVAL, "p not in {2,3,4}");
  CHECK_OK(check_ptr(ctx, out, "out", 1));
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  const int C = ncomp(p);
  HIP_TRY(ctx, hipMemcpyAsync(out, ctx->d_T[p], sizeof(double) * kNStencil * C * C,
                              hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return FMM_OK;
}

fmm_status fmm_autotune(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub, const double* M,
                        double* L, fmm_precision prec, void* stream, int32_t* chosen) {
  CHECK_OK(check_ctx(ctx));
  CHECK_OK(check_desc(ctx, desc, nsub));
  CHECK_OK(check_ptr(ctx, M, "M", nsub));
  CHECK_OK(check_ptr(ctx, L, "L", nsub));
  CHECK_OK(check_precision(ctx, desc, nsub, prec));
  if (ctx->host_only) return set_err(ctx, FMM_EUNSUPPORTED, "host-only context");
  if (nsub == 0) {
    if (chosen) *chosen = pick_config(ctx, nullptr, prec);
    return FMM_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, guard.err);
  DescEntry* e = nullptr;
  CHECK_OK(get_desc(ctx, desc, nsub, s, &e));
  if (prec == FMM_EXACT_SLICE) {
    // one kernel: nothing to time
    e->tuned[prec] = mfma_default_config(prec);
    if (chosen) *chosen = e->tuned[prec];
    return mark_used(ctx, e, s);
  }
  hipEvent_t t0, t1;
  HIP_TRY(ctx, hipEventCreate(&t0));
  HIP_TRY(ctx, hipEventCreate(&t1));
  int best = -1;
  float best_ms = 0.f;
  for (int cfg = 0; cfg < mfma_num_configs(); ++cfg) {
    if (!mfma_config_supports(cfg, prec)) continue;
    // one warm-up launch, then the best of three
    HIP_TRY(ctx, launch_m2l_mfma(ctx->mfma, work_for(e, prec == FMM_FP64_HARMONIC), e->d_desc, M, L, prec, cfg, s));
    float cfg_ms = 1e30f;
    for (int r = 0; r < 3; ++r) {
      HIP_TRY(ctx, hipEventRecord(t0, s));
      HIP_TRY(ctx, launch_m2l_mfma(ctx->mfma, work_for(e, prec == FMM_FP64_HARMONIC), e->d_desc, M, L, prec, cfg, s));
      HIP_TRY(ctx, hipEventRecord(t1, s));
      HIP_TRY(ctx, hipEventSynchronize(t1));
      float ms = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, t0, t1));
      cfg_ms = std::min(cfg_ms, ms);
    }
    if (best < 0 || cfg_ms < best_ms) {
      best = cfg;
      best_ms = cfg_ms;
    }
  }
  // small batches: the round split with the chosen configuration, timed the same way
  e->split_tuned[prec] = false;
  if (nsub <= kMaxSplitSubgrids && mfma_config_fusable(best) && ctx->m2l_kernel != 1) {
    CHECK_OK(run_split(ctx, e, M, L, prec, best, s));
    float split_ms = 1e30f;
    for (int r = 0; r < 3; ++r) {
      HIP_TRY(ctx, hipEventRecord(t0, s));
      CHECK_OK(run_split(ctx, e, M, L, prec, best, s));
      HIP_TRY(ctx, hipEventRecord(t1, s));
      HIP_TRY(ctx, hipEventSynchronize(t1));
      float ms = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, t0, t1));
      split_ms = std::min(split_ms, ms);
    }
    e->split_tuned[prec] = split_ms < best_ms;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  e->tuned[prec] = best;
  if (chosen) *chosen = best;
  return mark_used(ctx, e, s);
}

}  // extern "C"
