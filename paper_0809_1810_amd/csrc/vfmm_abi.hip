// C ABI of the vortex-particle FMM library: argument validation, workspace
// layout, and the order of the kernel launches (upward sweep, downward sweep,
// near field + evaluation; Cruz & Barba 2008, Section 3.1 and Fig. 3).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <new>
#include <string>
#include <vector>

#include "../../include/vfmm.h"
#include "vfmm_device.hpp"

using namespace vfmm;

struct vfmm_tree_s {
  Layout lay;
  TreeDev dev;
  char* ws;
  int64_t n;
  int levels;
  int p_max;
  int ops_p;        // order the operator tables were built for (-1 = none)
  int pack_p;       // order / mode of the packed matrix-core M2L operands
  int pack_mode;
  int last_p;       // order / precision of the last evaluation
  int last_prec;
  double near_radius;  // distance cut-off of the near field (0 = the paper's split)
  std::vector<hipEvent_t> ev;  // phase-timing ring: begin and end of each phase, per call
  int t_slots;
  int t_used;
  // the expansion sweeps run on `side` (default priority), concurrently with
  // the near-field schedule and the near field on the caller's stream: fork
  // after the gather of the circulations, L2P waits for the sweeps (join)
  hipStream_t side;
  hipEvent_t fork, join;
  // opt-in finiteness check of evaluations (vfmm_tree_set_check_finite):
  // the two device counters are read back into this pinned host pair
  int check_finite;
  unsigned long long* check_host;
  // recorded on the caller's stream at the end of every evaluation: the
  // handle (its stream and events) is released only once that work is done
  hipEvent_t done;
  ~vfmm_tree_s() {
    if (done) (void)hipEventSynchronize(done);
    if (side) (void)hipStreamSynchronize(side);
    if (done) (void)hipEventDestroy(done);
    if (check_host) (void)hipHostFree(check_host);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace {

thread_local std::string g_err;

vfmm_status_t fail(vfmm_status_t s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
vfmm_status_t fail(vfmm_status_t s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

}  // namespace

namespace vfmm {
void set_last_error(const char* msg) { g_err = msg; }

std::atomic<int> g_tile{kTile};
std::atomic<int> g_waves{4};
std::atomic<int> g_m2l_tile{0};
std::atomic<int> g_sym{0};
int tuning_tile() { return g_tile.load(); }
int tuning_waves() { return g_waves.load(); }
int tuning_m2l_tile() { return g_m2l_tile.load(); }
int tuning_sym() { return g_sym.load(); }

}  // namespace vfmm

namespace {

vfmm_status_t hip_fail(hipError_t e, const char* where) {
  return fail(hip_status(e), "%s: %s", where, hipGetErrorString(e));
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

bool finite_pos(double s) { return std::isfinite(s) && s > 0.0; }

vfmm_status_t check_common(int64_t n, int32_t levels, int32_t p_max) {
  if (n < 1 || n > 2147483647LL) return fail(VFMM_ERR_INVALID_ARG, "n=%lld out of [1, 2^31-1]", (long long)n);
  if (levels < 0 || levels > kMaxLevels)
    return fail(VFMM_ERR_INVALID_ARG, "levels=%d out of [0, %d]", levels, kMaxLevels);
  if (p_max < 1 || p_max > kMaxP) return fail(VFMM_ERR_INVALID_ARG, "p=%d out of [1, %d]", p_max, kMaxP);
  return VFMM_OK;
}

template <typename R>
__global__ void k_copy_expansion(const typename Types<R>::C* __restrict__ src, int64_t count,
                                 double* __restrict__ dst) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= count) return;
  const auto c = src[i];
  dst[2 * i] = double(c.x);
  dst[2 * i + 1] = double(c.y);
}

}  // namespace

namespace vfmm {

Layout make_layout(int64_t n, int levels, int p_max) {
  Layout L{};
  L.n = n;
  L.levels = levels;
  L.p_max = p_max;
  L.nleaves = int64_t(1) << (2 * levels);
  L.sort_blocks = (n + kSortPerBlock - 1) / kSortPerBlock;
  L.count_len = 256 * L.sort_blocks;
  const int64_t nonempty = n < L.nleaves ? n : L.nleaves;
  L.max_tiles = (n + kTileMin - 1) / kTileMin + nonempty;  // any tunable tile size fits
  int64_t scan_src = L.count_len > L.nleaves + 1 ? L.count_len : L.nleaves + 1;
  if (scan_src < L.max_tiles + 1) scan_src = L.max_tiles + 1;
  // block totals of a scan of up to scan_src elements, or of two scans at once
  const int64_t scan_tmp = 2 * ((scan_src + kScanPerBlock - 1) / kScanPerBlock) + 2;
  const int64_t nbox = n_boxes_2_to(levels);
  size_t off = 0;
  auto take = [&](size_t b) { size_t r = off; off += align256(b); return r; };
  L.root = take(8 * sizeof(double));
  L.bbox = take(size_t(kBBoxBlocks) * 4 * sizeof(double));
  L.keys0 = take(size_t(n) * 4);
  L.keys1 = take(size_t(n) * 4);
  L.idx0 = take(size_t(n) * 4);
  L.idx1 = take(size_t(n) * 4);
  L.counts = take(size_t(L.count_len) * 4);
  L.scan_tmp = take(size_t(scan_tmp) * 4);
  L.leaf_start = take(size_t(L.nleaves + 1) * 4);
  L.tile_off = take(size_t(L.nleaves + 1) * 4);
  L.tiles = take(size_t(L.max_tiles) * sizeof(Tile));
  L.ntiles = take(4);
  L.tile_box = take(size_t(L.max_tiles) * sizeof(float4));
  L.sched_cnt = take(size_t(L.max_tiles + 1) * 4);
  L.sched_poff = take(size_t(L.max_tiles + 1) * 4);
  L.sched_soff = take(size_t(L.max_tiles + 1) * 4);
  L.sched_parts = take(size_t(L.max_tiles + p2p_parts(L.max_tiles)) * sizeof(P2PPart));
  L.sched_partial = take(size_t(2 * p2p_parts(L.max_tiles)) * kTile * sizeof(double2));
  L.sched_near = take(size_t(n) * sizeof(double2));
  L.part64 = take(size_t(n) * sizeof(Part64));
  L.part32 = take(size_t(n) * sizeof(Part32));
  L.part32s = take(size_t(n) * sizeof(Part32));
  L.react = take(size_t(n) * sizeof(double2));
  L.xy = take(size_t(n) * sizeof(double2));
  L.me = take(size_t(nbox) * p_max * sizeof(double2));
  L.le = take(size_t(nbox) * p_max * sizeof(double2));
  const size_t nb32 = p_max > kShift64P ? size_t(nbox) * p_max * sizeof(float2) : 0;
  L.me32 = take(nb32);
  L.le32 = take(nb32);
  L.ops = take(ops_bytes(p_max));
  L.check = take(2 * sizeof(unsigned long long));
  L.total = off;
  return L;
}

}  // namespace vfmm

extern "C" {

int32_t vfmm_version(void) { return 100; }

const char* vfmm_status_string(vfmm_status_t s) {
  switch (s) {
    case VFMM_OK: return "ok";
    case VFMM_ERR_INVALID_ARG: return "invalid argument";
    case VFMM_ERR_OUT_OF_MEMORY: return "out of memory";
    case VFMM_ERR_NONFINITE: return "non-finite value";
    case VFMM_ERR_HIP: return "HIP runtime error";
    case VFMM_ERR_UNSUPPORTED: return "unsupported";
    case VFMM_ERR_WORKSPACE: return "workspace too small or misaligned";
    default: return "unknown status";
  }
}

const char* vfmm_last_error(void) { return g_err.c_str(); }

vfmm_status_t vfmm_workspace_bytes(int64_t n, int32_t levels, int32_t p_max, size_t* bytes) {
  if (!bytes) return fail(VFMM_ERR_INVALID_ARG, "bytes is NULL");
  vfmm_status_t s = check_common(n, levels, p_max);
  if (s) return s;
  *bytes = make_layout(n, levels, p_max).total;
  return VFMM_OK;
}

vfmm_status_t vfmm_build_tree(const double* x, const double* y, int64_t n, int32_t levels,
                              const double* domain, int32_t p_max, void* workspace,
                              size_t ws_bytes, void* stream, vfmm_tree_t* out) {
  if (!out) return fail(VFMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!x || !y) return fail(VFMM_ERR_INVALID_ARG, "x or y is NULL");
  if (!workspace) return fail(VFMM_ERR_INVALID_ARG, "workspace is NULL");
  vfmm_status_t s = check_common(n, levels, p_max);
  if (s) return s;
  if (domain && (!std::isfinite(domain[0]) || !std::isfinite(domain[1]) || !finite_pos(domain[2])))
    return fail(VFMM_ERR_INVALID_ARG, "domain must be finite with side > 0");
  const Layout lay = make_layout(n, levels, p_max);
  if (ws_bytes < lay.total)
    return fail(VFMM_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail(VFMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  vfmm_tree_s* t = new (std::nothrow) vfmm_tree_s{};
  if (!t) return fail(VFMM_ERR_OUT_OF_MEMORY, "host allocation of the tree handle failed");
  t->lay = lay;
  t->ws = static_cast<char*>(workspace);
  t->n = n;
  t->levels = levels;
  t->p_max = p_max;
  t->ops_p = -1;
  t->pack_p = -1;
  t->pack_mode = -1;
  t->last_p = -1;
  t->last_prec = -1;
  hipError_t e = hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&t->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&t->join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&t->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "tree stream / events");
  }
  t->dev.waves = tuning_waves();  // the launch shapes are the tree's from now on
  t->dev.m2l_tile = tuning_m2l_tile();
  e = launch_build_tree(x, y, n, levels, domain, lay, t->ws, tuning_tile(), t->dev,
                        static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "vfmm_build_tree");
  }
  t->dev.sym = tuning_sym() && t->dev.tile == 64 ? 1 : 0;
  *out = t;
  return VFMM_OK;
}

}  // extern "C"

namespace {

// Outputs u, v are checked only when there is something to write (`need_out`).
vfmm_status_t check_eval(vfmm_tree_t t, const double* gamma, double sigma, int32_t p,
                         int32_t precision, int32_t parts, const double* u, const double* v,
                         bool need_out = true) {
  if (!t) return fail(VFMM_ERR_INVALID_ARG, "tree is NULL");
  if (!gamma) return fail(VFMM_ERR_INVALID_ARG, "gamma is NULL");
  if (need_out && (!u || !v)) return fail(VFMM_ERR_INVALID_ARG, "u or v is NULL");
  if (!finite_pos(sigma)) return fail(VFMM_ERR_INVALID_ARG, "sigma must be finite and > 0");
  if (p < 1 || p > t->p_max)
    return fail(VFMM_ERR_INVALID_ARG, "p=%d out of [1, p_max=%d]", p, t->p_max);
  if (precision < VFMM_FP64 || precision > VFMM_M2L_FP16)
    return fail(VFMM_ERR_INVALID_ARG, "unknown precision %d", precision);
  if (parts < 1 || parts > 3) return fail(VFMM_ERR_INVALID_ARG, "parts must be 1, 2 or 3");
  return VFMM_OK;
}

// The opt-in finiteness check needs a synchronisation, which a stream under
// graph capture cannot take: refuse before anything is enqueued.
vfmm_status_t check_capture(vfmm_tree_t t, hipStream_t st) {
  if (!t->check_finite) return VFMM_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(VFMM_ERR_INVALID_ARG,
                "the finiteness check synchronises the stream; disable it under graph capture");
  return VFMM_OK;
}

// After an evaluation on st: counts NaN and infinite values among the inputs
// (circulations, the tree's box-local particle positions) and the nout
// velocities written, waits for the stream and reports them.
vfmm_status_t finite_check(vfmm_tree_t t, const double* gamma, const double* u, const double* v,
                           int64_t nout, hipStream_t st) {
  if (!t->check_finite) return VFMM_OK;
  unsigned long long* c = t->dev.check;
  hipError_t e = launch_clear_counter(c, st);
  if (e == hipSuccess) e = launch_clear_counter(c + 1, st);
  if (e == hipSuccess) e = launch_count_nonfinite(gamma, t->n, 1, c, st);
  const double* pos = reinterpret_cast<const double*>(t->dev.part64);
  const int64_t stride = sizeof(Part64) / sizeof(double);
  if (e == hipSuccess) e = launch_count_nonfinite(pos, t->n, stride, c, st);
  if (e == hipSuccess) e = launch_count_nonfinite(pos + 1, t->n, stride, c, st);
  if (e == hipSuccess) e = launch_count_nonfinite(u, nout, 1, c + 1, st);
  if (e == hipSuccess) e = launch_count_nonfinite(v, nout, 1, c + 1, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(t->check_host, c, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "finiteness check");
  const unsigned long long nin = t->check_host[0], nvel = t->check_host[1];
  if (nin || nvel)
    return fail(VFMM_ERR_NONFINITE, "%llu non-finite input values (circulations, positions), "
                "%llu non-finite velocity components", nin, nvel);
  return VFMM_OK;
}

// Phase-timing marks of one evaluation (no-op when timing is off or the ring
// is full): begin / end events of each phase, on the stream that runs it.
struct Marks {
  hipEvent_t* ev = nullptr;
  Marks(vfmm_tree_t t) {
    if (t->t_used < t->t_slots) ev = &t->ev[size_t(t->t_used++) * 2 * VFMM_N_PHASES];
  }
  void begin(int k, hipStream_t s) const {
    if (ev) (void)hipEventRecord(ev[2 * k], s);
  }
  void end(int k, hipStream_t s) const {
    if (ev) (void)hipEventRecord(ev[2 * k + 1], s);
  }
  void skip(int k, hipStream_t s) const {
    begin(k, s);
    end(k, s);
  }
};

enum Phase { kPhGather = 0, kPhTables, kPhP2M, kPhM2M, kPhM2L, kPhSched, kPhP2P, kPhL2P };

// One evaluation on target set tg (Fig. 3): the circulations into the sorted
// particles on the caller's stream; then on the tree's side stream the
// operator tables, P2M, M2M and M2L + L2L, while the caller's stream builds
// the near-field schedule and runs the near field; after both, L2P adds the
// far field to the near field and writes the result.  Every launch is ordered
// after the work queued on st before the call, and st waits for the side
// stream before L2P, so the call behaves as one ordered sequence on st.
vfmm_status_t evaluate(vfmm_tree_t t, const TargetsDev& tg, const double* gamma, double sigma,
                       int32_t p, int32_t precision, int32_t parts, double* u, double* v,
                       const Marks& mark, hipStream_t st) {
  const int L = t->levels;
  // the reduced-precision M2L variants share the FP32 pipeline
  const int prec = precision == VFMM_FP64 ? kFP64 : kFP32;
  const bool near = parts & VFMM_PART_NEAR;
  const bool far = L >= 2 && (parts & VFMM_PART_FAR);
  // reduced precision at high order: the shifts (P2M, M2M, L2L) in float64,
  // M2L still on the float32 / 16-bit matrix cores, L2P in float32
  const bool shift64 = prec == kFP32 && p > kShift64P;
  const int prec_up = shift64 ? kFP64 : prec;
  // the gather and the sweeps go to the side stream only when there is
  // near-field work to overlap
  hipStream_t sw = near && far ? t->side : st;
  // (the caller has opened the gather phase on st) the circulations into the
  // sorted particles, on st before the fork: the near field then depends on
  // nothing on the side stream (in a replayed graph, a node whose inputs come
  // from another branch was measured to start tens of microseconds after them)
  hipError_t e = launch_gather_gamma(t->dev, gamma, t->n, prec == kFP32 && near ? sigma : 0.0,
                                     prec == kFP64 || shift64, st);
  if (e != hipSuccess) return hip_fail(e, "gather");
  mark.end(kPhGather, st);
  if (sw != st) {
    e = hipEventRecord(t->fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(sw, t->fork, 0);
    if (e != hipSuccess) return hip_fail(e, "fork");
  }
  // the near-field schedule is enqueued before the sweeps: a captured graph
  // then keeps the caller's branch (schedule, near field) on the queue that
  // ran the gather
  mark.begin(kPhSched, st);
  if (near) {
    e = launch_p2p_schedule(t->dev, tg, L, prec, sigma, t->near_radius, st);
    if (e != hipSuccess) return hip_fail(e, "P2P schedule");
  }
  mark.end(kPhSched, st);
  mark.begin(kPhTables, sw);
  if (far && t->ops_p != p) {
    e = launch_build_ops(t->dev, p, prec, sw);
    if (e != hipSuccess) return hip_fail(e, "operator tables");
    t->ops_p = p;
    t->pack_p = -1;
  }
  if (far && prec != kFP64 && (t->pack_p != p || t->pack_mode != precision)) {
    e = launch_pack_m2l_mfma(t->dev, p, precision, sw);
    if (e != hipSuccess) return hip_fail(e, "matrix-core operands");
    t->pack_p = p;
    t->pack_mode = precision;
  }
  mark.end(kPhTables, sw);
  mark.begin(kPhP2M, sw);
  if (far) {
    e = launch_p2m(t->dev, L, p, prec_up, sw);
    if (e != hipSuccess) return hip_fail(e, "P2M");
  }
  mark.end(kPhP2M, sw);
  mark.begin(kPhM2M, sw);
  if (far) {
    e = launch_m2m(t->dev, L, p, prec_up, sw);
    if (e != hipSuccess) return hip_fail(e, "M2M");
  }
  mark.end(kPhM2M, sw);
  mark.begin(kPhM2L, sw);
  if (far) {
    e = prec == kFP64 ? launch_downward(t->dev, L, p, prec, sw)
        : shift64     ? launch_downward_shift64(t->dev, L, p, precision, sw)
                      : launch_downward_mfma(t->dev, L, p, precision, sw);
    if (e != hipSuccess) return hip_fail(e, "M2L/L2L");
    t->last_p = p;
    t->last_prec = prec_up;  // the float64 shift path keeps float64 ME / LE in t->dev.me, .le
  }
  mark.end(kPhM2L, sw);
  if (sw != st) {
    e = hipEventRecord(t->join, sw);
    if (e != hipSuccess) return hip_fail(e, "join");
  }
  mark.begin(kPhP2P, st);
  if (near) {
    e = launch_p2p(t->dev, tg, L, prec, sigma, t->near_radius, st);
    if (e != hipSuccess) return hip_fail(e, "P2P");
  }
  mark.end(kPhP2P, st);
  mark.begin(kPhL2P, st);
  if (sw != st) {
    e = hipStreamWaitEvent(st, t->join, 0);
    if (e != hipSuccess) return hip_fail(e, "join");
  }
  // near field plus far field (order 0: none, e.g. the far part alone of a
  // tree without one, L < 2, which is zeros), in the caller's order
  TreeDev tl = t->dev;
  if (shift64) tl.le = t->dev.le32;  // the leaf LEs rounded to float32
  e = launch_l2p(tl, tg, L, far ? p : 0, prec, near ? 1 : 0, u, v, st);
  if (e != hipSuccess) return hip_fail(e, "L2P");
  mark.end(kPhL2P, st);
  e = hipEventRecord(t->done, st);
  if (e != hipSuccess) return hip_fail(e, "done event");
  return VFMM_OK;
}

}  // namespace

namespace vfmm {

TargetLayout make_target_layout(int64_t nt, int levels) {
  TargetLayout L{};
  L.nt = nt;
  L.nleaves = int64_t(1) << (2 * levels);
  L.sort_blocks = (nt + kSortPerBlock - 1) / kSortPerBlock;
  L.count_len = 256 * L.sort_blocks;
  const int64_t nonempty = nt < L.nleaves ? nt : L.nleaves;
  L.max_tiles = (nt + kTileMin - 1) / kTileMin + nonempty;
  int64_t scan_src = L.count_len > L.nleaves + 1 ? L.count_len : L.nleaves + 1;
  if (scan_src < L.max_tiles + 1) scan_src = L.max_tiles + 1;
  // block totals of a scan of up to scan_src elements, or of two scans at once
  const int64_t scan_tmp = 2 * ((scan_src + kScanPerBlock - 1) / kScanPerBlock) + 2;
  size_t off = 0;
  auto take = [&](size_t b) { size_t r = off; off += align256(b); return r; };
  L.keys0 = take(size_t(nt) * 4);
  L.keys1 = take(size_t(nt) * 4);
  L.idx0 = take(size_t(nt) * 4);
  L.idx1 = take(size_t(nt) * 4);
  L.counts = take(size_t(L.count_len) * 4);
  L.scan_tmp = take(size_t(scan_tmp) * 4);
  L.leaf_start = take(size_t(L.nleaves + 1) * 4);
  L.tile_off = take(size_t(L.nleaves + 1) * 4);
  L.tiles = take(size_t(L.max_tiles) * sizeof(Tile));
  L.ntiles = take(4);
  L.tile_box = take(size_t(L.max_tiles) * sizeof(float4));
  L.sched_cnt = take(size_t(L.max_tiles + 1) * 4);
  L.sched_poff = take(size_t(L.max_tiles + 1) * 4);
  L.sched_soff = take(size_t(L.max_tiles + 1) * 4);
  L.sched_parts = take(size_t(L.max_tiles + p2p_parts(L.max_tiles)) * sizeof(P2PPart));
  L.sched_partial = take(size_t(2 * p2p_parts(L.max_tiles)) * kTile * sizeof(double2));
  L.sched_near = take(size_t(nt) * sizeof(double2));
  L.part64 = take(size_t(nt) * sizeof(Part64));
  L.part32 = take(size_t(nt) * sizeof(Part32));
  L.total = off;
  return L;
}

AdaptiveLayout make_adaptive_layout(int64_t n, int levels) {
  AdaptiveLayout L{};
  L.targets = make_target_layout(n, levels);
  size_t off = L.targets.total;
  auto take = [&](size_t b) { size_t r = off; off += align256(b); return r; };
  // box counts of levels 0 .. L: (4^(L+1) - 1) / 3 entries
  L.counts = take(size_t(((int64_t(1) << (2 * (levels + 1))) - 1) / 3) * 4);
  L.shift = take(size_t(int64_t(1) << (2 * levels)));
  L.perm = take(size_t(n) * 4);
  L.fine64 = take(size_t(n) * sizeof(Part64));
  L.total = off;
  return L;
}

}  // namespace vfmm

extern "C" {

vfmm_status_t vfmm_fmm_velocity_parts(vfmm_tree_t t, const double* gamma, double sigma, int32_t p,
                                      int32_t precision, int32_t parts, double* u, double* v,
                                      void* stream) {
  vfmm_status_t s = check_eval(t, gamma, sigma, p, precision, parts, u, v);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = check_capture(t, st))) return s;
  const Marks mark(t);
  mark.begin(kPhGather, st);
  s = evaluate(t, self_targets(t->dev, t->lay), gamma, sigma, p, precision, parts, u, v, mark, st);
  if (s) return s;
  return finite_check(t, gamma, u, v, t->n, st);
}

vfmm_status_t vfmm_targets_workspace_bytes(int64_t n_targets, int32_t levels, size_t* bytes) {
  if (!bytes) return fail(VFMM_ERR_INVALID_ARG, "bytes is NULL");
  if (n_targets < 0 || n_targets > 2147483647LL)
    return fail(VFMM_ERR_INVALID_ARG, "n_targets=%lld out of [0, 2^31-1]", (long long)n_targets);
  if (levels < 0 || levels > kMaxLevels)
    return fail(VFMM_ERR_INVALID_ARG, "levels=%d out of [0, %d]", levels, kMaxLevels);
  *bytes = make_target_layout(n_targets, levels).total;
  return VFMM_OK;
}

vfmm_status_t vfmm_fmm_velocity_at(vfmm_tree_t t, const double* gamma, double sigma, int32_t p,
                                   int32_t precision, int32_t parts, const double* xt,
                                   const double* yt, int64_t n_targets, void* workspace,
                                   size_t ws_bytes, double* u, double* v, void* stream) {
  vfmm_status_t s = check_eval(t, gamma, sigma, p, precision, parts, u, v, n_targets > 0);
  if (s) return s;
  if (n_targets < 0 || n_targets > 2147483647LL)
    return fail(VFMM_ERR_INVALID_ARG, "n_targets=%lld out of [0, 2^31-1]", (long long)n_targets);
  if (n_targets == 0) return VFMM_OK;
  if (!xt || !yt) return fail(VFMM_ERR_INVALID_ARG, "xt or yt is NULL");
  if (!workspace) return fail(VFMM_ERR_INVALID_ARG, "workspace is NULL");
  const TargetLayout lay = make_target_layout(n_targets, t->levels);
  if (ws_bytes < lay.total)
    return fail(VFMM_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail(VFMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = check_capture(t, st))) return s;
  const Marks mark(t);
  mark.begin(kPhGather, st);
  TargetsDev tg{};
  hipError_t e = launch_build_targets(xt, yt, n_targets, t->dev, t->levels, lay,
                                      static_cast<char*>(workspace), tg, st);
  if (e != hipSuccess) return hip_fail(e, "evaluation points");
  s = evaluate(t, tg, gamma, sigma, p, precision, parts, u, v, mark, st);
  if (s) return s;
  return finite_check(t, gamma, u, v, n_targets, st);
}

vfmm_status_t vfmm_adaptive_workspace_bytes(int64_t n, int32_t levels, size_t* bytes) {
  if (!bytes) return fail(VFMM_ERR_INVALID_ARG, "bytes is NULL");
  if (n < 1 || n > 2147483647LL) return fail(VFMM_ERR_INVALID_ARG, "n out of [1, 2^31-1]");
  if (levels < 0 || levels > kMaxLevels)
    return fail(VFMM_ERR_INVALID_ARG, "levels=%d out of [0, %d]", levels, kMaxLevels);
  *bytes = make_adaptive_layout(n, levels).total;
  return VFMM_OK;
}

vfmm_status_t vfmm_fmm_velocity_adaptive(vfmm_tree_t t, const double* gamma, double sigma,
                                         int32_t p, int32_t precision, int32_t parts,
                                         int64_t leaf_capacity, void* workspace, size_t ws_bytes,
                                         double* u, double* v, void* stream) {
  vfmm_status_t s = check_eval(t, gamma, sigma, p, precision, parts, u, v);
  if (s) return s;
  if (leaf_capacity < 0) return fail(VFMM_ERR_INVALID_ARG, "leaf_capacity < 0");
  if (!workspace) return fail(VFMM_ERR_INVALID_ARG, "workspace is NULL");
  const AdaptiveLayout lay = make_adaptive_layout(t->n, t->levels);
  if (ws_bytes < lay.total)
    return fail(VFMM_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail(VFMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = check_capture(t, st))) return s;
  const Marks mark(t);
  mark.begin(kPhGather, st);
  TargetsDev tg{};
  hipError_t e = launch_build_adaptive(t->dev, t->levels, leaf_capacity, lay,
                                       static_cast<char*>(workspace), tg, st);
  if (e != hipSuccess) return hip_fail(e, "adaptive targets");
  s = evaluate(t, tg, gamma, sigma, p, precision, parts, u, v, mark, st);
  if (s) return s;
  return finite_check(t, gamma, u, v, t->n, st);
}

vfmm_status_t vfmm_error_field(const double* u, const double* v, const double* ur,
                               const double* vr, int64_t n, const double* metrics, double* out,
                               void* stream) {
  if (!u || !v || !ur || !vr || !metrics || !out) return fail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (n < 0) return fail(VFMM_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return VFMM_OK;
  hipError_t e = launch_error_field(u, v, ur, vr, n, metrics, out, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? VFMM_OK : hip_fail(e, "error field");
}

vfmm_status_t vfmm_fmm_velocity(vfmm_tree_t t, const double* gamma, double sigma, int32_t p,
                                int32_t precision, double* u, double* v, void* stream) {
  return vfmm_fmm_velocity_parts(t, gamma, sigma, p, precision, VFMM_PART_ALL, u, v, stream);
}

vfmm_status_t vfmm_fmm_velocity_oneshot(const double* x, const double* y, const double* gamma,
                                        int64_t n, double sigma, int32_t p, int32_t levels,
                                        int32_t precision, double* u, double* v, void* workspace,
                                        size_t ws_bytes, void* stream) {
  vfmm_tree_t t = nullptr;
  vfmm_status_t s = vfmm_build_tree(x, y, n, levels, nullptr, p, workspace, ws_bytes, stream, &t);
  if (s) return s;
  s = vfmm_fmm_velocity(t, gamma, sigma, p, precision, u, v, stream);
  vfmm_tree_destroy(t);
  return s;
}

vfmm_status_t vfmm_direct_velocity(const double* x, const double* y, const double* gamma,
                                   int64_t n, double sigma, const int64_t* targets,
                                   int64_t n_targets, double* u, double* v, void* stream) {
  if (!x || !y || !gamma || !u || !v) return fail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (n < 1) return fail(VFMM_ERR_INVALID_ARG, "n must be >= 1");
  if (!finite_pos(sigma)) return fail(VFMM_ERR_INVALID_ARG, "sigma must be finite and > 0");
  if (!targets && n_targets != n)
    return fail(VFMM_ERR_INVALID_ARG, "n_targets must equal n when targets is NULL");
  if (n_targets < 0) return fail(VFMM_ERR_INVALID_ARG, "n_targets < 0");
  if (n_targets == 0) return VFMM_OK;
  hipError_t e = launch_direct(x, y, gamma, n, sigma, targets, nullptr, nullptr, n_targets, u, v,
                               static_cast<hipStream_t>(stream));
  return e == hipSuccess ? VFMM_OK : hip_fail(e, "direct");
}

vfmm_status_t vfmm_direct_velocity_at(const double* x, const double* y, const double* gamma,
                                      int64_t n, double sigma, const double* xt, const double* yt,
                                      int64_t n_targets, double* u, double* v, void* stream) {
  if (!x || !y || !gamma) return fail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (n < 1) return fail(VFMM_ERR_INVALID_ARG, "n must be >= 1");
  if (!finite_pos(sigma)) return fail(VFMM_ERR_INVALID_ARG, "sigma must be finite and > 0");
  if (n_targets < 0) return fail(VFMM_ERR_INVALID_ARG, "n_targets < 0");
  if (n_targets == 0) return VFMM_OK;
  if (!xt || !yt || !u || !v) return fail(VFMM_ERR_INVALID_ARG, "null pointer");
  hipError_t e = launch_direct(x, y, gamma, n, sigma, nullptr, xt, yt, n_targets, u, v,
                               static_cast<hipStream_t>(stream));
  return e == hipSuccess ? VFMM_OK : hip_fail(e, "direct");
}

size_t vfmm_metrics_scratch_bytes(void) { return size_t(kReduceBlocks) * 3 * sizeof(double); }

vfmm_status_t vfmm_error_metrics(const double* u, const double* v, const double* ur,
                                 const double* vr, int64_t n, void* scratch, double* out,
                                 void* stream) {
  if (!u || !v || !ur || !vr || !scratch || !out) return fail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (n < 1) return fail(VFMM_ERR_INVALID_ARG, "n must be >= 1");
  hipError_t e = launch_error_metrics(u, v, ur, vr, n, static_cast<double*>(scratch), out,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? VFMM_OK : hip_fail(e, "metrics");
}

vfmm_status_t vfmm_tree_arrays(vfmm_tree_t t, double* root, int32_t* perm, int32_t* leaf_start,
                               void* stream) {
  if (!t) return fail(VFMM_ERR_INVALID_ARG, "tree is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (root && e == hipSuccess)
    e = hipMemcpyAsync(root, t->dev.root, 4 * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (perm && e == hipSuccess)
    e = hipMemcpyAsync(perm, t->dev.perm, size_t(t->n) * 4, hipMemcpyDeviceToDevice, st);
  if (leaf_start && e == hipSuccess)
    e = hipMemcpyAsync(leaf_start, t->dev.leaf_start, size_t(t->lay.nleaves + 1) * 4,
                       hipMemcpyDeviceToDevice, st);
  return e == hipSuccess ? VFMM_OK : hip_fail(e, "tree arrays");
}

vfmm_status_t vfmm_tree_expansions(vfmm_tree_t t, int32_t kind, int32_t level, double* dst,
                                   void* stream) {
  if (!t || !dst) return fail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (kind != 0 && kind != 1) return fail(VFMM_ERR_INVALID_ARG, "kind must be 0 or 1");
  if (t->last_p < 1) return fail(VFMM_ERR_INVALID_ARG, "no far-field evaluation yet");
  if (level < 2 || level > t->levels)
    return fail(VFMM_ERR_INVALID_ARG, "level %d out of [2, %d]", level, t->levels);
  const int p = t->last_p;
  const int64_t count = (int64_t(1) << (2 * level)) * p;
  const int64_t off = level_offset(level) * p;
  const void* base = kind == 0 ? t->dev.me : t->dev.le;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned nb = unsigned((count + 255) / 256);
  if (t->last_prec == kFP64)
    hipLaunchKernelGGL(k_copy_expansion<double>, dim3(nb), dim3(256), 0, st,
                       static_cast<const double2*>(base) + off, count, dst);
  else
    hipLaunchKernelGGL(k_copy_expansion<float>, dim3(nb), dim3(256), 0, st,
                       static_cast<const float2*>(base) + off, count, dst);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? VFMM_OK : hip_fail(e, "expansions");
}

vfmm_status_t vfmm_tree_rebuild(vfmm_tree_t t, const double* x, const double* y,
                                const double* domain, void* stream) {
  if (!t) return fail(VFMM_ERR_INVALID_ARG, "tree is NULL");
  if (!x || !y) return fail(VFMM_ERR_INVALID_ARG, "x or y is NULL");
  if (domain && (!std::isfinite(domain[0]) || !std::isfinite(domain[1]) || !finite_pos(domain[2])))
    return fail(VFMM_ERR_INVALID_ARG, "domain must be finite with side > 0");
  hipError_t e = launch_build_tree(x, y, t->n, t->levels, domain, t->lay, t->ws, t->dev.tile,
                                   t->dev, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "vfmm_tree_rebuild");
  t->last_p = -1;
  return VFMM_OK;
}

vfmm_status_t vfmm_advect_workspace_bytes(int64_t n, size_t* bytes) {
  if (!bytes) return fail(VFMM_ERR_INVALID_ARG, "bytes is NULL");
  if (n < 1 || n > 2147483647LL) return fail(VFMM_ERR_INVALID_ARG, "n out of [1, 2^31-1]");
  *bytes = 6 * align256(size_t(n) * sizeof(double));
  return VFMM_OK;
}

vfmm_status_t vfmm_advect(vfmm_tree_t t, double* x, double* y, const double* gamma, double sigma,
                          int32_t p, int32_t precision, double dt, int32_t steps, void* workspace,
                          size_t ws_bytes, void* stream) {
  vfmm_status_t s = check_eval(t, gamma, sigma, p, precision, VFMM_PART_ALL, x, y);
  if (s) return s;
  if (!std::isfinite(dt)) return fail(VFMM_ERR_INVALID_ARG, "dt must be finite");
  if (steps < 0) return fail(VFMM_ERR_INVALID_ARG, "steps < 0");
  if (!workspace) return fail(VFMM_ERR_INVALID_ARG, "workspace is NULL");
  const size_t a = align256(size_t(t->n) * sizeof(double));
  if (ws_bytes < 6 * a)
    return fail(VFMM_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, 6 * a);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail(VFMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  char* w = static_cast<char*>(workspace);
  double* u1 = reinterpret_cast<double*>(w);
  double* v1 = reinterpret_cast<double*>(w + a);
  double* u2 = reinterpret_cast<double*>(w + 2 * a);
  double* v2 = reinterpret_cast<double*>(w + 3 * a);
  double* xs = reinterpret_cast<double*>(w + 4 * a);
  double* ys = reinterpret_cast<double*>(w + 5 * a);
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int k = 0; k < steps; ++k) {
    if ((s = vfmm_tree_rebuild(t, x, y, nullptr, stream))) return s;
    if ((s = vfmm_fmm_velocity(t, gamma, sigma, p, precision, u1, v1, stream))) return s;
    hipError_t e = launch_heun_predict(x, y, u1, v1, t->n, dt, xs, ys, st);
    if (e != hipSuccess) return hip_fail(e, "Heun predictor");
    if ((s = vfmm_tree_rebuild(t, xs, ys, nullptr, stream))) return s;
    if ((s = vfmm_fmm_velocity(t, gamma, sigma, p, precision, u2, v2, stream))) return s;
    e = launch_heun_correct(x, y, u1, v1, u2, v2, t->n, dt, st);
    if (e != hipSuccess) return hip_fail(e, "Heun corrector");
  }
  return VFMM_OK;
}

vfmm_status_t vfmm_tree_set_near_radius(vfmm_tree_t t, double radius) {
  if (!t) return fail(VFMM_ERR_INVALID_ARG, "tree is NULL");
  if (std::isnan(radius) || std::isinf(radius))
    return fail(VFMM_ERR_INVALID_ARG, "radius must be finite");
  t->near_radius = radius < 0.0 ? -1.0 : radius;
  return VFMM_OK;
}

// Kernel substitution of the far field (eq. 6 against eq. 15): every pair
// closer than d = max(w_L, a) is summed with K_sigma; beyond it the far field
// takes K', which differs from K_sigma by exp(-r^2 / 2 sigma^2) |K'|, i.e. by
// e / (1 - e) |K_sigma| with e = exp(-d^2 / 2 sigma^2) at r = d.
vfmm_status_t vfmm_substitution_bound(double root_side, int32_t levels, double sigma,
                                      double near_radius, int32_t precision, double* distance,
                                      double* bound) {
  if (!bound) return fail(VFMM_ERR_INVALID_ARG, "bound is NULL");
  if (!(root_side > 0.0) || !std::isfinite(root_side))
    return fail(VFMM_ERR_INVALID_ARG, "root side must be finite and > 0");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(VFMM_ERR_INVALID_ARG, "sigma must be finite and > 0");
  if (levels < 0 || levels > VFMM_MAX_LEVELS)
    return fail(VFMM_ERR_INVALID_ARG, "levels %d out of [0, %d]", levels, VFMM_MAX_LEVELS);
  if (!std::isfinite(near_radius)) return fail(VFMM_ERR_INVALID_ARG, "radius must be finite");
  if (precision < VFMM_FP64 || precision > VFMM_M2L_FP16)
    return fail(VFMM_ERR_INVALID_ARG, "unknown precision %d", precision);
  const double w = root_side / std::ldexp(1.0, levels);
  const double a = std::sqrt(near_cut2(near_radius < 0.0 ? -1.0 : near_radius, sigma,
                                       precision == VFMM_FP64 ? kFP64 : kFP32));
  const double d = std::fmax(w, std::fmin(a, VFMM_NEAR_RINGS_MAX * w));
  const double q = d * d / (2.0 * sigma * sigma);
  if (distance) *distance = d;
  // e / (1 - e) = 1 / expm1(q), without cancellation for small q
  *bound = q > 0.0 ? 1.0 / std::expm1(q) : HUGE_VAL;
  return VFMM_OK;
}

vfmm_status_t vfmm_tree_enable_timing(vfmm_tree_t t, int32_t max_calls) {
  if (!t) return fail(VFMM_ERR_INVALID_ARG, "tree is NULL");
  if (max_calls < 0 || max_calls > 100000) return fail(VFMM_ERR_INVALID_ARG, "max_calls out of range");
  const size_t need = size_t(max_calls) * 2 * VFMM_N_PHASES;
  try {
    t->ev.reserve(need);
  } catch (const std::bad_alloc&) {
    return fail(VFMM_ERR_OUT_OF_MEMORY, "host allocation of %zu timing events failed", need);
  }
  while (t->ev.size() < need) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return hip_fail(r, "hipEventCreate");
    t->ev.push_back(e);
  }
  t->t_slots = max_calls;
  t->t_used = 0;
  return VFMM_OK;
}

vfmm_status_t vfmm_tree_read_timing(vfmm_tree_t t, double* ms, int32_t* n_calls) {
  if (!t || !ms || !n_calls) return fail(VFMM_ERR_INVALID_ARG, "null pointer");
  const int used = t->t_used;
  for (int c = 0; c < used; ++c) {
    hipEvent_t* ev = &t->ev[size_t(c) * 2 * VFMM_N_PHASES];
    for (int k = 0; k < VFMM_N_PHASES; ++k) {
      hipError_t r = hipEventSynchronize(ev[2 * k + 1]);
      if (r != hipSuccess) return hip_fail(r, "hipEventSynchronize");
      float f = 0.f;
      r = hipEventElapsedTime(&f, ev[2 * k], ev[2 * k + 1]);
      if (r != hipSuccess) return hip_fail(r, "hipEventElapsedTime");
      ms[size_t(c) * VFMM_N_PHASES + k] = double(f);
    }
  }
  *n_calls = used;
  t->t_used = 0;
  return VFMM_OK;
}

vfmm_status_t vfmm_set_tuning(int32_t param, int32_t value) {
  if (param == VFMM_TUNE_P2P_TILE) {
    if (value != 64 && value != 32 && value != 16)
      return fail(VFMM_ERR_INVALID_ARG, "P2P tile must be 64, 32 or 16");
    g_tile.store(value);
    return VFMM_OK;
  }
  if (param == VFMM_TUNE_P2P_WAVES) {
    if (value != 1 && value != 2 && value != 4 && value != 8)
      return fail(VFMM_ERR_INVALID_ARG, "P2P waves per workgroup must be 1, 2, 4 or 8");
    g_waves.store(value);
    return VFMM_OK;
  }
  if (param == VFMM_TUNE_M2L_TILE) {
    if (value < 0 || value > 2) return fail(VFMM_ERR_INVALID_ARG, "M2L tile must be 0, 1 or 2");
    g_m2l_tile.store(value);
    return VFMM_OK;
  }
  if (param == VFMM_TUNE_P2P_SYMMETRIC) {
    if (value != 0 && value != 1) return fail(VFMM_ERR_INVALID_ARG, "P2P symmetric must be 0 or 1");
    g_sym.store(value);
    return VFMM_OK;
  }
  return fail(VFMM_ERR_INVALID_ARG, "unknown tuning parameter %d", param);
}

int32_t vfmm_get_tuning(int32_t param) {
  if (param == VFMM_TUNE_P2P_TILE) return g_tile.load();
  if (param == VFMM_TUNE_P2P_WAVES) return g_waves.load();
  if (param == VFMM_TUNE_M2L_TILE) return g_m2l_tile.load();
  if (param == VFMM_TUNE_P2P_SYMMETRIC) return g_sym.load();
  return -1;
}

int32_t vfmm_tree_get_tuning(vfmm_tree_t t, int32_t param) {
  if (!t) return -1;
  if (param == VFMM_TUNE_P2P_TILE) return t->dev.tile;
  if (param == VFMM_TUNE_P2P_WAVES) return t->dev.waves;
  if (param == VFMM_TUNE_M2L_TILE) return t->dev.m2l_tile;
  if (param == VFMM_TUNE_P2P_SYMMETRIC) return t->dev.sym;
  return -1;
}

vfmm_status_t vfmm_tree_set_check_finite(vfmm_tree_t t, int32_t enable) {
  if (!t) return fail(VFMM_ERR_INVALID_ARG, "tree is NULL");
  if (enable && !t->check_host) {
    void* h = nullptr;
    hipError_t e = hipHostMalloc(&h, 2 * sizeof(unsigned long long), hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "pinned host counters");
    t->check_host = static_cast<unsigned long long*>(h);
  }
  t->check_finite = enable ? 1 : 0;
  return VFMM_OK;
}

void vfmm_tree_destroy(vfmm_tree_t t) { delete t; }

}  // extern "C"
