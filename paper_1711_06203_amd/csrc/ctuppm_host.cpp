// Host runtime of the CTU/PPM library: problems and boxes, ghost-fill tags,
// per-stage work lists, the per-box / batched / graph / waves step forms,
// guarded steps, the two-level step, regridding, timing.
//
// Device memory: the library allocates none.  Every device table (problem
// records, box records, work lists, fill and boundary tags, the two-level
// tables) lives at the start of the workspace the caller binds to a problem,
// and is written with asynchronous copies on the context stream from pinned
// host staging buffers.  A launch reaches the tables of up to kMaxSeg problems
// through its kernel argument (a segment list), so stepping a new set of
// problems together needs neither a new table nor an allocation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "ctuppm.h"
#include "ctuppm_internal.h"

using namespace ctu;

namespace {

constexpr int kRecForms = 4;      // box records per form: own scratch, one shared scratch, wave slots, static scratch
constexpr int kFormStatic = 4;    // internal form of ctuppm_step_static: batched, stage scratch in the static array
constexpr int kMaxProblems = 4096;  // host-mapped rejection flags per context
constexpr int kMaxRetryDepth = 3;   // ctuppm_step_checked halves a rejected step at most this often

struct Level {
  std::vector<ctuppm_box> boxes;
  std::vector<double*> Ua, Ub;
  bool bound = false;
};

// Device tables of one level of a problem (pointers into its workspace) and
// the host-side ranges of the work lists: box b's units of region k (variant
// z) are upre[z][k][b] .. upre[z][k][b+1]-1, its fill chunks fpre[b] ..
// fpre[b+1]-1, its boundary chunks along d bpre[d][b] .. bpre[d][b+1]-1.
// Unit variants: 0 the batched forms, with the per-stage planes; 1 the
// per-box form; 2 the batched forms for launches too small for deep units.
constexpr int kUnitVariants = 3;
struct LevelTables {
  BoxRec* recs[kRecForms] = {};
  March* units[kUnitVariants][kNumRegions] = {};
  std::vector<int> upre[kUnitVariants][kNumRegions];
  FillTag* ftags = nullptr;
  Chunk* fch = nullptr;
  std::vector<int> fpre;
  BcTag* btags[3] = {};
  Chunk* bch[3] = {};
  std::vector<int> bpre[3];
};

// Device tables of a two-level problem.  The register faces are ordered by
// group g = 2 d + side (the face on the low / high side of the fine level
// along d); group g holds faces fgrp[g] .. fgrp[g+1]-1.  Within a group no
// two faces correct the same coarse cell.
struct TwoTables {
  TwoLevelArgs args{};
  GatherTag* gtags = nullptr;
  Chunk* gch = nullptr;
  int ngch = 0;
  CfTag* ctags = nullptr;
  Chunk* cch = nullptr;
  int ncch = 0;
  RegFace* faces = nullptr;
  int nfaces = 0;
  int fgrp[7] = {};
  AvgTag* atags = nullptr;
  Chunk* ach = nullptr;
  int nach = 0;
};

struct Problem {
  int id = -1;
  ctuppm_params prm{};
  int nlevels = 1;
  Level lev[2];
  void* ws = nullptr;
  size_t ws_bytes = 0;
  ProbDev tmpl[2]{};       // host template of the device records (constants, fixed dt, test hook)
  ProbDev* dP = nullptr;   // device record of level 0 (at the start of the workspace)
  ProbDev* dPf = nullptr;  // device record of level 1 (two-level problems)
  size_t rec_bytes = 0;    // bytes of the records at the start of the workspace
  size_t tab_bytes = 0;    // bytes reserved for the tables after them
  long long nregf = 0;     // register faces of a two-level problem
  bool tables_ok = false;  // tables uploaded for the current binding, tuning and wave size
  LevelTables lt[2];
  TwoTables tt;
  int cur = 0;             // host mirror of the level-0 parity
  long long steps = 0;
  int hslot = -1;          // slot of the host-mapped rejection flag
  int acked = 0;           // rejections the host has acknowledged
  bool guarded = false;    // guarded steps enqueued since the host mirror was last read back
  // two-level geometry: bounding box of the fine boxes (fine index flo..fhi),
  // the coarse cells clo..chi under it
  int flo[3] = {0, 0, 0}, fhi[3] = {0, 0, 0}, clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
  // a step taken in pieces (fill, dt, advance per level, average down, reflux)
  int phase = 0;                     // 0 between steps; 1 coarse level advanced, fine substeps under way
  int fine_done = 0;                 // fine substeps taken in this coarse step
  bool filled[2] = {false, false};   // ghosts of the level's current state filled since it last changed
  bool dt_ready = false;             // dt computed since the last advance
  bool averaged = false;             // fine level averaged down in this coarse step
  void state_changed() {
    filled[0] = filled[1] = false;
    dt_ready = false;
  }
};

// A set of problems stepped together in one form (host only: the device
// tables are the problems' own).  Box numbering is global over the set, in
// the order of its problems.
struct StepSet {
  std::vector<int> pids;
  std::vector<Problem*> probs;
  std::vector<int> box_off;  // first global box of each problem, plus the total
  int form = 0;
  int level = 0;
  int scheme = 0;   // shared by every problem of the set
  int riemann = 0;  // likewise
  int limiter = 0;  // likewise (reconstruction variant: 0 CW84, 1 CS, 2 CW84 + steepening)
  int species = 0;  // 1 when a problem of the set carries passive species
  int nboxes = 0;
  int zvar = 0;     // work-unit variant of its launches (LevelTables)
  hipGraph_t graph[2] = {nullptr, nullptr};  // captured step, unguarded / guarded
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  ~StepSet() {
    for (int g = 0; g < 2; ++g) {
      if (exec[g]) (void)hipGraphExecDestroy(exec[g]);
      if (graph[g]) (void)hipGraphDestroy(graph[g]);
    }
  }
  bool has_graph() const { return exec[0] || exec[1]; }
};

// Two-level step of one problem: the level sets and the captured step.
struct TwoLevel {
  StepSet* cset = nullptr;  // level-0 set (owned by ctx->sets)
  StepSet* fset = nullptr;  // level-1 set
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  ~TwoLevel() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

struct TimedLaunch {
  int stage;
  hipEvent_t a, b;
};

// Pinned host buffer of the asynchronous uploads; reusable once the copy
// recorded by its event has run.
struct Staging {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};

}  // namespace

struct ctuppm_ctx {
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;
  hipStream_t side[2] = {nullptr, nullptr};  // extra capture streams for the direction branches
  hipEvent_t fj[12] = {};                      // fork / join events of a captured step
  int concurrent = 0;                          // graphs run the three directions concurrently
  std::string err;
  std::map<int, std::unique_ptr<Problem>> probs;
  int next_id = 1;
  std::map<std::tuple<std::vector<int>, int, int>, std::unique_ptr<StepSet>> sets;
  std::map<int, std::unique_ptr<TwoLevel>> two;
  bool timing = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  double acc_ms[kNumStages] = {};
  long long acc_n[kNumStages] = {};
  int num_cus = 256;
  int blocks_per_cu = 0;  // 0: one block per work unit
  int wave_boxes = 64;    // boxes per wave of the waves form (they share this many scratch slots)
  int zseg_batched = 1;   // planes per march unit, batched / graph / waves forms
  int zseg_per_box = 1;   // planes per march unit, per-box form
  int ytile = 0;          // rows per tile of the march units (0: whole plane)
  // planes per march unit of each work region in the batched, graph and
  // waves forms, times their zseg:
  // cons->prim two (each thread converts two independent cells), the merged
  // tracing four (measured: 2.31 -> 2.13 ms at KH 256^3), the rest one
  int region_planes[kNumRegions] = {1, 2, 1, 1, 1, 1, 1, 1, 1, 4};
  static_assert(kNumRegions == 10 && kGrown == 1 && kCells1T == 9, "one default per work region");
  bool region_set[kNumRegions] = {};  // set by the caller: used as given (defaults adapt to the level size)
  int fused = 1;          // CTU cell stages: tracing and stage 1 of the three directions in one kernel each
  std::vector<Staging> staging;
  void* static_ptr = nullptr;  // this device's static stage scratch (ctuppm_step_static)
  int* hflags = nullptr;   // host-mapped rejection counters, one slot per problem
  int* dflags = nullptr;   // their device address
  std::vector<int> free_slots;
  std::vector<std::pair<int, hipEvent_t>> parked_slots;  // freed slots, reusable once the stream passes the event
};

namespace {

int fail(ctuppm_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(ctx, expr)                                                                     \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess) return fail(ctx, CTUPPM_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

int box_n(const ctuppm_box& b, int d) { return b.hi[d] - b.lo[d] + 1; }

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t box_scratch_bytes(const ctuppm_box& b, int nspec) {
  const int n[3] = {box_n(b, 0), box_n(b, 1), box_n(b, 2)};
  return align256(size_t(scratch_doubles(n, nspec)) * sizeof(double));
}

// Runge-Kutta stage fabs per box of a MOL problem (after the tables in its workspace).
int stage_fabs(const ctuppm_params& p) { return p.scheme == 1 ? 1 : (p.scheme == 2 ? 2 : 0); }

size_t box_fab_bytes(const ctuppm_box& b, int nspec) {
  size_t v = size_t(kNV + nspec);
  for (int d = 0; d < 3; ++d) v *= size_t(box_n(b, d) + 2 * kNG);
  return align256(v * sizeof(double));
}

// Bytes of the stage fabs of all level-0 boxes (zero for CTU problems).
size_t stage_fab_bytes(const std::vector<ctuppm_box>& boxes, const ctuppm_params& p) {
  size_t t = 0;
  for (const auto& b : boxes) t += box_fab_bytes(b, p.nspec);
  return t * size_t(stage_fabs(p));
}

Problem* get_problem(ctuppm_ctx* c, int pid) {
  auto it = c->probs.find(pid);
  return it == c->probs.end() ? nullptr : it->second.get();
}

void level_domain(const ctuppm_params& p, int level, int lo[3], int hi[3]) {
  for (int d = 0; d < 3; ++d) {
    const int r = 1 << level;
    lo[d] = p.domain_lo[d] * r;
    hi[d] = (p.domain_hi[d] + 1) * r - 1;
  }
}

bool overlap(const ctuppm_box& a, const ctuppm_box& b) {
  for (int d = 0; d < 3; ++d)
    if (a.hi[d] < b.lo[d] || b.hi[d] < a.lo[d]) return false;
  return true;
}

// Intersection of [alo, ahi] and [blo, bhi] per direction; false if empty.
bool intersect(const int alo[3], const int ahi[3], const int blo[3], const int bhi[3], int lo[3], int hi[3]) {
  for (int d = 0; d < 3; ++d) {
    lo[d] = std::max(alo[d], blo[d]);
    hi[d] = std::min(ahi[d], bhi[d]);
    if (lo[d] > hi[d]) return false;
  }
  return true;
}

// The pieces of box a outside box b (disjoint; none if b covers a): slabs
// below and above b along x, then along y, then along z.
void subtract_box(const ctuppm_box& a, const ctuppm_box& b, std::vector<ctuppm_box>& out) {
  if (!overlap(a, b)) {
    out.push_back(a);
    return;
  }
  ctuppm_box rest = a;
  for (int d = 0; d < 3; ++d) {
    if (rest.lo[d] < b.lo[d]) {
      ctuppm_box p = rest;
      p.hi[d] = b.lo[d] - 1;
      out.push_back(p);
      rest.lo[d] = b.lo[d];
    }
    if (rest.hi[d] > b.hi[d]) {
      ctuppm_box p = rest;
      p.lo[d] = b.hi[d] + 1;
      out.push_back(p);
      rest.hi[d] = b.hi[d];
    }
  }
}

// Box a minus the union of `boxes`, as disjoint boxes.
std::vector<ctuppm_box> subtract_all(const ctuppm_box& a, const std::vector<ctuppm_box>& boxes) {
  std::vector<ctuppm_box> cur{a}, next;
  for (const auto& b : boxes) {
    next.clear();
    for (const auto& p : cur) subtract_box(p, b, next);
    cur.swap(next);
    if (cur.empty()) break;
  }
  return cur;
}

long long box_vol(const ctuppm_box& b) {
  long long v = 1;
  for (int d = 0; d < 3; ++d) v *= box_n(b, d);
  return v;
}

void chunk_region(std::vector<Chunk>& out, int box, long long items) {
  for (long long s = 0; s < items; s += kBlock) out.push_back(Chunk{box, int(s)});
}

// March units of one box region.  The (x, y) plane is cut into tiles of
// `ytile` rows (0: the whole plane); the units of a tile run through z
// segments of `zseg` planes, each segment cut into 256-item pieces.  Units are
// ordered (tile, segment, piece), so a unit's y neighbour is the next unit and
// its z neighbour a tile's worth of pieces later.
void march_region(std::vector<March>& out, int box, const int org[3], const int ext[3], int zseg, int ytile) {
  const int rows = ytile > 0 ? ytile : ext[1];
  for (int y0 = 0; y0 < ext[1]; y0 += rows) {
    const int y1 = std::min(ext[1], y0 + rows);
    const int beg = y0 * ext[0], end = y1 * ext[0];
    for (int z0 = 0; z0 < ext[2]; z0 += zseg) {
      const int z1 = std::min(ext[2], z0 + zseg);
      for (int s = beg; s < end; s += kBlock) out.push_back(March{box, s, end, org[2] + z0, org[2] + z1, 0});
    }
  }
}

constexpr int kMinUnitsPerCu = 8;  // deeper work units only while a level keeps this many per CU

// Most march units one box region can have under any tuning (one row per
// tile, one plane per unit).
long long max_units(const int n[3], int kind) {
  int org[3], ext[3];
  region_of(kind, n, org, ext);
  return (long long)ext[1] * ext[2] * ((ext[0] + kBlock - 1) / kBlock);
}

int grid_for(const ctuppm_ctx* c, int nchunks, bool persistent) {
  int g = (nchunks + 7) / 8 * 8;
  if (persistent && c->blocks_per_cu > 0) g = std::min(g, c->blocks_per_cu * c->num_cus);
  return std::max(8, g);
}

hipEvent_t take_event(ctuppm_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// ------------------------------------------------------------------ uploads

// Copy n bytes from host memory to device address dst, asynchronously on the
// context stream, through a pinned staging buffer (the source may be reused
// as soon as this returns).
int upload(ctuppm_ctx* c, void* dst, const void* src, size_t n) {
  if (n == 0) return CTUPPM_OK;
  Staging* st = nullptr;
  for (auto& b : c->staging) {
    if (b.cap < n) continue;
    if (b.used) {
      const hipError_t q = hipEventQuery(b.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return fail(c, CTUPPM_EHIP, "hipEventQuery: %s", hipGetErrorString(q));
    }
    if (!st || b.cap < st->cap) st = &b;
  }
  if (!st) {
    Staging b;
    b.cap = std::max<size_t>(size_t(1) << 16, (n + 4095) & ~size_t(4095));
    HIPCHK(c, hipHostMalloc(&b.host, b.cap, hipHostMallocDefault));
    HIPCHK(c, hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
    c->staging.push_back(b);
    st = &c->staging.back();
  }
  std::memcpy(st->host, src, n);
  HIPCHK(c, hipMemcpyAsync(dst, st->host, n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipEventRecord(st->done, c->stream));
  st->used = true;
  return CTUPPM_OK;
}

// Read n bytes of device memory (synchronises the context stream).
int download(ctuppm_ctx* c, void* dst, const void* src, size_t n) {
  HIPCHK(c, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CTUPPM_OK;
}

// Host image of a block of device tables: put() appends an array (256-byte
// aligned) and returns the device address it will have.
struct Packer {
  std::vector<char> buf;
  char* dbase = nullptr;
  template <class T>
  T* put(const std::vector<T>& v) {
    const size_t off = align256(buf.size());
    buf.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
    return v.empty() ? nullptr : (T*)(dbase + off);
  }
  void reserve_bytes(size_t n) { buf.resize(align256(buf.size()) + n); }
};

// Bytes the packer reserves for an array of n T's.
template <class T>
size_t packed(long long n) {
  return align256(size_t(n) * sizeof(T));
}

// ------------------------------------------------------------ launch helpers

// Per-launch arguments of the stages that take them (array selection and the
// Runge-Kutta combination of the MOL update).
struct StageArgs {
  int arr = kArrCur;
  int out = kArrNext;
  int comb = 0;
  double c = 0.0;
  int last = 1;
  int rs = 0;
  int lim = 0;
  int sp = 0;
  int mol = 0;
  int spstage = 0;
};

// Launch one stage over a segment list with optional timing.
int launch_segs(ctuppm_ctx* c, hipStream_t s, int stage, const Segs& G, bool persistent, bool timed,
                const StageArgs& A) {
  if (G.n <= 0 || G.beg[G.n] <= 0) return CTUPPM_OK;
  Launch L{};
  L.segs = G;
  L.grid = grid_for(c, G.beg[G.n], persistent);
  L.stream = s;
  L.arr = A.arr;
  L.out = A.out;
  L.comb = A.comb;
  L.c = A.c;
  L.last = A.last;
  L.rs = A.rs;
  L.lim = A.lim;
  L.sp = A.sp;
  L.mol = A.mol;
  L.spstage = A.spstage;
  hipEvent_t a = nullptr, b = nullptr;
  if (timed) {
    a = take_event(c);
    b = take_event(c);
    if (!a || !b) return fail(c, CTUPPM_EHIP, "hipEventCreate failed");
    HIPCHK(c, hipEventRecord(a, s));
  }
  hipError_t e = launch_stage(stage, L);
  if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "launch of %s: %s", stage_name(stage), hipGetErrorString(e));
  if (timed) {
    HIPCHK(c, hipEventRecord(b, s));
    c->timed.push_back(TimedLaunch{stage, a, b});
  }
  return CTUPPM_OK;
}

// Collects the segments of one stage, launching whenever kMaxSeg are full.
struct SegRun {
  ctuppm_ctx* c;
  hipStream_t s;
  int stage;
  bool persistent, timed;
  StageArgs A;
  Segs G{};
  int add(const BoxRec* boxes, const void* work, const void* tags, ProbDev* P, int count) {
    if (count <= 0) return CTUPPM_OK;
    if (G.n == kMaxSeg) {
      const int rc = flush();
      if (rc) return rc;
    }
    G.s[G.n] = Seg{boxes, work, tags, P};
    G.beg[G.n + 1] = G.beg[G.n] + count;
    G.n += 1;
    return CTUPPM_OK;
  }
  int flush() {
    const int rc = launch_segs(c, s, stage, G, persistent, timed, A);
    G = Segs{};
    return rc;
  }
};

int rec_form(int form) {
  return form == CTUPPM_FORM_PER_BOX ? 1 : (form == CTUPPM_FORM_WAVES ? 2 : (form == kFormStatic ? 3 : 0));
}

ProbDev* level_rec(Problem* P, int level) { return level == 0 ? P->dP : P->dPf; }

// Run one stage of a set over its global boxes b0..b1-1 (their work is
// contiguous in each problem's lists): march units for the cell stages, tag
// chunks for the ghost fill and the boundaries.
int run_range(ctuppm_ctx* c, StepSet* S, hipStream_t s, int stage, int b0, int b1, bool timed,
              const StageArgs& A0 = StageArgs()) {
  // the species stage of the merged kernels: for sets with species, unless
  // the merged kernels trace them (fused mode 2)
  const int spstage = S->species && c->fused == 1;
  if (stage == kStSpec3 && !spstage) return CTUPPM_OK;
  SegRun R{c, s, stage, S->form != CTUPPM_FORM_PER_BOX, timed, A0};
  R.A.rs = S->riemann;
  R.A.lim = S->limiter;
  R.A.sp = S->species;
  R.A.mol = S->scheme != 0;
  R.A.spstage = spstage;
  const int rf = rec_form(S->form), zv = S->zvar;
  for (size_t ip = 0; ip < S->probs.size(); ++ip) {
    const int off = S->box_off[ip], nb = S->box_off[ip + 1] - off;
    const int lb0 = std::max(0, b0 - off), lb1 = std::min(nb, b1 - off);
    if (lb0 >= lb1) continue;
    Problem* P = S->probs[ip];
    const LevelTables& T = P->lt[S->level];
    ProbDev* rec = level_rec(P, S->level);
    int rc;
    if (stage == kStFill) {
      rc = R.add(T.recs[rf], T.fch + T.fpre[lb0], T.ftags, rec, T.fpre[lb1] - T.fpre[lb0]);
    } else if (stage >= kStBcX && stage <= kStBcZ) {
      const int d = stage - kStBcX;
      rc = R.add(T.recs[rf], T.bch[d] + T.bpre[d][lb0], T.btags[d], rec, T.bpre[d][lb1] - T.bpre[d][lb0]);
    } else {
      const int k = stage_region(stage);
      const std::vector<int>& pre = T.upre[zv][k];
      rc = R.add(T.recs[rf], T.units[zv][k] + pre[lb0], nullptr, rec, pre[lb1] - pre[lb0]);
    }
    if (rc) return rc;
  }
  return R.flush();
}

int run_all(ctuppm_ctx* c, StepSet* S, hipStream_t s, int stage, bool timed, const StageArgs& A = StageArgs()) {
  return run_range(c, S, s, stage, 0, S->nboxes, timed, A);
}

// dt (launch_dt) or commit (launch_flip) of every problem of a set.
int run_probs(ctuppm_ctx* c, StepSet* S, hipStream_t s, bool flip, int guard) {
  Segs G{};
  auto go = [&]() -> int {
    hipError_t e = flip ? launch_flip(G, guard, s) : launch_dt(G, s);
    if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "%s launch: %s", flip ? "flip" : "dt", hipGetErrorString(e));
    G = Segs{};
    return CTUPPM_OK;
  };
  for (Problem* P : S->probs) {
    if (G.n == kMaxSeg) {
      const int rc = go();
      if (rc) return rc;
    }
    G.s[G.n++].P = level_rec(P, S->level);
  }
  return go();
}

// ------------------------------------------------------------- validation

// Boxes of level l: inside the level's domain, non-empty, edges <= 256, disjoint.
int check_level(ctuppm_ctx* c, const ctuppm_params& prm, int l, const ctuppm_box* boxes, int n) {
  int dlo[3], dhi[3];
  level_domain(prm, l, dlo, dhi);
  for (int b = 0; b < n; ++b) {
    const ctuppm_box& B = boxes[b];
    for (int d = 0; d < 3; ++d) {
      if (B.lo[d] > B.hi[d] || B.lo[d] < dlo[d] || B.hi[d] > dhi[d])
        return fail(c, CTUPPM_EINVAL, "level %d box %d outside the domain or empty", l, b);
      if (B.hi[d] - B.lo[d] + 1 > 256)
        return fail(c, CTUPPM_EINVAL, "level %d box %d: edges above 256 cells are not supported", l, b);
    }
    for (int o = 0; o < b; ++o)
      if (overlap(B, boxes[o])) return fail(c, CTUPPM_EINVAL, "level %d boxes %d and %d overlap", l, o, b);
  }
  return CTUPPM_OK;
}

// Fine boxes: aligned to coarse cells (even first, odd last index), each at
// least 3 coarse cells inside the domain.  Gives the bounding box of the fine
// level (fine flo..fhi, coarse clo..chi).
int fine_geometry(ctuppm_ctx* c, const ctuppm_params& prm, const std::vector<ctuppm_box>& fb, int flo[3],
                  int fhi[3], int clo[3], int chi[3]) {
  for (int d = 0; d < 3; ++d) {
    flo[d] = fb[0].lo[d];
    fhi[d] = fb[0].hi[d];
  }
  for (const auto& b : fb)
    for (int d = 0; d < 3; ++d) {
      if ((b.lo[d] & 1) || !(b.hi[d] & 1))
        return fail(c, CTUPPM_EINVAL, "fine boxes must start at even and end at odd indices");
      if (b.lo[d] / 2 - 3 < prm.domain_lo[d] || (b.hi[d] + 1) / 2 - 1 + 3 > prm.domain_hi[d])
        return fail(c, CTUPPM_EINVAL, "fine boxes must lie at least 3 coarse cells inside the domain");
      flo[d] = std::min(flo[d], b.lo[d]);
      fhi[d] = std::max(fhi[d], b.hi[d]);
    }
  for (int d = 0; d < 3; ++d) {
    clo[d] = flo[d] / 2;
    chi[d] = (fhi[d] + 1) / 2 - 1;
  }
  return CTUPPM_OK;
}

// Coarse region of a two-level problem: coarse cells clo-3..chi+3 around the
// fine level's bounding box (the parents of every fine ghost cell and their
// neighbours).
long long region_cells(const Problem* P, int ext[3], int lo[3]) {
  long long v = 1;
  for (int d = 0; d < 3; ++d) {
    lo[d] = P->clo[d] - 3;
    ext[d] = P->chi[d] - P->clo[d] + 7;
    v *= ext[d];
  }
  return v;
}

// Workspace after the stage scratch of both levels: the region at t^n and at
// t^{n+1} (nv = 5 + nspec doubles per cell each), then 2 nv doubles per
// register face.
size_t two_level_extra_bytes(const Problem* P, long long nfaces) {
  if (P->nlevels != 2) return 0;
  int ext[3], lo[3];
  const long long rc = region_cells(P, ext, lo);
  const size_t nv = size_t(kNV + P->prm.nspec);
  return 2 * align256(size_t(rc) * nv * sizeof(double)) + align256(size_t(nfaces) * 2 * nv * sizeof(double));
}

// Forget the cached sets (and graphs) that involve problem pid.
void drop_sets(ctuppm_ctx* c, int pid) {
  bool graphs = false;
  for (auto& kv : c->sets) {
    const auto& v = std::get<0>(kv.first);
    if (std::find(v.begin(), v.end(), pid) != v.end() && kv.second->has_graph()) graphs = true;
  }
  if (c->two.count(pid) && c->two[pid]->exec) graphs = true;
  if (graphs) (void)hipStreamSynchronize(c->stream);  // an executable graph may still be running
  c->two.erase(pid);
  for (auto it = c->sets.begin(); it != c->sets.end();) {
    const auto& v = std::get<0>(it->first);
    if (std::find(v.begin(), v.end(), pid) != v.end()) it = c->sets.erase(it);
    else ++it;
  }
}

// The problem's tables must be rebuilt (binding, tuning or wave size changed).
void invalidate(ctuppm_ctx* c, Problem* P) {
  P->tables_ok = false;
  drop_sets(c, P->id);
}

// ------------------------------------------------------------ table builders

// Same-level ghost copies of level l (periodic images included), sorted by
// destination box, with their chunks; fpre gets each box's chunk range.
void fill_tags(const Problem* P, int l, std::vector<FillTag>& ft, std::vector<Chunk>& fch, std::vector<int>& fpre) {
  const auto& B = P->lev[l].boxes;
  const int nb = int(B.size());
  int dlo[3], dhi[3];
  level_domain(P->prm, l, dlo, dhi);
  int shifts[3][3];
  int nsh[3];
  for (int d = 0; d < 3; ++d) {
    const int len = dhi[d] - dlo[d] + 1;
    nsh[d] = 0;
    shifts[d][nsh[d]++] = 0;
    if (P->prm.bc_lo[d] == CTUPPM_BC_PERIODIC) {
      shifts[d][nsh[d]++] = len;
      shifts[d][nsh[d]++] = -len;
    }
  }
  ft.clear();
  for (int db = 0; db < nb; ++db) {
    const ctuppm_box& D = B[db];
    int glo[3], ghi[3];
    for (int d = 0; d < 3; ++d) {
      glo[d] = D.lo[d] - kNG;
      ghi[d] = D.hi[d] + kNG;
    }
    for (int sb = 0; sb < nb; ++sb) {
      const ctuppm_box& Sx = B[sb];
      for (int a = 0; a < nsh[0]; ++a)
        for (int bb = 0; bb < nsh[1]; ++bb)
          for (int cc = 0; cc < nsh[2]; ++cc) {
            const int sh[3] = {shifts[0][a], shifts[1][bb], shifts[2][cc]};
            if (sb == db && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) continue;
            // image of the source's valid cells, in the destination's frame
            int slo[3], shi[3], lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
              slo[d] = Sx.lo[d] - sh[d];
              shi[d] = Sx.hi[d] - sh[d];
            }
            if (!intersect(glo, ghi, slo, shi, lo, hi)) continue;
            FillTag t{};
            t.dst = db;
            t.src = sb;
            for (int d = 0; d < 3; ++d) {
              t.lo[d] = lo[d] - D.lo[d];
              t.ext[d] = hi[d] - lo[d] + 1;
              t.off[d] = D.lo[d] + sh[d] - Sx.lo[d];
            }
            ft.push_back(t);
          }
    }
  }
  // tags are generated destination by destination, so a box's chunks are contiguous
  fch.clear();
  fpre.assign(nb + 1, 0);
  for (size_t t = 0; t < ft.size(); ++t) {
    chunk_region(fch, int(t), (long long)ft[t].ext[0] * ft[t].ext[1] * ft[t].ext[2]);
    fpre[ft[t].dst + 1] = int(fch.size());
  }
  for (int b = 0; b < nb; ++b) fpre[b + 1] = std::max(fpre[b + 1], fpre[b]);
}

// Physical-boundary tags of level l along d, with chunks and per-box ranges.
void bc_tags(const Problem* P, int l, int d, std::vector<BcTag>& bt, std::vector<Chunk>& bch, std::vector<int>& bpre) {
  const auto& B = P->lev[l].boxes;
  const int nb = int(B.size());
  int dlo[3], dhi[3];
  level_domain(P->prm, l, dlo, dhi);
  const double rgm1 = 1.0 / (P->prm.gamma - 1.0);
  const double* s = P->prm.inflow;
  double inflow_cons[kMaxV];
  inflow_cons[0] = s[0];
  inflow_cons[1] = s[0] * s[1];
  inflow_cons[2] = s[0] * s[2];
  inflow_cons[3] = s[0] * s[3];
  inflow_cons[4] = s[4] * rgm1 + 0.5 * s[0] * ((s[1] * s[1] + s[2] * s[2]) + s[3] * s[3]);
  for (int sp = 0; sp < P->prm.nspec; ++sp) inflow_cons[kNV + sp] = s[0] * P->prm.inflow_X[sp];
  bt.clear();
  bch.clear();
  bpre.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    if (P->prm.bc_lo[d] != CTUPPM_BC_PERIODIC) {
      const ctuppm_box& Bx = B[b];
      for (int side = 0; side < 2; ++side) {
        BcTag t{};
        t.box = b;
        t.dir = d;
        t.side = side;
        t.bc = side == 0 ? P->prm.bc_lo[d] : P->prm.bc_hi[d];
        t.dom_lo = dlo[d];
        t.dom_hi = dhi[d];
        for (int m = 0; m < kNV + P->prm.nspec; ++m) t.inflow[m] = inflow_cons[m];
        bool any = true;
        long long vol = 1;
        for (int e = 0; e < 3; ++e) {
          int lo = -kNG, hi = box_n(Bx, e) + kNG - 1;  // box-local grown range
          if (e == d) {
            if (side == 0) hi = std::min(hi, dlo[d] - 1 - Bx.lo[d]);
            else lo = std::max(lo, dhi[d] + 1 - Bx.lo[d]);
          }
          if (lo > hi) any = false;
          t.lo[e] = lo;
          t.ext[e] = hi - lo + 1;
          vol *= std::max(0, t.ext[e]);
        }
        if (!any) continue;
        chunk_region(bch, int(bt.size()), vol);
        bt.push_back(t);
      }
    }
    bpre[b + 1] = int(bch.size());
  }
}

// Host tables of a two-level problem (box indices local to each level).
struct TwoHost {
  std::vector<GatherTag> gt;
  std::vector<Chunk> gch;
  std::vector<CfTag> ct;
  std::vector<Chunk> cch;
  std::vector<RegFace> rf;
  int fgrp[7] = {};
  std::vector<AvgTag> at;
  std::vector<Chunk> ach;
};

int find_box(const std::vector<ctuppm_box>& boxes, const int x[3]) {
  for (size_t b = 0; b < boxes.size(); ++b) {
    const ctuppm_box& B = boxes[b];
    if (x[0] >= B.lo[0] && x[0] <= B.hi[0] && x[1] >= B.lo[1] && x[1] <= B.hi[1] && x[2] >= B.lo[2] &&
        x[2] <= B.hi[2])
      return int(b);
  }
  return -1;
}

// Gather tags of the coarse boxes' valid cells inside region rlo..rlo+rext-1.
void gather_tags(const std::vector<ctuppm_box>& CB, const int rlo[3], const int rext[3], std::vector<GatherTag>& gt,
                 std::vector<Chunk>& gch) {
  int rhi[3];
  for (int d = 0; d < 3; ++d) rhi[d] = rlo[d] + rext[d] - 1;
  for (size_t b = 0; b < CB.size(); ++b) {
    int lo[3], hi[3];
    if (!intersect(CB[b].lo, CB[b].hi, rlo, rhi, lo, hi)) continue;
    GatherTag t{};
    t.box = int(b);
    long long vol = 1;
    for (int d = 0; d < 3; ++d) {
      t.lo[d] = lo[d] - CB[b].lo[d];
      t.ext[d] = hi[d] - lo[d] + 1;
      t.roff[d] = lo[d] - rlo[d];
      vol *= t.ext[d];
    }
    chunk_region(gch, int(gt.size()), vol);
    gt.push_back(t);
  }
}

// The coarse footprint (coarse cells under it) of a fine box.
ctuppm_box coarsen(const ctuppm_box& f) {
  ctuppm_box c{};
  for (int d = 0; d < 3; ++d) {
    c.lo[d] = f.lo[d] / 2;
    c.hi[d] = (f.hi[d] + 1) / 2 - 1;
  }
  return c;
}

int two_level_host(ctuppm_ctx* c, const Problem* P, TwoHost& H) {
  const auto& CB = P->lev[0].boxes;
  const auto& FB = P->lev[1].boxes;
  int rext[3], rlo[3];
  region_cells(P, rext, rlo);
  gather_tags(CB, rlo, rext, H.gt, H.gch);
  // coarse-to-fine: the ghost cells of each fine box that no fine box covers
  for (size_t b = 0; b < FB.size(); ++b) {
    ctuppm_box g = FB[b];
    for (int d = 0; d < 3; ++d) {
      g.lo[d] -= kNG;
      g.hi[d] += kNG;
    }
    for (const auto& piece : subtract_all(g, FB)) {
      CfTag t{};
      t.box = int(b);
      for (int d = 0; d < 3; ++d) {
        t.lo[d] = piece.lo[d] - FB[b].lo[d];
        t.ext[d] = box_n(piece, d);
      }
      chunk_region(H.cch, int(H.ct.size()), box_vol(piece));
      H.ct.push_back(t);
    }
  }
  // covered coarse cells (under some fine box), over the coarse bounding box
  int cext[3];
  for (int d = 0; d < 3; ++d) cext[d] = P->chi[d] - P->clo[d] + 1;
  std::vector<unsigned char> cov(size_t(cext[0]) * cext[1] * cext[2], 0);
  auto covered = [&](const int u[3]) {
    for (int d = 0; d < 3; ++d)
      if (u[d] < P->clo[d] || u[d] > P->chi[d]) return false;
    return cov[(size_t(u[2] - P->clo[2]) * cext[1] + (u[1] - P->clo[1])) * cext[0] + (u[0] - P->clo[0])] != 0;
  };
  for (const auto& f : FB) {
    const ctuppm_box cf = coarsen(f);
    for (int k = cf.lo[2]; k <= cf.hi[2]; ++k)
      for (int j = cf.lo[1]; j <= cf.hi[1]; ++j)
        for (int i = cf.lo[0]; i <= cf.hi[0]; ++i)
          cov[(size_t(k - P->clo[2]) * cext[1] + (j - P->clo[1])) * cext[0] + (i - P->clo[0])] = 1;
  }
  // register faces: coarse faces between an uncovered coarse cell and a
  // fine box, grouped by (direction, side of the fine level)
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    for (int side = 0; side < 2; ++side) {
      H.fgrp[2 * d + side] = int(H.rf.size());
      for (size_t fb = 0; fb < FB.size(); ++fb) {
        const ctuppm_box& Fb = FB[fb];
        const ctuppm_box cf = coarsen(Fb);
        const int cface = side == 0 ? cf.lo[d] : cf.hi[d] + 1;   // coarse face index along d
        const int uc = side == 0 ? cf.lo[d] - 1 : cf.hi[d] + 1;  // the outside coarse cell
        const int fface = side == 0 ? 0 : box_n(Fb, d);           // fine box-local face index
        for (int b2 = cf.lo[t2]; b2 <= cf.hi[t2]; ++b2)
          for (int b1 = cf.lo[t1]; b1 <= cf.hi[t1]; ++b1) {
            int u[3];
            u[d] = uc;
            u[t1] = b1;
            u[t2] = b2;
            if (covered(u)) continue;  // a face between two fine boxes
            RegFace F{};
            F.d = d;
            F.side = side;
            F.cbox = find_box(CB, u);
            F.fbox = int(fb);
            if (F.cbox < 0) return fail(c, CTUPPM_EINVAL, "coarse-fine face without a coarse box");
            const ctuppm_box& C = CB[F.cbox];
            for (int e = 0; e < 3; ++e) {
              F.ucell[e] = u[e] - C.lo[e];
              F.cface[e] = (e == d ? cface : u[e]) - C.lo[e];
            }
            F.fface[d] = fface;
            F.fface[t1] = 2 * b1 - Fb.lo[t1];
            F.fface[t2] = 2 * b2 - Fb.lo[t2];
            H.rf.push_back(F);
          }
      }
    }
  }
  H.fgrp[6] = int(H.rf.size());
  // average down: coarse cells covered by each fine box
  for (size_t cb = 0; cb < CB.size(); ++cb)
    for (size_t fb = 0; fb < FB.size(); ++fb) {
      const ctuppm_box cf = coarsen(FB[fb]);
      int lo[3], hi[3];
      if (!intersect(CB[cb].lo, CB[cb].hi, cf.lo, cf.hi, lo, hi)) continue;
      AvgTag t{};
      t.cbox = int(cb);
      t.fbox = int(fb);
      long long vol = 1;
      for (int d = 0; d < 3; ++d) {
        t.clo[d] = lo[d] - CB[cb].lo[d];
        t.ext[d] = hi[d] - lo[d] + 1;
        t.flo[d] = 2 * lo[d] - FB[fb].lo[d];
        vol *= t.ext[d];
      }
      chunk_region(H.ach, int(H.at.size()), vol);
      H.at.push_back(t);
    }
  return CTUPPM_OK;
}

// Bytes of the records at the start of a problem's workspace, and of the
// tables after them (the work lists sized for the tuning with the most units).
void meta_bytes(ctuppm_ctx* c, Problem* P) {
  P->rec_bytes = size_t(P->nlevels) * align256(sizeof(ProbDev));
  size_t t = 0;
  for (int l = 0; l < P->nlevels; ++l) {
    const auto& B = P->lev[l].boxes;
    t += kRecForms * packed<BoxRec>((long long)B.size());
    for (int k = 0; k < kNumRegions; ++k) {
      long long u = 0;
      for (const auto& b : B) {
        const int n[3] = {box_n(b, 0), box_n(b, 1), box_n(b, 2)};
        u += max_units(n, k);
      }
      t += kUnitVariants * packed<March>(u);
    }
    std::vector<FillTag> ft;
    std::vector<Chunk> fch;
    std::vector<int> pre;
    fill_tags(P, l, ft, fch, pre);
    t += packed<FillTag>((long long)ft.size()) + packed<Chunk>((long long)fch.size());
    for (int d = 0; d < 3; ++d) {
      std::vector<BcTag> bt;
      std::vector<Chunk> bch;
      bc_tags(P, l, d, bt, bch, pre);
      t += packed<BcTag>((long long)bt.size()) + packed<Chunk>((long long)bch.size());
    }
  }
  if (P->nlevels == 2) {
    TwoHost H;
    (void)two_level_host(c, P, H);
    P->nregf = (long long)H.rf.size();
    t += packed<GatherTag>((long long)H.gt.size()) + packed<Chunk>((long long)H.gch.size()) +
         packed<CfTag>((long long)H.ct.size()) + packed<Chunk>((long long)H.cch.size()) +
         packed<RegFace>((long long)H.rf.size()) + packed<AvgTag>((long long)H.at.size()) +
         packed<Chunk>((long long)H.ach.size());
  }
  P->tab_bytes = t;
}

size_t meta_total(const Problem* P) { return P->rec_bytes + P->tab_bytes; }

// Workspace offsets: the records and tables, the Runge-Kutta stage fabs (MOL),
// the stage scratch, the two-level region and register.
size_t scratch_base(const Problem* P) { return meta_total(P) + stage_fab_bytes(P->lev[0].boxes, P->prm); }

// Build the problem's device tables for the current binding, tuning and wave
// size, and upload them (asynchronously) into its workspace.
int ensure_tables(ctuppm_ctx* c, Problem* P) {
  if (P->tables_ok) return CTUPPM_OK;
  if (!P->ws) return fail(c, CTUPPM_ESTATE, "problem %d: no workspace bound", P->id);
  if (P->ws_bytes < meta_total(P))
    return fail(c, CTUPPM_ENOMEM, "problem %d: workspace %zu < %zu bytes of device tables", P->id, P->ws_bytes,
                meta_total(P));
  for (int l = 0; l < P->nlevels; ++l)
    if (!P->lev[l].bound) return fail(c, CTUPPM_ESTATE, "problem %d: level %d state not bound", P->id, l);
  Packer K;
  K.dbase = (char*)P->ws + P->rec_bytes;
  const int ns = P->prm.nspec;
  const size_t wbytes = stage_fab_bytes(P->lev[0].boxes, P->prm);
  const size_t sbase = scratch_base(P);
  size_t level_off = sbase;  // batched layout: every box its own scratch, level 1 after level 0
  for (int l = 0; l < P->nlevels; ++l) {
    const auto& B = P->lev[l].boxes;
    const Level& L = P->lev[l];
    LevelTables& T = P->lt[l];
    const int nb = int(B.size());
    int dlo[3], dhi[3];
    level_domain(P->prm, l, dlo, dhi);
    size_t slot = 0;  // waves form: every box fits any of the shared scratch slots
    for (const auto& b : B) slot = std::max(slot, box_scratch_bytes(b, ns));
    std::vector<BoxRec> recs[kRecForms];
    size_t off = level_off, woff = meta_total(P), soff = 0;
    for (int b = 0; b < nb; ++b) {
      BoxRec r{};
      r.U[0] = L.Ua[b];
      r.U[1] = L.Ub[b];
      r.P = level_rec(P, l);
      r.level = l;
      r.ns = ns;
      for (int w = 0; w < stage_fabs(P->prm); ++w)
        r.W[w] = (double*)((char*)P->ws + woff + size_t(w) * (wbytes / size_t(stage_fabs(P->prm))));
      woff += box_fab_bytes(B[b], ns);
      for (int d = 0; d < 3; ++d) {
        r.n[d] = box_n(B[b], d);
        r.lo[d] = B[b].lo[d];
        // reflecting domain walls on the box's faces (a fine level lies inside the domain)
        r.wall[d] = l == 0 ? ((B[b].lo[d] == dlo[d] && P->prm.bc_lo[d] == CTUPPM_BC_REFLECT ? 1 : 0) |
                              (B[b].hi[d] == dhi[d] && P->prm.bc_hi[d] == CTUPPM_BC_REFLECT ? 2 : 0))
                           : 0;
      }
      r.scr = (double*)((char*)P->ws + off);
      recs[0].push_back(r);
      r.scr = (double*)((char*)P->ws + sbase);
      recs[1].push_back(r);
      r.scr = (double*)((char*)P->ws + sbase + size_t(b % c->wave_boxes) * slot);
      recs[2].push_back(r);
      // the static array in the batched layout (used only when it all fits)
      r.scr = c->static_ptr && l == 0 ? (double*)((char*)c->static_ptr + soff) : nullptr;
      recs[3].push_back(r);
      soff += box_scratch_bytes(B[b], ns);
      off += box_scratch_bytes(B[b], ns);
    }
    level_off = off;
    for (int f = 0; f < kRecForms; ++f) T.recs[f] = K.put(recs[f]);
    const int zs[kUnitVariants] = {c->zseg_batched, c->zseg_per_box, c->zseg_batched};
    for (int z = 0; z < kUnitVariants; ++z)
      for (int k = 0; k < kNumRegions; ++k) {
        // variant 0: the per-stage planes; 1 (per box) and 2 (small batched
        // launches): one plane, two for cons->prim, unless the caller set the
        // stage's planes
        const int planes = z == 0 || c->region_set[k] ? c->region_planes[k] : (k == kGrown ? 2 : 1);
        std::vector<March> u;
        T.upre[z][k].assign(nb + 1, 0);
        long long cap = 0;
        for (int b = 0; b < nb; ++b) {
          int org[3], ext[3];
          region_of(k, recs[0][b].n, org, ext);
          march_region(u, b, org, ext, planes * zs[z], c->ytile);
          T.upre[z][k][b + 1] = int(u.size());
          cap += max_units(recs[0][b].n, k);
        }
        T.units[z][k] = K.put(u);
        K.reserve_bytes(packed<March>(cap) - packed<March>((long long)u.size()));
      }
    std::vector<FillTag> ft;
    std::vector<Chunk> fch;
    fill_tags(P, l, ft, fch, T.fpre);
    T.ftags = K.put(ft);
    T.fch = K.put(fch);
    for (int d = 0; d < 3; ++d) {
      std::vector<BcTag> bt;
      std::vector<Chunk> bch;
      bc_tags(P, l, d, bt, bch, T.bpre[d]);
      T.btags[d] = K.put(bt);
      T.bch[d] = K.put(bch);
    }
  }
  if (P->nlevels == 2) {
    TwoHost H;
    int rc = two_level_host(c, P, H);
    if (rc) return rc;
    TwoTables& W = P->tt;
    W.gtags = K.put(H.gt);
    W.gch = K.put(H.gch);
    W.ngch = int(H.gch.size());
    W.ctags = K.put(H.ct);
    W.cch = K.put(H.cch);
    W.ncch = int(H.cch.size());
    W.faces = K.put(H.rf);
    W.nfaces = int(H.rf.size());
    std::copy(H.fgrp, H.fgrp + 7, W.fgrp);
    W.atags = K.put(H.at);
    W.ach = K.put(H.ach);
    W.nach = int(H.ach.size());
    TwoLevelArgs& A = W.args;
    int rext[3], rlo[3];
    const long long rcells = region_cells(P, rext, rlo);
    const size_t nv = size_t(kNV + ns);
    char* base = (char*)P->ws + level_off;
    A.ct0 = (double*)base;
    A.ct1 = (double*)(base + align256(size_t(rcells) * nv * sizeof(double)));
    A.reg = (double*)(base + 2 * align256(size_t(rcells) * nv * sizeof(double)));
    A.cboxes = P->lt[0].recs[0];
    A.fboxes = P->lt[1].recs[0];
    A.Pc = P->dP;
    A.Pf = P->dPf;
    for (int d = 0; d < 3; ++d) {
      A.rlo[d] = rlo[d];
      A.rext[d] = rext[d];
    }
  }
  if (align256(K.buf.size()) > P->tab_bytes)
    return fail(c, CTUPPM_EINVAL, "problem %d: tables need %zu bytes, %zu reserved", P->id, K.buf.size(),
                P->tab_bytes);
  int rc = upload(c, K.dbase, K.buf.data(), K.buf.size());
  if (rc) return rc;
  P->tables_ok = true;
  return CTUPPM_OK;
}

// Upload the tables as soon as the state and the workspace are bound, so the
// steps that follow (ctuppm_step_static in particular) find them in place; a
// failure here is reported by the first step instead.
void eager_tables(ctuppm_ctx* c, Problem* P) {
  if (!P->ws) return;
  for (int l = 0; l < P->nlevels; ++l)
    if (!P->lev[l].bound) return;
  const std::string keep = c->err;
  if (ensure_tables(c, P) != CTUPPM_OK) c->err = keep;
}

// ---------------------------------------------------------------- step sets

// The set of problems `pids` stepped together in `form` on level `level`.
int build_set(ctuppm_ctx* c, const std::vector<int>& pids, int form, StepSet** out, int level = 0) {
  for (int pid : pids) {
    Problem* P = get_problem(c, pid);
    if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
    if (level >= P->nlevels) return fail(c, CTUPPM_EINVAL, "problem %d has no level %d", pid, level);
    if (!P->lev[level].bound || !P->ws)
      return fail(c, CTUPPM_ESTATE, "problem %d: state or workspace not bound", pid);
    size_t need = scratch_base(P);  // the static form's scratch is the library's
    if (form != kFormStatic && ctuppm_workspace_bytes(c, pid, form, &need) != CTUPPM_OK) return CTUPPM_EINVAL;
    if (P->ws_bytes < need)
      return fail(c, CTUPPM_ENOMEM, "problem %d: workspace %zu < %zu bytes", pid, P->ws_bytes, need);
    const int rc = ensure_tables(c, P);
    if (rc) return rc;
  }
  auto key = std::make_tuple(pids, form == CTUPPM_FORM_GRAPH ? CTUPPM_FORM_BATCHED : form, level);
  auto it = c->sets.find(key);
  if (it != c->sets.end()) {
    *out = it->second.get();
    return CTUPPM_OK;
  }
  std::unique_ptr<StepSet> S(new StepSet);
  S->pids = pids;
  S->form = std::get<1>(key);
  S->level = level;
  S->box_off.push_back(0);
  for (size_t ip = 0; ip < pids.size(); ++ip) {
    Problem* P = get_problem(c, pids[ip]);
    const int var = P->prm.limiter == CTUPPM_LIMITER_CS ? 1 : (P->prm.steepen ? 2 : 0);
    if (ip == 0) {
      S->scheme = P->prm.scheme;
      S->riemann = P->prm.riemann;
      S->limiter = var;
    }
    if (P->prm.scheme != S->scheme || P->prm.riemann != S->riemann || var != S->limiter)
      return fail(c, CTUPPM_EINVAL,
                  "problems stepped together must use the same scheme, Riemann solver and limiter");
    if (P->prm.nspec > 0) S->species = 1;
    S->probs.push_back(P);
    S->box_off.push_back(S->box_off.back() + int(P->lev[level].boxes.size()));
  }
  S->nboxes = S->box_off.back();
  // deep work units only when the set's launches keep kMinUnitsPerCu units per
  // CU at the depth of the merged tracing (a few small problems stepped alone
  // leave CUs idle with them; many stepped together do not)
  long long deep = 0;
  for (Problem* P : S->probs) deep += P->lt[level].upre[0][kCells1T].back();
  S->zvar = S->form == CTUPPM_FORM_PER_BOX ? 1 : (deep < (long long)kMinUnitsPerCu * c->num_cus ? 2 : 0);
  *out = S.get();
  c->sets[key] = std::move(S);
  return CTUPPM_OK;
}

// Cell stages of a CTU step after cons->prim: one kernel per direction, or
// (fused, the default) the flattening with the tracing of the three
// directions in one kernel and the first transverse stage of the three
// directions in another.  Both give the same bits.
const int kCellStagesSplit[] = {kStFlatten, kStTraceX, kStTraceY, kStTraceZ, kStRiemX, kStRiemY, kStRiemZ,
                                kStT1X, kStT1Y, kStT1Z, kStT2X, kStT2Y, kStT2Z, kStUpdate};
const int kCellStagesFused[] = {kStTrace3, kStSpec3, kStRiemX, kStRiemY, kStRiemZ, kStT1All,
                                kStT2X, kStT2Y, kStT2Z, kStUpdate};

std::vector<int> cell_stages(const ctuppm_ctx* c) {
  if (c->fused) return std::vector<int>(std::begin(kCellStagesFused), std::end(kCellStagesFused));
  return std::vector<int>(std::begin(kCellStagesSplit), std::end(kCellStagesSplit));
}

// Groups of boxes whose cell stages launch together: one per box (per-box
// form), all boxes (batched), or waves of wave_boxes consecutive boxes
// (waves form, the boxes of a wave use distinct scratch slots).
std::vector<std::pair<int, int>> box_groups(const ctuppm_ctx* c, const StepSet* S) {
  std::vector<std::pair<int, int>> g;
  const int w = S->form == CTUPPM_FORM_PER_BOX ? 1 : S->form == CTUPPM_FORM_WAVES ? c->wave_boxes : S->nboxes;
  for (int b = 0; b < S->nboxes; b += w) g.push_back({b, std::min(S->nboxes, b + w)});
  return g;
}

// Ghost fill of the state array `arr` of every box of a set: same-level
// copies, then the physical boundaries x, y, z (box by box in the per-box form).
int fill_arr(ctuppm_ctx* c, StepSet* S, hipStream_t s, bool timed, int arr) {
  StageArgs A;
  A.arr = arr;
  int rc;
  if (S->form == CTUPPM_FORM_PER_BOX) {
    for (int b = 0; b < S->nboxes; ++b)
      if ((rc = run_range(c, S, s, kStFill, b, b + 1, timed, A))) return rc;
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < S->nboxes; ++b)
        if ((rc = run_range(c, S, s, kStBcX + d, b, b + 1, timed, A))) return rc;
    return CTUPPM_OK;
  }
  for (int st = kStFill; st <= kStBcZ; ++st)
    if ((rc = run_all(c, S, s, st, timed, A))) return rc;
  return CTUPPM_OK;
}

// One method-of-lines step (SSP-RK2 or RK3): per stage a ghost fill of the
// stage's input, cons->prim (with the CFL reduction and dt in the first
// stage), flattening, edge-value face states and normal fluxes along x, y, z,
// and the stage update; the last stage writes the other fab.
int enqueue_mol(ctuppm_ctx* c, StepSet* S, hipStream_t s, bool timed, int guard) {
  const bool per_box = S->form == CTUPPM_FORM_PER_BOX;
  const int nst = S->scheme == 1 ? 2 : 3;
  // face states: flattening and the three directions in one kernel (fused,
  // the default) or one kernel each
  static const std::vector<int> fused = {kStRecon3, kStSpec3, kStRiemX, kStRiemY, kStRiemZ};
  static const std::vector<int> split = {kStFlatten, kStReconX, kStReconY, kStReconZ, kStRiemX, kStRiemY, kStRiemZ};
  const std::vector<int>& cells = c->fused ? fused : split;
  int rc;
  for (int r = 0; r < nst; ++r) {
    const int arr = r == 0 ? kArrCur : (r == 1 ? kArrW0 : kArrW1);
    if ((rc = fill_arr(c, S, s, timed, arr))) return rc;
    StageArgs A;
    A.arr = arr;
    if (r == 0) {
      if (per_box) {
        for (int b = 0; b < S->nboxes; ++b)
          if ((rc = run_range(c, S, s, kStCfl, b, b + 1, timed, A))) return rc;
      } else if ((rc = run_all(c, S, s, S->form == CTUPPM_FORM_WAVES ? kStCfl : kStC2P, timed, A))) {
        return rc;
      }
      if ((rc = run_probs(c, S, s, false, 0))) return rc;
    }
    StageArgs U;
    U.arr = arr;
    U.out = r == nst - 1 ? kArrNext : (r == 0 ? kArrW0 : kArrW1);
    U.comb = r > 0;
    U.c = nst == 2 ? 0.5 : (r == 1 ? 0.25 : 2.0 / 3.0);
    U.last = r == nst - 1;
    for (const auto& g : box_groups(c, S)) {
      // batched: the first stage's primitives came with the CFL pass
      if ((per_box || S->form == CTUPPM_FORM_WAVES || r > 0) &&
          (rc = run_range(c, S, s, kStC2POnly, g.first, g.second, timed, A)))
        return rc;
      for (int st : cells)
        if ((rc = run_range(c, S, s, st, g.first, g.second, timed))) return rc;
      if ((rc = run_range(c, S, s, kStMolUpdate, g.first, g.second, timed, U))) return rc;
    }
  }
  return run_probs(c, S, s, true, guard);
}

// Fork the two side streams off s (event slot k), and join them back.
int fork_side(ctuppm_ctx* c, hipStream_t s, int k) {
  HIPCHK(c, hipEventRecord(c->fj[k], s));
  for (auto& st : c->side) HIPCHK(c, hipStreamWaitEvent(st, c->fj[k], 0));
  return CTUPPM_OK;
}
int join_side(ctuppm_ctx* c, hipStream_t s, int k) {
  for (int i = 0; i < 2; ++i) {
    HIPCHK(c, hipEventRecord(c->fj[k + i], c->side[i]));
    HIPCHK(c, hipStreamWaitEvent(s, c->fj[k + i], 0));
  }
  return CTUPPM_OK;
}

// A CTU step of a set for graph capture, with the three directions of each
// phase on three streams: tracing and normal fluxes of x, y, z; the first
// transverse stage of x, y, z; the second of x, y, z.  Each phase reads only
// what the previous phases wrote, so the captured graph runs the directions
// concurrently (a tracing kernel's arithmetic overlaps another direction's
// memory traffic, and kernel tails overlap).
int enqueue_step_branched(ctuppm_ctx* c, StepSet* S, hipStream_t s, int guard) {
  int rc;
  if ((rc = fill_arr(c, S, s, false, kArrCur))) return rc;
  if ((rc = run_all(c, S, s, kStC2P, false))) return rc;
  if ((rc = run_probs(c, S, s, false, 0))) return rc;
  if ((rc = run_all(c, S, s, kStFlatten, false))) return rc;
  const hipStream_t str[3] = {s, c->side[0], c->side[1]};
  const int phases[3][2] = {{kStTraceX, kStRiemX}, {kStT1X, -1}, {kStT2X, -1}};
  for (int ph = 0; ph < 3; ++ph) {
    if ((rc = fork_side(c, s, 3 * ph))) return rc;
    for (int d = 0; d < 3; ++d)
      for (int q = 0; q < 2; ++q)
        if (phases[ph][q] >= 0 && (rc = run_all(c, S, str[d], phases[ph][q] + d, false))) return rc;
    if ((rc = join_side(c, s, 3 * ph + 1))) return rc;
  }
  if ((rc = run_all(c, S, s, kStUpdate, false))) return rc;
  return run_probs(c, S, s, true, guard);
}

// Enqueue one step of a set on stream s.
int enqueue_step(ctuppm_ctx* c, StepSet* S, hipStream_t s, bool timed, int guard) {
  if (S->scheme != 0) return enqueue_mol(c, S, s, timed, guard);
  const bool per_box = S->form == CTUPPM_FORM_PER_BOX;
  const bool waves = S->form == CTUPPM_FORM_WAVES;
  int rc;
  if ((rc = fill_arr(c, S, s, timed, kArrCur))) return rc;
  if (per_box) {
    for (int b = 0; b < S->nboxes; ++b)
      if ((rc = run_range(c, S, s, kStCfl, b, b + 1, timed))) return rc;
  } else if ((rc = run_all(c, S, s, waves ? kStCfl : kStC2P, timed))) {
    // the waves form converts each wave into its shared scratch right before
    // the wave's stages, so only the CFL pass runs over all boxes here
    return rc;
  }
  if ((rc = run_probs(c, S, s, false, 0))) return rc;
  for (const auto& g : box_groups(c, S)) {
    if ((per_box || waves) && (rc = run_range(c, S, s, kStC2POnly, g.first, g.second, timed))) return rc;
    for (int st : cell_stages(c))
      if ((rc = run_range(c, S, s, st, g.first, g.second, timed))) return rc;
  }
  return run_probs(c, S, s, true, guard);
}

// ------------------------------------------------------------------ two levels

#define TLCHK(expr)                                                                                \
  do {                                                                                             \
    hipError_t _e = (expr);                                                                        \
    if (_e != hipSuccess) return fail(c, CTUPPM_EHIP, "two-level launch %s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

int build_two_level(ctuppm_ctx* c, int pid, TwoLevel** out) {
  StepSet *cs = nullptr, *fs = nullptr;
  const std::vector<int> v{pid};
  int rc = build_set(c, v, CTUPPM_FORM_BATCHED, &cs, 0);
  if (!rc) rc = build_set(c, v, CTUPPM_FORM_BATCHED, &fs, 1);
  if (rc) return rc;
  auto it = c->two.find(pid);
  if (it == c->two.end()) {
    std::unique_ptr<TwoLevel> T(new TwoLevel);
    it = c->two.emplace(pid, std::move(T)).first;
  }
  it->second->cset = cs;
  it->second->fset = fs;
  *out = it->second.get();
  return CTUPPM_OK;
}

// Coarse-fine ghost interpolation of the fine level's current state at time
// fraction theta of the coarse step.
int cf_fill(ctuppm_ctx* c, Problem* P, hipStream_t s, double theta) {
  const TwoTables& W = P->tt;
  TLCHK(launch_cfinterp(W.args, W.ctags, W.cch, W.ncch, theta, s));
  return CTUPPM_OK;
}

// Reflux the coarse cells beside the fine level, one face group after another
// (x low, x high, y low, ... side of the fine level), so a coarse cell beside
// the fine level on several sides takes its corrections in that order.  The
// reflux kernel finds a face's register slot by its position in the list it
// is given, so each group's launch gets the register from the group's first
// slot on.
int reflux_groups(ctuppm_ctx* c, Problem* P, hipStream_t s) {
  const TwoTables& W = P->tt;
  const int nv = kNV + P->prm.nspec;
  for (int g = 0; g < 6; ++g) {
    TwoLevelArgs A = W.args;
    A.reg = W.args.reg + size_t(2 * nv) * size_t(W.fgrp[g]);
    TLCHK(launch_reflux(A, W.faces + W.fgrp[g], W.fgrp[g + 1] - W.fgrp[g], s));
  }
  return CTUPPM_OK;
}

// One coarse step of a two-level problem: coarse advance, two fine substeps
// with coarse-to-fine ghost cells at theta = 0 and 1/2, average down, reflux.
int enqueue_two_level(ctuppm_ctx* c, Problem* P, TwoLevel* T, hipStream_t s, bool timed) {
  StepSet* C = T->cset;
  StepSet* F = T->fset;
  const TwoTables& W = P->tt;
  const TwoLevelArgs& A = W.args;
  int rc;
  if ((rc = fill_arr(c, C, s, timed, kArrCur))) return rc;
  if ((rc = run_all(c, C, s, kStC2P, timed))) return rc;
  if ((rc = run_all(c, F, s, kStCfl, timed))) return rc;
  TLCHK(launch_dt2(P->dP, P->dPf, s));
  TLCHK(launch_gather(A, W.gtags, W.gch, W.ngch, 0, s));
  for (int st : cell_stages(c))
    if ((rc = run_all(c, C, s, st, timed))) return rc;
  TLCHK(launch_reg_coarse(A, W.faces, W.nfaces, s));
  TLCHK(launch_gather(A, W.gtags, W.gch, W.ngch, 1, s));
  for (int sub = 0; sub < 2; ++sub) {
    if ((rc = fill_arr(c, F, s, timed, kArrCur))) return rc;
    if ((rc = cf_fill(c, P, s, sub == 0 ? 0.0 : 0.5))) return rc;
    if ((rc = run_all(c, F, s, kStC2POnly, timed))) return rc;
    for (int st : cell_stages(c))
      if ((rc = run_all(c, F, s, st, timed))) return rc;
    TLCHK(launch_reg_fine(A, W.faces, W.nfaces, s));
    if ((rc = run_probs(c, F, s, true, 0))) return rc;
  }
  TLCHK(launch_avgdown(A, W.atags, W.ach, W.nach, s));
  if ((rc = reflux_groups(c, P, s))) return rc;
  return run_probs(c, C, s, true, 0);
}

int step_two_level(ctuppm_ctx* c, int pid, int form) {
  Problem* P = get_problem(c, pid);
  if (form == CTUPPM_FORM_PER_BOX || form == CTUPPM_FORM_WAVES)
    return fail(c, CTUPPM_EINVAL, "two-level problems step in the batched forms only");
  TwoLevel* T = nullptr;
  int rc = build_two_level(c, pid, &T);
  if (rc) return rc;
  if (form == CTUPPM_FORM_GRAPH) {
    if (!T->exec) {
      HIPCHK(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
      rc = enqueue_two_level(c, P, T, c->capture, false);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->capture, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "graph capture: %s", hipGetErrorString(e));
      T->graph = g;
      HIPCHK(c, hipGraphInstantiate(&T->exec, g, nullptr, nullptr, 0));
    }
    HIPCHK(c, hipGraphLaunch(T->exec, c->stream));
  } else {
    rc = enqueue_two_level(c, P, T, c->stream, c->timing);
    if (rc) return rc;
  }
  P->cur ^= 1;
  P->steps += 1;
  P->state_changed();
  return CTUPPM_OK;
}

// ------------------------------------------------------------ a step in pieces

#define LCHK(expr)                                                                                  \
  do {                                                                                              \
    hipError_t _e = (expr);                                                                         \
    if (_e != hipSuccess) return fail(c, CTUPPM_EHIP, "launch %s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// The problem of a piece call, and the form its launches take.
int piece_problem(ctuppm_ctx* c, int pid, int form, Problem** out) {
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (P->prm.scheme != CTUPPM_SCHEME_CTU)
    return fail(c, CTUPPM_EINVAL, "problem %d: the method-of-lines schemes step with ctuppm_step only", pid);
  if (form != CTUPPM_FORM_PER_BOX && form != CTUPPM_FORM_BATCHED && form != CTUPPM_FORM_WAVES)
    return fail(c, CTUPPM_EINVAL, "a step in pieces takes the per-box, batched or waves form");
  if (P->nlevels == 2 && form != CTUPPM_FORM_BATCHED)
    return fail(c, CTUPPM_EINVAL, "two-level problems step in the batched form");
  *out = P;
  return CTUPPM_OK;
}

int single_set(ctuppm_ctx* c, int pid, int form, StepSet** S) {
  const std::vector<int> v{pid};
  return build_set(c, v, form, S);
}

// The CFL pass over the valid cells of a single-level set, box by box in the per-box form.
int cfl_pass(ctuppm_ctx* c, StepSet* S, hipStream_t s) {
  if (S->form != CTUPPM_FORM_PER_BOX) return run_all(c, S, s, kStCfl, c->timing);
  for (int b = 0; b < S->nboxes; ++b) {
    const int rc = run_range(c, S, s, kStCfl, b, b + 1, c->timing);
    if (rc) return rc;
  }
  return CTUPPM_OK;
}

// cons->prim and the cell stages of a level, box by box in the per-box form.
int advance_cells(ctuppm_ctx* c, StepSet* S, hipStream_t s) {
  for (const auto& g : box_groups(c, S)) {
    int rc = run_range(c, S, s, kStC2POnly, g.first, g.second, c->timing);
    for (int st : cell_stages(c)) {
      if (rc) break;
      rc = run_range(c, S, s, st, g.first, g.second, c->timing);
    }
    if (rc) return rc;
  }
  return CTUPPM_OK;
}

// ------------------------------------------------------------- host flags

int take_slot(ctuppm_ctx* c) {
  for (auto it = c->parked_slots.begin(); it != c->parked_slots.end(); ++it)
    if (hipEventQuery(it->second) == hipSuccess) {
      c->free_slots.push_back(it->first);
      c->event_pool.push_back(it->second);
      c->parked_slots.erase(it);
      break;
    }
  if (c->free_slots.empty()) return -1;
  const int s = c->free_slots.back();
  c->free_slots.pop_back();
  return s;
}

// Rejections of guarded steps the device has reported for P (host-mapped,
// read without synchronising).
int host_rejections(const ctuppm_ctx* c, const Problem* P) {
  return __atomic_load_n(&c->hflags[P->hslot], __ATOMIC_ACQUIRE);
}

// Re-read the committed parity and step count of level 0 after guarded steps
// (synchronises).
int sync_mirror(ctuppm_ctx* c, Problem* P) {
  if (!P->guarded || !P->ws) return CTUPPM_OK;
  ProbDev h;
  int rc = download(c, &h, P->dP, sizeof(ProbDev));
  if (rc) return rc;
  P->cur = h.cur;
  P->steps = h.nsteps;
  P->guarded = false;
  return CTUPPM_OK;
}

// Write one field of a problem's device record (and keep it in the template).
template <class T>
int set_field(ctuppm_ctx* c, Problem* P, int level, T ProbDev::*field, T v) {
  P->tmpl[level].*field = v;
  if (!P->ws) return CTUPPM_OK;
  ProbDev* d = level_rec(P, level);
  return upload(c, &(d->*field), &v, sizeof(T));
}

// One single-level step (any form) with the guard on: enqueue and return.
int step_set(ctuppm_ctx* c, const std::vector<int>& v, int form, int guard) {
  StepSet* S = nullptr;
  int rc = build_set(c, v, form, &S);
  if (rc) return rc;
  if (form == CTUPPM_FORM_GRAPH) {
    if (!S->exec[guard]) {
      HIPCHK(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
      rc = (c->concurrent && S->scheme == 0) ? enqueue_step_branched(c, S, c->capture, guard)
                                             : enqueue_step(c, S, c->capture, false, guard);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->capture, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "graph capture: %s", hipGetErrorString(e));
      S->graph[guard] = g;
      HIPCHK(c, hipGraphInstantiate(&S->exec[guard], g, nullptr, nullptr, 0));
    }
    HIPCHK(c, hipGraphLaunch(S->exec[guard], c->stream));
  } else {
    rc = enqueue_step(c, S, c->stream, c->timing, guard);
    if (rc) return rc;
  }
  for (int pid : v) {
    Problem* P = get_problem(c, pid);
    P->cur ^= 1;
    P->steps += 1;
    if (guard) P->guarded = true;  // the mirror holds only if no step is rejected
    P->state_changed();
  }
  return CTUPPM_OK;
}

// Validate a list of problems for a step; 1 in *two for a lone two-level problem.
int check_step_list(ctuppm_ctx* c, const int* pids, int npids, int form, std::vector<int>& v, int* two) {
  if (!pids || npids < 1) return fail(c, CTUPPM_EINVAL, "no problems");
  if (form < CTUPPM_FORM_PER_BOX || form > CTUPPM_FORM_WAVES) return fail(c, CTUPPM_EINVAL, "unknown form %d", form);
  v.assign(pids, pids + npids);
  *two = 0;
  for (size_t i = 0; i < v.size(); ++i) {
    for (size_t j = 0; j < i; ++j)
      if (v[i] == v[j]) return fail(c, CTUPPM_EINVAL, "problem %d listed twice", v[i]);
    Problem* P = get_problem(c, v[i]);
    if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", v[i]);
    if (P->phase != 0)
      return fail(c, CTUPPM_ESTATE, "problem %d is in the middle of a step taken in pieces", v[i]);
    if (P->nlevels == 2) {
      if (npids != 1) return fail(c, CTUPPM_EINVAL, "a two-level problem steps on its own");
      *two = 1;
    }
  }
  return CTUPPM_OK;
}

}  // namespace

// ======================================================================== ABI

extern "C" {

int ctuppm_ctx_create(void* hip_stream, ctuppm_ctx** out) {
  if (!out) return CTUPPM_EINVAL;
  *out = nullptr;
  std::unique_ptr<ctuppm_ctx> c(new ctuppm_ctx);
  c->stream = (hipStream_t)hip_stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CTUPPM_EHIP;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    c->num_cus = cus;
  if (hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) return CTUPPM_EHIP;
  for (auto& st : c->side)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return CTUPPM_EHIP;
  for (auto& e : c->fj)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return CTUPPM_EHIP;
  void* h = nullptr;
  if (hipHostMalloc(&h, kMaxProblems * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return CTUPPM_EHIP;
  c->hflags = (int*)h;
  std::memset(h, 0, kMaxProblems * sizeof(int));
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) return CTUPPM_EHIP;
  c->dflags = (int*)d;
  for (int s = kMaxProblems - 1; s >= 0; --s) c->free_slots.push_back(s);
  if (static_scratch(dev, &c->static_ptr) != hipSuccess) return CTUPPM_EHIP;
  *out = c.release();
  return CTUPPM_OK;
}

int ctuppm_ctx_destroy(ctuppm_ctx* c) {
  if (!c) return CTUPPM_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  c->two.clear();
  c->sets.clear();
  c->probs.clear();
  for (auto& t : c->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  for (auto& p : c->parked_slots) (void)hipEventDestroy(p.second);
  for (auto& b : c->staging) {
    (void)hipEventDestroy(b.done);
    (void)hipHostFree(b.host);
  }
  if (c->hflags) (void)hipHostFree(c->hflags);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  for (auto& st : c->side)
    if (st) (void)hipStreamDestroy(st);
  for (auto& e : c->fj)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return CTUPPM_OK;
}

const char* ctuppm_last_error(ctuppm_ctx* c) { return c ? c->err.c_str() : "null context"; }

int ctuppm_fab_elems(const ctuppm_box* b, int nspec, long long* elems) {
  if (!b || !elems || nspec < 0 || nspec > kMaxSpec) return CTUPPM_EINVAL;
  long long v = kNV + nspec;
  for (int d = 0; d < 3; ++d) {
    const int n = b->hi[d] - b->lo[d] + 1;
    if (n < 1) return CTUPPM_EINVAL;
    v *= n + 2 * kNG;
  }
  *elems = v;
  return CTUPPM_OK;
}

int ctuppm_problem_create(ctuppm_ctx* c, const ctuppm_params* prm, int nlevels, const ctuppm_box* const* boxes,
                          const int* nboxes, int* pid_out) {
  if (!c || !prm || !boxes || !nboxes || !pid_out) return CTUPPM_EINVAL;
  if (nlevels != 1 && nlevels != 2) return fail(c, CTUPPM_EINVAL, "nlevels must be 1 or 2");
  if (!(prm->gamma > 1.0)) return fail(c, CTUPPM_EINVAL, "gamma must be > 1");
  if (prm->nspec < 0 || prm->nspec > kMaxSpec)
    return fail(c, CTUPPM_EINVAL, "nspec must be in 0..%d", kMaxSpec);
  if (prm->scheme < CTUPPM_SCHEME_CTU || prm->scheme > CTUPPM_SCHEME_MOL_RK3)
    return fail(c, CTUPPM_EINVAL, "unknown scheme %d", prm->scheme);
  if (prm->riemann != CTUPPM_RIEMANN_HLLC && prm->riemann != CTUPPM_RIEMANN_TWO_SHOCK)
    return fail(c, CTUPPM_EINVAL, "unknown Riemann solver %d", prm->riemann);
  if (prm->limiter != CTUPPM_LIMITER_CW84 && prm->limiter != CTUPPM_LIMITER_CS)
    return fail(c, CTUPPM_EINVAL, "unknown limiter %d", prm->limiter);
  if (prm->steepen != 0 && prm->steepen != 1) return fail(c, CTUPPM_EINVAL, "steepen must be 0 or 1");
  if (prm->steepen && prm->limiter != CTUPPM_LIMITER_CW84)
    return fail(c, CTUPPM_EINVAL, "contact steepening goes with the CW84 limiter");
  if (prm->scheme != CTUPPM_SCHEME_CTU && nlevels != 1)
    return fail(c, CTUPPM_EINVAL, "the method-of-lines schemes are single-level");
  for (int d = 0; d < 3; ++d) {
    if (!(prm->dx[d] > 0.0)) return fail(c, CTUPPM_EINVAL, "dx must be > 0");
    if (prm->domain_hi[d] < prm->domain_lo[d]) return fail(c, CTUPPM_EINVAL, "empty domain");
    const bool plo = prm->bc_lo[d] == CTUPPM_BC_PERIODIC, phi = prm->bc_hi[d] == CTUPPM_BC_PERIODIC;
    if (plo != phi) return fail(c, CTUPPM_EINVAL, "direction %d periodic on one side only", d);
    if (plo && prm->domain_hi[d] - prm->domain_lo[d] + 1 < kNG)
      return fail(c, CTUPPM_EINVAL, "periodic extent along %d below %d cells", d, kNG);
    for (int s = 0; s < 2; ++s) {
      const int bc = s ? prm->bc_hi[d] : prm->bc_lo[d];
      if (bc < 0 || bc > 3) return fail(c, CTUPPM_EINVAL, "unknown boundary condition %d", bc);
    }
  }
  std::unique_ptr<Problem> P(new Problem);
  P->prm = *prm;
  P->nlevels = nlevels;
  for (int l = 0; l < nlevels; ++l) {
    if (nboxes[l] < 1 || !boxes[l]) return fail(c, CTUPPM_EINVAL, "level %d has no boxes", l);
    const int rc = check_level(c, *prm, l, boxes[l], nboxes[l]);
    if (rc) return rc;
    P->lev[l].boxes.assign(boxes[l], boxes[l] + nboxes[l]);
  }
  if (nlevels == 2) {
    const int rc = fine_geometry(c, *prm, P->lev[1].boxes, P->flo, P->fhi, P->clo, P->chi);
    if (rc) return rc;
  }
  const int slot = take_slot(c);
  if (slot < 0) return fail(c, CTUPPM_EINVAL, "more than %d problems on one context", kMaxProblems);
  ProbDev& h = P->tmpl[0];
  h.gamma = prm->gamma;
  h.gm1 = prm->gamma - 1.0;
  h.rgm1 = 1.0 / (prm->gamma - 1.0);
  h.cfl = prm->cfl;
  h.small_dens = prm->small_dens;
  h.small_pres = prm->small_pres;
  h.grav_z = prm->grav_z;
  for (int d = 0; d < 3; ++d) {
    h.dx[d] = prm->dx[d];
    h.rdx[d] = 1.0 / prm->dx[d];
  }
  h.nlevels = nlevels;
  h.nspec = prm->nspec;
  h.scheme = prm->scheme;
  h.riemann = prm->riemann;
  h.limiter = prm->limiter;
  h.steepen = prm->steepen;
  h.fail_step = -1;
  h.hflag = c->dflags + slot;
  if (nlevels == 2) {
    P->tmpl[1] = h;
    for (int d = 0; d < 3; ++d) {
      P->tmpl[1].dx[d] = prm->dx[d] / 2.0;
      P->tmpl[1].rdx[d] = 1.0 / P->tmpl[1].dx[d];
    }
    P->tmpl[1].hflag = nullptr;
  }
  P->hslot = slot;
  c->hflags[slot] = 0;
  meta_bytes(c, P.get());
  P->id = c->next_id++;
  *pid_out = P->id;
  c->probs[P->id] = std::move(P);
  return CTUPPM_OK;
}

int ctuppm_problem_destroy(ctuppm_ctx* c, int pid) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  drop_sets(c, pid);
  // the flag slot is reused once the stream has passed every step enqueued so far
  hipEvent_t e = take_event(c);
  if (e && hipEventRecord(e, c->stream) == hipSuccess) c->parked_slots.push_back({P->hslot, e});
  c->probs.erase(pid);
  return CTUPPM_OK;
}

int ctuppm_workspace_bytes(ctuppm_ctx* c, int pid, int form, size_t* bytes) {
  if (!c || !bytes) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  size_t total = 0, mx = 0;
  for (int l = 0; l < P->nlevels; ++l)
    for (const auto& b : P->lev[l].boxes) {
      const size_t s = box_scratch_bytes(b, P->prm.nspec);
      total += s;
      mx = std::max(mx, s);
    }
  const size_t base = scratch_base(P);
  if (form == CTUPPM_FORM_PER_BOX) {
    if (P->nlevels == 2) return fail(c, CTUPPM_EINVAL, "two-level problems step in the batched forms only");
    *bytes = base + mx;
  } else if (form == CTUPPM_FORM_BATCHED || form == CTUPPM_FORM_GRAPH) {
    *bytes = base + total + two_level_extra_bytes(P, P->nregf);
  } else if (form == CTUPPM_FORM_WAVES) {
    if (P->nlevels == 2) return fail(c, CTUPPM_EINVAL, "two-level problems step in the batched forms only");
    *bytes = base + std::min(size_t(c->wave_boxes), P->lev[0].boxes.size()) * mx;
  } else {
    return fail(c, CTUPPM_EINVAL, "unknown form %d", form);
  }
  return CTUPPM_OK;
}

int ctuppm_workspace_meta_bytes(ctuppm_ctx* c, int pid, size_t* bytes) {
  if (!c || !bytes) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  *bytes = meta_total(P);
  return CTUPPM_OK;
}

int ctuppm_bind_state(ctuppm_ctx* c, int pid, int level, double* const* Ua, double* const* Ub) {
  if (!c || !Ua || !Ub) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (level < 0 || level >= P->nlevels) return fail(c, CTUPPM_EINVAL, "bad level %d", level);
  if (P->phase != 0) return fail(c, CTUPPM_ESTATE, "problem %d is in the middle of a step taken in pieces", pid);
  Level& L = P->lev[level];
  for (size_t b = 0; b < L.boxes.size(); ++b)
    if (!Ua[b] || !Ub[b] || ((uintptr_t)Ua[b] & 7) || ((uintptr_t)Ub[b] & 7))
      return fail(c, CTUPPM_EINVAL, "box %zu: null or misaligned fab pointer", b);
  L.Ua.assign(Ua, Ua + L.boxes.size());
  L.Ub.assign(Ub, Ub + L.boxes.size());
  L.bound = true;
  if (level == 0) {
    P->cur = 0;
    P->guarded = false;
  }
  invalidate(c, P);
  P->state_changed();
  // parity back to A (asynchronous, after everything enqueued before)
  const int rc = set_field(c, P, level, &ProbDev::cur, 0);
  if (rc) return rc;
  eager_tables(c, P);
  return CTUPPM_OK;
}

int ctuppm_bind_workspace(ctuppm_ctx* c, int pid, void* ws, size_t bytes) {
  if (!c || !ws) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if ((uintptr_t)ws & 255) return fail(c, CTUPPM_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < meta_total(P))
    return fail(c, CTUPPM_ENOMEM, "workspace %zu < %zu bytes of device tables", bytes, meta_total(P));
  if (P->phase != 0) return fail(c, CTUPPM_ESTATE, "problem %d is in the middle of a step taken in pieces", pid);
  void* old = P->ws;
  const size_t rb = align256(sizeof(ProbDev));
  if (old && old != ws) {
    // the problem's live records (parity, counters, dt) move with it
    HIPCHK(c, hipMemcpyAsync(ws, old, size_t(P->nlevels) * rb, hipMemcpyDeviceToDevice, c->stream));
  } else if (!old) {
    for (int l = 0; l < P->nlevels; ++l) {
      P->tmpl[l].cur = 0;
      const int rc = upload(c, (char*)ws + size_t(l) * rb, &P->tmpl[l], sizeof(ProbDev));
      if (rc) return rc;
    }
  }
  P->ws = ws;
  P->ws_bytes = bytes;
  P->dP = (ProbDev*)ws;
  P->dPf = P->nlevels == 2 ? (ProbDev*)((char*)ws + rb) : nullptr;
  invalidate(c, P);
  eager_tables(c, P);
  return CTUPPM_OK;
}

int ctuppm_set_fixed_dt(ctuppm_ctx* c, int pid, double dt) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  return set_field(c, P, 0, &ProbDev::fixed_dt, dt > 0.0 ? dt : 0.0);
}

int ctuppm_step(ctuppm_ctx* c, const int* pids, int npids, int form) {
  if (!c) return CTUPPM_EINVAL;
  std::vector<int> v;
  int two = 0;
  int rc = check_step_list(c, pids, npids, form, v, &two);
  if (rc) return rc;
  if (two) return step_two_level(c, v[0], form);
  return step_set(c, v, form, 0);
}

int ctuppm_step_guarded(ctuppm_ctx* c, const int* pids, int npids, int form) {
  if (!c) return CTUPPM_EINVAL;
  std::vector<int> v;
  int two = 0;
  int rc = check_step_list(c, pids, npids, form, v, &two);
  if (rc) return rc;
  if (two) return fail(c, CTUPPM_EINVAL, "guarded steps are for single-level problems");
  for (int pid : v) {
    Problem* P = get_problem(c, pid);
    if (host_rejections(c, P) != P->acked)
      return fail(c, CTUPPM_ERETRY, "problem %d: a guarded step was rejected (acknowledge with ctuppm_rejections)",
                  pid);
  }
  return step_set(c, v, form, 1);
}

int ctuppm_step_static(ctuppm_ctx* c, int pid) {
  if (!c) return CTUPPM_EINVAL;
  std::vector<int> v;
  int two = 0;
  int rc = check_step_list(c, &pid, 1, CTUPPM_FORM_BATCHED, v, &two);
  if (rc) return rc;
  if (two) return fail(c, CTUPPM_EINVAL, "the static step is for single-level problems");
  Problem* P = get_problem(c, pid);
  size_t need = 0;
  for (const auto& b : P->lev[0].boxes) need += box_scratch_bytes(b, P->prm.nspec);
  if (need > kStaticScratchBytes)
    return fail(c, CTUPPM_EINVAL, "problem %d: stage scratch of %zu bytes exceeds the static %zu bytes", pid, need,
                kStaticScratchBytes);
  if (!c->static_ptr) return fail(c, CTUPPM_EHIP, "no static scratch on this device");
  if (!P->ws || !P->lev[0].bound) return fail(c, CTUPPM_ESTATE, "problem %d: state or workspace not bound", pid);
  if (!P->tables_ok)
    return fail(c, CTUPPM_ESTATE, "problem %d: device tables not uploaded (re-bind the workspace)", pid);
  return step_set(c, v, kFormStatic, 0);
}

int ctuppm_rejections(ctuppm_ctx* c, int pid, long long* rejected) {
  if (!c || !rejected) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (!P->ws) {
    *rejected = 0;
    return CTUPPM_OK;
  }
  ProbDev h;
  int rc = download(c, &h, P->dP, sizeof(ProbDev));
  if (rc) return rc;
  P->cur = h.cur;
  P->steps = h.nsteps;
  P->guarded = false;
  P->acked = h.rejected;
  *rejected = h.rejected;
  return CTUPPM_OK;
}

int ctuppm_rejections_seen(ctuppm_ctx* c, int pid, long long* rejected) {
  if (!c || !rejected) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  *rejected = host_rejections(c, P);
  P->acked = int(*rejected);
  return CTUPPM_OK;
}

int ctuppm_fill_ghosts(ctuppm_ctx* c, int pid, int level, int form) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = nullptr;
  int rc = piece_problem(c, pid, form, &P);
  if (rc) return rc;
  if (level < 0 || level >= P->nlevels) return fail(c, CTUPPM_EINVAL, "problem %d has no level %d", pid, level);
  if ((rc = sync_mirror(c, P))) return rc;
  if (P->nlevels == 1) {
    StepSet* S = nullptr;
    if ((rc = single_set(c, pid, form, &S)) || (rc = fill_arr(c, S, c->stream, c->timing, kArrCur))) return rc;
  } else {
    TwoLevel* T = nullptr;
    if ((rc = build_two_level(c, pid, &T))) return rc;
    if (level == 0) {
      if (P->phase != 0)
        return fail(c, CTUPPM_ESTATE, "problem %d: the coarse step is under way (fine substeps, average down, reflux)",
                    pid);
      if ((rc = fill_arr(c, T->cset, c->stream, c->timing, kArrCur))) return rc;
    } else {
      if (P->phase != 1 || P->fine_done >= 2)
        return fail(c, CTUPPM_ESTATE, "problem %d: fine ghost cells are filled after the coarse advance, before "
                    "each of the two fine substeps", pid);
      if ((rc = fill_arr(c, T->fset, c->stream, c->timing, kArrCur))) return rc;
      if ((rc = cf_fill(c, P, c->stream, 0.5 * P->fine_done))) return rc;
    }
  }
  P->filled[level] = true;
  return CTUPPM_OK;
}

int ctuppm_compute_dt(ctuppm_ctx* c, int pid, int form, double* dt_dev) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = nullptr;
  int rc = piece_problem(c, pid, form, &P);
  if (rc) return rc;
  if (P->phase != 0) return fail(c, CTUPPM_ESTATE, "problem %d: dt is computed between steps", pid);
  if (P->nlevels == 1) {
    StepSet* S = nullptr;
    if ((rc = single_set(c, pid, form, &S)) || (rc = cfl_pass(c, S, c->stream))) return rc;
    if ((rc = run_probs(c, S, c->stream, false, 0))) return rc;
  } else {
    TwoLevel* T = nullptr;
    if ((rc = build_two_level(c, pid, &T))) return rc;
    if ((rc = run_all(c, T->cset, c->stream, kStCfl, c->timing)) ||
        (rc = run_all(c, T->fset, c->stream, kStCfl, c->timing)))
      return rc;
    LCHK(launch_dt2(P->dP, P->dPf, c->stream));
  }
  if (dt_dev) HIPCHK(c, hipMemcpyAsync(dt_dev, &P->dP->dt, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  P->dt_ready = true;
  return CTUPPM_OK;
}

int ctuppm_advance_level(ctuppm_ctx* c, int pid, int level, int form, const double* dt_dev) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = nullptr;
  int rc = piece_problem(c, pid, form, &P);
  if (rc) return rc;
  if (level < 0 || level >= P->nlevels) return fail(c, CTUPPM_EINVAL, "problem %d has no level %d", pid, level);
  hipStream_t s = c->stream;
  if (level == 0) {
    if (P->phase != 0) return fail(c, CTUPPM_ESTATE, "problem %d: the coarse step is under way", pid);
    if (!P->filled[0])
      return fail(c, CTUPPM_ESTATE, "problem %d: level 0 ghost cells not filled since the state changed", pid);
    if (!dt_dev && !P->dt_ready) return fail(c, CTUPPM_ESTATE, "problem %d: no dt (compute it or pass one)", pid);
  }
  if (P->nlevels == 1) {
    StepSet* S = nullptr;
    if ((rc = single_set(c, pid, form, &S))) return rc;
    if (dt_dev) LCHK(launch_set_dt(P->dP, nullptr, dt_dev, s));
    if ((rc = advance_cells(c, S, s))) return rc;
    if ((rc = run_probs(c, S, s, true, 0))) return rc;
    P->cur ^= 1;
    P->steps += 1;
    P->state_changed();
    return CTUPPM_OK;
  }
  TwoLevel* T = nullptr;
  if ((rc = build_two_level(c, pid, &T))) return rc;
  const TwoTables& W = P->tt;
  const TwoLevelArgs& A = W.args;
  if (level == 0) {
    if (dt_dev) LCHK(launch_set_dt(P->dP, P->dPf, dt_dev, s));
    LCHK(launch_gather(A, W.gtags, W.gch, W.ngch, 0, s));
    if ((rc = advance_cells(c, T->cset, s))) return rc;
    LCHK(launch_reg_coarse(A, W.faces, W.nfaces, s));
    LCHK(launch_gather(A, W.gtags, W.gch, W.ngch, 1, s));
    P->phase = 1;
    P->fine_done = 0;
    P->state_changed();
    return CTUPPM_OK;
  }
  if (dt_dev) return fail(c, CTUPPM_EINVAL, "the fine level takes half the coarse dt (pass NULL)");
  if (P->phase != 1 || P->fine_done >= 2)
    return fail(c, CTUPPM_ESTATE, "problem %d: a fine substep follows the coarse advance, twice", pid);
  if (!P->filled[1])
    return fail(c, CTUPPM_ESTATE, "problem %d: level 1 ghost cells not filled for this substep", pid);
  if ((rc = advance_cells(c, T->fset, s))) return rc;
  LCHK(launch_reg_fine(A, W.faces, W.nfaces, s));
  if ((rc = run_probs(c, T->fset, s, true, 0))) return rc;
  P->fine_done += 1;
  P->filled[1] = false;
  return CTUPPM_OK;
}

int ctuppm_average_down(ctuppm_ctx* c, int pid) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (P->nlevels != 2) return fail(c, CTUPPM_EINVAL, "problem %d has one level", pid);
  if (P->phase != 1 || P->fine_done != 2 || P->averaged)
    return fail(c, CTUPPM_ESTATE, "problem %d: averaging down follows the second fine substep, once", pid);
  TwoLevel* T = nullptr;
  int rc = build_two_level(c, pid, &T);
  if (rc) return rc;
  const TwoTables& W = P->tt;
  LCHK(launch_avgdown(W.args, W.atags, W.ach, W.nach, c->stream));
  P->averaged = true;
  return CTUPPM_OK;
}

int ctuppm_reflux(ctuppm_ctx* c, int pid) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (P->nlevels != 2) return fail(c, CTUPPM_EINVAL, "problem %d has one level", pid);
  if (P->phase != 1 || !P->averaged)
    return fail(c, CTUPPM_ESTATE, "problem %d: refluxing follows averaging down", pid);
  TwoLevel* T = nullptr;
  int rc = build_two_level(c, pid, &T);
  if (rc) return rc;
  if ((rc = reflux_groups(c, P, c->stream))) return rc;
  if ((rc = run_probs(c, T->cset, c->stream, true, 0))) return rc;
  P->phase = 0;
  P->fine_done = 0;
  P->averaged = false;
  P->cur ^= 1;
  P->steps += 1;
  P->state_changed();
  return CTUPPM_OK;
}

}  // extern "C"

namespace {

// One guarded step of dt h (fixed), and on rejection the interval again in
// two halves, recursively to depth kMaxRetryDepth.  Synchronises after each
// step to read the verdict; *deepest records the deepest halving used.
int checked_interval(ctuppm_ctx* c, Problem* P, int form, double h, int depth, int* deepest) {
  int rc = set_field(c, P, 0, &ProbDev::fixed_dt, h);
  if (rc) return rc;
  const std::vector<int> v{P->id};
  if ((rc = step_set(c, v, form, 1))) return rc;
  long long rej = 0;
  const int before = P->acked;
  if ((rc = ctuppm_rejections(c, P->id, &rej))) return rc;
  if (rej == before) return CTUPPM_OK;
  if (depth == kMaxRetryDepth)
    return fail(c, CTUPPM_ERETRY, "problem %d: step still rejected after %d halvings", P->id, depth);
  *deepest = std::max(*deepest, depth + 1);
  for (int half = 0; half < 2; ++half)
    if ((rc = checked_interval(c, P, form, 0.5 * h, depth + 1, deepest))) return rc;
  return CTUPPM_OK;
}

}  // namespace

extern "C" {

int ctuppm_step_checked(ctuppm_ctx* c, int pid, int form, int* retried) {
  if (!c || !retried) return CTUPPM_EINVAL;
  *retried = 0;
  std::vector<int> v;
  int two = 0;
  int rc = check_step_list(c, &pid, 1, form, v, &two);
  if (rc) return rc;
  if (two) return fail(c, CTUPPM_EINVAL, "checked steps are for single-level problems");
  Problem* P = get_problem(c, pid);
  long long rej = 0;
  if ((rc = ctuppm_rejections(c, pid, &rej))) return rc;  // acknowledge earlier guarded steps
  if ((rc = step_set(c, v, form, 1))) return rc;
  const int before = P->acked;
  if ((rc = ctuppm_rejections(c, pid, &rej))) return rc;
  if (rej == before) return CTUPPM_OK;
  // rejected: U^n is still current; redo the interval of the rejected dt in halves
  ProbDev h;
  if ((rc = download(c, &h, P->dP, sizeof(ProbDev)))) return rc;
  const double keep = P->tmpl[0].fixed_dt;
  int deepest = 1;
  rc = CTUPPM_OK;
  for (int half = 0; half < 2 && !rc; ++half) rc = checked_interval(c, P, form, 0.5 * h.dt, 1, &deepest);
  *retried = deepest;
  const int rc2 = set_field(c, P, 0, &ProbDev::fixed_dt, keep);
  return rc ? rc : rc2;
}

int ctuppm_set_fail_hook(ctuppm_ctx* c, int pid, int step_index) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  return set_field(c, P, 0, &ProbDev::fail_step, step_index);
}

int ctuppm_current_state(ctuppm_ctx* c, int pid, int* which) {
  if (!c || !which) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  const int rc = sync_mirror(c, P);
  if (rc) return rc;
  *which = P->cur;
  return CTUPPM_OK;
}

int ctuppm_get_dt(ctuppm_ctx* c, int pid, double* dt) {
  if (!c || !dt) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (!P->ws) return fail(c, CTUPPM_ESTATE, "problem %d: no workspace bound", pid);
  return download(c, dt, &P->dP->dt, sizeof(double));
}

int ctuppm_status(ctuppm_ctx* c, int pid, long long counters[6]) {
  if (!c || !counters) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (!P->ws) {
    for (int i = 0; i < 6; ++i) counters[i] = 0;
    return CTUPPM_OK;
  }
  ProbDev h[2];
  int rc = download(c, h, P->dP, sizeof(ProbDev));
  if (!rc && P->dPf) rc = download(c, &h[1], P->dPf, sizeof(ProbDev));
  if (rc) return rc;
  for (int i = 0; i < 5; ++i) counters[i] = (long long)h[0].cnt[i] + (P->dPf ? (long long)h[1].cnt[i] : 0);
  counters[5] = h[0].nsteps;
  return CTUPPM_OK;
}

int ctuppm_set_timing(ctuppm_ctx* c, int on) {
  if (!c) return CTUPPM_EINVAL;
  c->timing = on != 0;
  return CTUPPM_OK;
}

int ctuppm_stage_times(ctuppm_ctx* c, double* ms, long long* launches, int n) {
  if (!c || !ms || !launches || n < 0 || n > kNumStages) return CTUPPM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& t : c->timed) {
    float v = 0.f;
    HIPCHK(c, hipEventElapsedTime(&v, t.a, t.b));
    c->acc_ms[t.stage] += v;
    c->acc_n[t.stage] += 1;
    c->event_pool.push_back(t.a);
    c->event_pool.push_back(t.b);
  }
  c->timed.clear();
  for (int s = 0; s < n; ++s) {
    ms[s] = c->acc_ms[s];
    launches[s] = c->acc_n[s];
    c->acc_ms[s] = 0.0;
    c->acc_n[s] = 0;
  }
  return CTUPPM_OK;
}

int ctuppm_num_stages(void) { return kNumStages; }
const char* ctuppm_stage_name(int s) { return stage_name(s); }

int ctuppm_tag(ctuppm_ctx* c, int pid, double threshold, unsigned char* tags) {
  if (!c || !tags || !(threshold >= 0.0)) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (P->phase != 0) return fail(c, CTUPPM_ESTATE, "problem %d is in the middle of a step taken in pieces", pid);
  int rc = sync_mirror(c, P);
  if (rc) return rc;
  StepSet* S = nullptr;
  const std::vector<int> v{pid};
  if ((rc = build_set(c, v, CTUPPM_FORM_BATCHED, &S, 0))) return rc;
  if ((rc = fill_arr(c, S, c->stream, false, kArrCur))) return rc;
  int dn[3];
  for (int d = 0; d < 3; ++d) dn[d] = P->prm.domain_hi[d] - P->prm.domain_lo[d] + 1;
  const LevelTables& T = P->lt[0];
  const int nu = T.upre[0][kValid].back();
  Segs G{};
  G.n = 1;
  G.s[0] = Seg{T.recs[0], T.units[0][kValid], nullptr, P->dP};
  G.beg[1] = nu;
  hipError_t e = launch_tag(G, grid_for(c, nu, false), threshold, tags, dn, P->prm.domain_lo, c->stream);
  if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "tag launch: %s", hipGetErrorString(e));
  return CTUPPM_OK;
}

int ctuppm_regrid(ctuppm_ctx* c, int pid, const ctuppm_box* fine_boxes, int nfine, double* const* Ua,
                  double* const* Ub) {
  if (!c || !fine_boxes || nfine < 1 || !Ua || !Ub) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (P->nlevels != 2) return fail(c, CTUPPM_EINVAL, "problem %d has no fine level", pid);
  if (!P->lev[0].bound || !P->lev[1].bound) return fail(c, CTUPPM_ESTATE, "problem %d: state not bound", pid);
  if (P->phase != 0) return fail(c, CTUPPM_ESTATE, "problem %d is in the middle of a step taken in pieces", pid);
  for (int b = 0; b < nfine; ++b)
    if (!Ua[b] || !Ub[b] || ((uintptr_t)Ua[b] & 7) || ((uintptr_t)Ub[b] & 7))
      return fail(c, CTUPPM_EINVAL, "null or misaligned fab for fine box %d", b);
  int rc = check_level(c, P->prm, 1, fine_boxes, nfine);
  if (rc) return rc;
  const std::vector<ctuppm_box> NB(fine_boxes, fine_boxes + nfine);
  int flo[3], fhi[3], clo[3], chi[3];
  if ((rc = fine_geometry(c, P->prm, NB, flo, fhi, clo, chi))) return rc;
  size_t need = 0;
  if ((rc = ctuppm_workspace_bytes(c, pid, CTUPPM_FORM_BATCHED, &need))) return rc;
  if (P->ws_bytes < need) return fail(c, CTUPPM_ENOMEM, "problem %d: workspace %zu < %zu bytes", pid, P->ws_bytes, need);
  if ((rc = ensure_tables(c, P))) return rc;
  // the coarse cells the interpolation reads: parents and their neighbours
  TwoLevelArgs A{};
  long long rcells = 1;
  for (int d = 0; d < 3; ++d) {
    A.rlo[d] = clo[d] - 1;
    A.rext[d] = chi[d] - clo[d] + 3;
    rcells *= A.rext[d];
  }
  std::vector<GatherTag> gt;
  std::vector<Chunk> gch;
  gather_tags(P->lev[0].boxes, A.rlo, A.rext, gt, gch);
  // new fine box records (fabs A/B of the caller), and the copy / interpolate tags
  const int ns = P->prm.nspec;
  std::vector<BoxRec> nrec(nfine);
  for (int b = 0; b < nfine; ++b) {
    BoxRec& r = nrec[b];
    r = BoxRec{};
    r.U[0] = Ua[b];
    r.U[1] = Ub[b];
    r.P = P->dPf;
    r.level = 1;
    r.ns = ns;
    for (int d = 0; d < 3; ++d) {
      r.n[d] = box_n(NB[b], d);
      r.lo[d] = NB[b].lo[d];
    }
  }
  const auto& OB = P->lev[1].boxes;
  std::vector<ProlongTag> pt;
  std::vector<Chunk> pch;
  auto add = [&](int box, int src, const int lo[3], const int hi[3]) {
    ProlongTag t{};
    t.box = box;
    t.src = src;
    long long vol = 1;
    for (int d = 0; d < 3; ++d) {
      t.lo[d] = lo[d] - NB[box].lo[d];
      t.ext[d] = hi[d] - lo[d] + 1;
      vol *= t.ext[d];
    }
    chunk_region(pch, int(pt.size()), vol);
    pt.push_back(t);
  };
  for (int b = 0; b < nfine; ++b) {
    // cells under an old fine box keep its values; the rest is interpolated
    for (size_t o = 0; o < OB.size(); ++o) {
      int ilo[3], ihi[3];
      if (intersect(NB[b].lo, NB[b].hi, OB[o].lo, OB[o].hi, ilo, ihi)) add(b, int(o), ilo, ihi);
    }
    for (const auto& piece : subtract_all(NB[b], OB)) add(b, -1, piece.lo, piece.hi);
  }
  // region and tables go in the stage scratch, unused between steps
  Packer K;
  const size_t rbytes = align256(size_t(rcells) * size_t(kNV + ns) * sizeof(double));
  K.dbase = (char*)P->ws + scratch_base(P) + rbytes;
  GatherTag* dgt = K.put(gt);
  Chunk* dgch = K.put(gch);
  ProlongTag* dpt = K.put(pt);
  Chunk* dpch = K.put(pch);
  BoxRec* dnrec = K.put(nrec);
  size_t scr = 0;
  for (const auto& b : P->lev[0].boxes) scr += box_scratch_bytes(b, ns);
  if (rbytes + align256(K.buf.size()) > scr)
    return fail(c, CTUPPM_ENOMEM, "problem %d: regrid needs %zu bytes of level-0 scratch, has %zu", pid,
                rbytes + K.buf.size(), scr);
  if ((rc = upload(c, K.dbase, K.buf.data(), K.buf.size()))) return rc;
  A.cboxes = P->lt[0].recs[0];
  A.fboxes = P->lt[1].recs[0];
  A.Pc = P->dP;
  A.Pf = P->dPf;
  A.ct0 = (double*)((char*)P->ws + scratch_base(P));
  hipError_t e = launch_gather(A, dgt, dgch, int(gch.size()), 0, c->stream);
  if (e == hipSuccess) e = launch_prolong(A, dnrec, A.fboxes, dpt, dpch, int(pch.size()), c->stream);
  if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "regrid launch: %s", hipGetErrorString(e));
  // the fine level's parity: the new state is in the A fabs
  if ((rc = set_field(c, P, 1, &ProbDev::cur, 0))) return rc;
  P->lev[1].boxes = NB;
  P->lev[1].Ua.assign(Ua, Ua + nfine);
  P->lev[1].Ub.assign(Ub, Ub + nfine);
  P->lev[1].bound = true;
  for (int d = 0; d < 3; ++d) {
    P->flo[d] = flo[d];
    P->fhi[d] = fhi[d];
    P->clo[d] = clo[d];
    P->chi[d] = chi[d];
  }
  // the tables grow or shrink with the fine level: the workspace is re-bound
  // next (its records move with it); until then the old one stays bound
  meta_bytes(c, P);
  invalidate(c, P);
  P->state_changed();
  return CTUPPM_OK;
}

int ctuppm_debug_stage(ctuppm_ctx* c, int pid, int level, int box, int array, int form, double* out,
                       long long* elems) {
  if (!c || !elems) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (level < 0 || level >= P->nlevels) return fail(c, CTUPPM_EINVAL, "problem %d has no level %d", pid, level);
  const auto& L = P->lev[level].boxes;
  if (box < 0 || box >= int(L.size())) return fail(c, CTUPPM_EINVAL, "level %d has no box %d", level, box);
  if (array < 0 || array > 19) return fail(c, CTUPPM_EINVAL, "unknown stage array %d", array);
  if (form < CTUPPM_FORM_PER_BOX || form > CTUPPM_FORM_WAVES) return fail(c, CTUPPM_EINVAL, "unknown form %d", form);
  if (P->nlevels == 2 && (form == CTUPPM_FORM_PER_BOX || form == CTUPPM_FORM_WAVES))
    return fail(c, CTUPPM_EINVAL, "two-level problems step in the batched forms only");
  if (!P->ws) return fail(c, CTUPPM_ESTATE, "problem %d: no workspace bound", pid);
  // the box's scratch, laid out as the step of that form laid it out
  const int ns = P->prm.nspec;
  size_t off = scratch_base(P);
  if (form == CTUPPM_FORM_WAVES) {
    size_t slot = 0;
    for (const auto& b : L) slot = std::max(slot, box_scratch_bytes(b, ns));
    off += size_t(box % c->wave_boxes) * slot;
  } else if (form != CTUPPM_FORM_PER_BOX) {
    if (level == 1)
      for (const auto& b : P->lev[0].boxes) off += box_scratch_bytes(b, ns);
    for (int b = 0; b < box; ++b) off += box_scratch_bytes(L[b], ns);
  }
  const int n[3] = {box_n(L[box], 0), box_n(L[box], 1), box_n(L[box], 2)};
  const long long grown = grown_cells(n), h1 = h1_cells(n);
  const long long nq = kNV + 1 + ns, nv = kNV + ns;
  const long long plane = (long long)(n[0] + 2) * (n[1] + 2), pplane = h1_plane(n);  // dense / padded
  long long first, ncomp;  // in doubles from the scratch start; components
  if (array == 0) {
    first = 0;
    ncomp = nq;
  } else if (array == 1) {
    first = nq * grown;
    ncomp = 1;
  } else {
    first = nq * grown + (1 + nv * (array - 2)) * h1;
    ncomp = nv;
  }
  const long long count = array == 0 ? nq * grown : ncomp * plane * (n[2] + 2);  // dense, as returned
  *elems = count;
  const size_t end = off + size_t(first + (array == 0 ? count : ncomp * h1)) * sizeof(double);
  if (end > P->ws_bytes)
    return fail(c, CTUPPM_ENOMEM, "problem %d: array %d of box %d in form %d ends at byte %zu of a %zu-byte workspace",
                pid, array, box, form, end, P->ws_bytes);
  if (!out) return CTUPPM_OK;
  const double* src = (const double*)((const char*)P->ws + off) + first;
  if (array == 0) {
    HIPCHK(c, hipMemcpyAsync(out, src, size_t(count) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return CTUPPM_OK;
  }
  // halo-1 arrays: drop the plane padding; the left states (arrays 2..4) are
  // stored at the cell below each face, so face f is read from f - stride
  if (array >= 2 && array <= 4) {
    const int d = array - 2;
    src -= d == 0 ? 1 : (d == 1 ? (n[0] + 2) : pplane);
  }
  HIPCHK(c, hipMemcpy2DAsync(out, size_t(plane) * sizeof(double), src, size_t(pplane) * sizeof(double),
                             size_t(plane) * sizeof(double), size_t(ncomp * (n[2] + 2)), hipMemcpyDeviceToDevice,
                             c->stream));
  return CTUPPM_OK;
}

int ctuppm_set_wave_boxes(ctuppm_ctx* c, int boxes) {
  if (!c || boxes < 1) return CTUPPM_EINVAL;
  c->wave_boxes = boxes;
  for (auto& kv : c->probs) invalidate(c, kv.second.get());  // slot assignment changes
  return CTUPPM_OK;
}

int ctuppm_set_concurrency(ctuppm_ctx* c, int on) {
  if (!c) return CTUPPM_EINVAL;
  bool graphs = false;
  for (auto& kv : c->sets) graphs = graphs || kv.second->has_graph();
  if (graphs) HIPCHK(c, hipStreamSynchronize(c->stream));
  c->concurrent = on ? 1 : 0;
  for (auto& kv : c->sets)  // graphs are re-captured
    for (int g = 0; g < 2; ++g)
      if (kv.second->exec[g]) {
        (void)hipGraphExecDestroy(kv.second->exec[g]);
        (void)hipGraphDestroy(kv.second->graph[g]);
        kv.second->exec[g] = nullptr;
        kv.second->graph[g] = nullptr;
      }
  return CTUPPM_OK;
}

int ctuppm_set_fused(ctuppm_ctx* c, int on) {
  if (!c) return CTUPPM_EINVAL;
  if (on < 0 || on > 2) return fail(c, CTUPPM_EINVAL, "fused mode must be 0, 1 or 2");
  c->fused = on;
  for (auto& kv : c->probs) drop_sets(c, kv.first);  // captured graphs hold the old kernels
  return CTUPPM_OK;
}

int ctuppm_bandwidth_probe(ctuppm_ctx* c, int kind, const void* src, void* dst, size_t bytes, int reps,
                           double* gbs) {
  if (!c || !gbs || kind < 0 || kind > 2 || reps < 1 || bytes < 16 || (bytes & 15)) return CTUPPM_EINVAL;
  if ((kind != 2 && !src) || (kind != 1 && !dst) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
    return fail(c, CTUPPM_EINVAL, "bandwidth probe: null or misaligned buffer");
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return fail(c, CTUPPM_EHIP, "hipEventCreate failed");
  double best = 0.0;
  // a few grid sizes (blocks per CU); the best rate is the ceiling
  for (int per_cu : {4, 8, 16, 32}) {
    const int blocks = per_cu * c->num_cus;
    LCHK(launch_probe(kind, src, dst, bytes, blocks, c->stream));  // warm
    HIPCHK(c, hipEventRecord(a, c->stream));
    for (int r = 0; r < reps; ++r) LCHK(launch_probe(kind, src, dst, bytes, blocks, c->stream));
    HIPCHK(c, hipEventRecord(b, c->stream));
    HIPCHK(c, hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, a, b));
    const double moved = double(bytes) * (kind == 0 ? 2.0 : 1.0);
    best = std::max(best, moved * reps / (double(ms) * 1e-3) / 1e9);
  }
  c->event_pool.push_back(a);
  c->event_pool.push_back(b);
  *gbs = best;
  return CTUPPM_OK;
}

int ctuppm_set_tuning(ctuppm_ctx* c, int bpc, int zb, int zp) {
  return ctuppm_set_tuning2(c, bpc, zb, zp, c ? c->ytile : 0);
}

int ctuppm_set_tuning2(ctuppm_ctx* c, int bpc, int zb, int zp, int ytile) {
  if (!c || bpc < 0 || zb < 1 || zp < 1 || ytile < 0) return CTUPPM_EINVAL;
  c->ytile = ytile;
  c->blocks_per_cu = bpc;
  c->zseg_batched = zb;
  c->zseg_per_box = zp;
  for (auto& kv : c->probs) invalidate(c, kv.second.get());  // work lists and graphs depend on the tuning
  return CTUPPM_OK;
}

int ctuppm_set_stage_planes(ctuppm_ctx* c, int stage, int planes) {
  if (!c) return CTUPPM_EINVAL;
  if (stage < 0 || stage >= kNumStages || stage_region(stage) < 0)
    return fail(c, CTUPPM_EINVAL, "stage %d has no work units", stage);
  if (planes < 1 || planes > 64) return fail(c, CTUPPM_EINVAL, "planes per unit %d outside 1..64", planes);
  c->region_planes[stage_region(stage)] = planes;
  c->region_set[stage_region(stage)] = true;
  for (auto& kv : c->probs) invalidate(c, kv.second.get());  // work lists and graphs depend on it
  return CTUPPM_OK;
}

int ctuppm_stage_planes(ctuppm_ctx* c, int stage, int* planes, int* group) {
  if (!c || !planes || !group) return CTUPPM_EINVAL;
  if (stage < 0 || stage >= kNumStages || stage_region(stage) < 0)
    return fail(c, CTUPPM_EINVAL, "stage %d has no work units", stage);
  *group = stage_region(stage);
  *planes = c->region_planes[*group];
  return CTUPPM_OK;
}

int ctuppm_stage_bytes(ctuppm_ctx* c, int pid, int stage, double* bytes) {
  if (!c || !bytes) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  double tot = 0.0;
  const double W = 8.0;  // bytes per double
  std::vector<ctuppm_box> all(P->lev[0].boxes);
  if (P->nlevels == 2)  // the fine level runs two substeps per step
    for (int r = 0; r < 2; ++r) all.insert(all.end(), P->lev[1].boxes.begin(), P->lev[1].boxes.end());
  const double nv = kNV + P->prm.nspec, nq = nv + 1;  // conserved / primitive components
  // launches per step of a stage run once per Runge-Kutta stage (MOL)
  const int scheme = P->prm.scheme;
  const double nst = scheme == 1 ? 2.0 : (scheme == 2 ? 3.0 : 1.0);
  for (const auto& bx : all) {
    const double n0 = box_n(bx, 0), n1 = box_n(bx, 1), n2 = box_n(bx, 2);
    const double nn[3] = {n0, n1, n2};
    const double valid = n0 * n1 * n2;
    const double grown = (n0 + 8) * (n1 + 8) * (n2 + 8);
    const double cells1 = (n0 + 2) * (n1 + 2) * (n2 + 2);
    auto face = [&](int d) { return cells1 / (nn[d] + 2) * (nn[d] + 1); };           // faces 0..n x -1..n
    auto fin = [&](int d) { return valid / nn[d] * (nn[d] + 1); };                    // faces 0..n x 0..n-1
    auto half = [&](int a, int b) { return face(a) / (nn[b] + 2) * nn[b]; };         // F^{a|b} region
    switch (stage) {
      case kStFill: tot += nst * 2 * nv * W * (grown - valid); break;
      case kStC2P: tot += (nv + nq) * W * grown; break;
      case kStC2POnly: tot += (scheme ? nst - 1 : 1.0) * (nv + nq) * W * grown; break;
      case kStCfl: tot += 5 * W * valid; break;
      case kStFlatten: tot += nst * (4 * W * cells1 + W * cells1); break;
      case kStReconX: case kStReconY: case kStReconZ: {
        const int d = stage - kStReconX;
        // q without the sound speed over the stencils of cells -1..n, phi, the face states
        tot += nst * ((nq - 1) * W * cells1 / (nn[d] + 2) * (nn[d] + 6) + W * cells1 + 2 * nv * W * face(d));
        break;
      }
      case kStMolUpdate:
        // per stage: the stage input, three flux arrays and the output; the
        // combination stages also read the current state
        tot += nst * (2 * nv * W * valid + nv * W * (fin(0) + fin(1) + fin(2))) + (nst - 1) * nv * W * valid;
        break;
      case kStTraceX: case kStTraceY: case kStTraceZ: {
        const int d = stage - kStTraceX;
        // q over cells -3..n+2 along d (the 5-cell stencils of cells -1..n), phi,
        // then the left and right states of faces 0..n
        tot += nq * W * cells1 / (nn[d] + 2) * (nn[d] + 6) + W * cells1 + 2 * nv * W * face(d);
        break;
      }
      case kStRiemX: case kStRiemY: case kStRiemZ: tot += nst * 3 * nv * W * face(stage - kStRiemX); break;
      case kStT1X: case kStT1Y: case kStT1Z: {
        const int a = stage - kStT1X, b = (a + 1) % 3, cc = (a + 2) % 3;
        tot += 2 * nv * W * face(a) + nv * W * face(b) + nv * W * face(cc) + nv * W * (half(a, b) + half(a, cc));
        break;
      }
      case kStT2X: case kStT2Y: case kStT2Z: {
        const int a = stage - kStT2X, b = (a + 1) % 3, cc = (a + 2) % 3;
        tot += 2 * nv * W * fin(a) + nv * W * half(b, cc) + nv * W * half(cc, b) + nv * W * fin(a);
        break;
      }
      case kStUpdate: tot += 2 * nv * W * valid + nv * W * (fin(0) + fin(1) + fin(2)); break;
      case kStTrace3: {
        // q over the union of the three directions' stencils of cells -1..n
        // (cells -1..n extended by 2 along one direction at a time), phi
        // written once, the face states of the three directions; the hydro
        // components only (the species are the species stage's)
        const double ext = (n0 + 6) * (n1 + 2) * (n2 + 2) + (n0 + 2) * (n1 + 6) * (n2 + 2) +
                           (n0 + 2) * (n1 + 2) * (n2 + 6) - 2 * cells1;
        // the flattening reads the pressure one cell further along each direction
        const double pext = (n0 + 8) * (n1 + 2) * (n2 + 2) + (n0 + 2) * (n1 + 8) * (n2 + 2) +
                            (n0 + 2) * (n1 + 2) * (n2 + 8) - 2 * cells1;
        tot += kNV * W * ext + W * pext + W * cells1 + 2 * kNV * W * (face(0) + face(1) + face(2));
        break;
      }
      case kStSpec3: {
        // each species over the union of its stencils, the face states of
        // the three directions; phi, the three velocities and the sound speed
        // of cells -1..n once
        // (the method of lines: phi only, per Runge-Kutta stage)
        const double ns = P->prm.nspec;
        if (ns == 0) break;
        const double ext = (n0 + 6) * (n1 + 2) * (n2 + 2) + (n0 + 2) * (n1 + 6) * (n2 + 2) +
                           (n0 + 2) * (n1 + 2) * (n2 + 6) - 2 * cells1;
        tot += nst * (ns * W * ext + (scheme ? 1 : 5) * W * cells1 + 2 * ns * W * (face(0) + face(1) + face(2)));
        break;
      }
      case kStRecon3: {
        // as the merged tracing, per Runge-Kutta stage: the union of the three
        // directions' stencils, the flattening's pressures, phi, the face
        // states (hydro components; the species are the species stage's)
        const double ext = (n0 + 6) * (n1 + 2) * (n2 + 2) + (n0 + 2) * (n1 + 6) * (n2 + 2) +
                           (n0 + 2) * (n1 + 2) * (n2 + 6) - 2 * cells1;
        const double pext = (n0 + 8) * (n1 + 2) * (n2 + 2) + (n0 + 2) * (n1 + 8) * (n2 + 2) +
                            (n0 + 2) * (n1 + 2) * (n2 + 8) - 2 * cells1;
        tot += nst * (kNV * W * ext + W * pext + W * cells1 + 2 * kNV * W * (face(0) + face(1) + face(2)));
        break;
      }
      case kStT1All:
        // the three directions' face states and normal fluxes once each, the six stage-1 fluxes
        for (int a = 0; a < 3; ++a) {
          const int b = (a + 1) % 3, cc = (a + 2) % 3;
          tot += 2 * nv * W * face(a) + nv * W * face(a) + nv * W * (half(a, b) + half(a, cc));
        }
        break;
      default: break;
    }
  }
  *bytes = tot;
  return CTUPPM_OK;
}

}  // extern "C"
