// Host runtime of the CTU/PPM library: problems and boxes, ghost-fill tags,
// per-stage work lists, the per-box / batched / graph step forms, timing.
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

struct DevAlloc {
  std::vector<void*> ptrs;
  hipError_t upload(const void* src, size_t bytes, void** out) {
    *out = nullptr;
    if (bytes == 0) return hipSuccess;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return e;
    ptrs.push_back(p);
    e = hipMemcpy(p, src, bytes, hipMemcpyHostToDevice);
    *out = p;
    return e;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

struct Level {
  std::vector<ctuppm_box> boxes;
  std::vector<double*> Ua, Ub;
  bool bound = false;
};

struct Problem {
  int id = -1;
  ctuppm_params prm{};
  int nlevels = 1;
  Level lev[2];
  void* ws = nullptr;
  size_t ws_bytes = 0;
  ProbDev* dP = nullptr;   // device record of level 0 (library-allocated)
  ProbDev* dPf = nullptr;  // device record of level 1 (two-level problems)
  int cur = 0;             // host mirror of the level-0 parity
  long long steps = 0;
  // two-level geometry: fine level = fine cells flo..fhi = coarse cells clo..chi
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

// Work lists of one set of problems stepped together in one form.
struct StepSet {
  std::vector<int> pids;
  int form = 0;
  int level = 0;
  int scheme = 0;   // shared by every problem of the set
  int riemann = 0;  // likewise
  int limiter = 0;  // likewise (reconstruction variant: 0 CW84, 1 CS, 2 CW84 + steepening)
  int nboxes = 0;
  BoxRec* boxes = nullptr;
  March* units[kNumRegions] = {};
  int nch[kNumRegions] = {};
  std::vector<int> box_beg[kNumRegions], box_cnt[kNumRegions];
  FillTag* ftags = nullptr;
  Chunk* fchunks = nullptr;
  int nfch = 0;
  std::vector<int> fbox_beg, fbox_cnt;
  BcTag* btags[3] = {};
  Chunk* bchunks[3] = {};
  int nbch[3] = {};
  std::vector<int> bbox_beg[3], bbox_cnt[3];
  ProbDev** probs = nullptr;
  int nprobs = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  DevAlloc mem;
  ~StepSet() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    mem.release();
  }
};

// Device tables of one two-level problem (batched forms).
struct TwoLevel {
  StepSet* cset = nullptr;  // level-0 work lists (owned by ctx->sets)
  StepSet* fset = nullptr;  // level-1 work lists
  TwoLevelArgs args{};
  GatherTag* gtags = nullptr;
  Chunk* gchunks = nullptr;
  int ngch = 0;
  CfTag* ctags = nullptr;
  Chunk* cchunks = nullptr;
  int ncch = 0;
  RegFace* faces = nullptr;
  int nfaces = 0;
  AvgTag* atags = nullptr;
  Chunk* achunks = nullptr;
  int nach = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  DevAlloc mem;
  ~TwoLevel() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    mem.release();
  }
};

struct TimedLaunch {
  int stage;
  hipEvent_t a, b;
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
  int zseg_batched = 1;   // planes per march unit, batched / graph forms
  int zseg_per_box = 1;   // planes per march unit, per-box form
  int ytile = 0;          // rows per tile of the march units (0: whole plane)
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

// Runge-Kutta stage fabs per box of a MOL problem (at the start of its workspace).
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
};

// Launch one stage over a work range (march units, or fill/bc tag chunks) with optional timing.
int run_stage(ctuppm_ctx* c, hipStream_t s, int stage, const BoxRec* boxes, const void* tags,
              const void* work, int nwork, bool persistent, bool timed, const StageArgs& A = StageArgs()) {
  if (nwork <= 0) return CTUPPM_OK;
  Launch L{boxes, tags, work, nwork, grid_for(c, nwork, persistent), s};
  L.arr = A.arr;
  L.out = A.out;
  L.comb = A.comb;
  L.c = A.c;
  L.last = A.last;
  L.rs = A.rs;
  L.lim = A.lim;
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

// The fine level must be one rectangle of boxes aligned to coarse cells, at
// least 3 coarse cells inside the domain; gives its fine range flo..fhi and
// the coarse cells clo..chi it covers.
int fine_geometry(ctuppm_ctx* c, const ctuppm_params& prm, const std::vector<ctuppm_box>& fb, int flo[3],
                  int fhi[3], int clo[3], int chi[3]) {
  long long vol = 0;
  for (int d = 0; d < 3; ++d) {
    flo[d] = fb[0].lo[d];
    fhi[d] = fb[0].hi[d];
  }
  for (const auto& b : fb) {
    long long v = 1;
    for (int d = 0; d < 3; ++d) {
      if ((b.lo[d] & 1) || !(b.hi[d] & 1))
        return fail(c, CTUPPM_EINVAL, "fine boxes must start at even and end at odd indices");
      flo[d] = std::min(flo[d], b.lo[d]);
      fhi[d] = std::max(fhi[d], b.hi[d]);
      v *= box_n(b, d);
    }
    vol += v;
  }
  long long bb = 1;
  for (int d = 0; d < 3; ++d) {
    bb *= fhi[d] - flo[d] + 1;
    clo[d] = flo[d] / 2;
    chi[d] = (fhi[d] + 1) / 2 - 1;
    if (clo[d] - 3 < prm.domain_lo[d] || chi[d] + 3 > prm.domain_hi[d])
      return fail(c, CTUPPM_EINVAL, "fine level must lie at least 3 coarse cells inside the domain");
  }
  if (bb != vol) return fail(c, CTUPPM_EINVAL, "fine boxes must tile one rectangle");
  return CTUPPM_OK;
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

// Coarse region of a two-level problem: coarse cells clo-3..chi+3.
long long region_cells(const Problem* P, int ext[3], int lo[3]) {
  long long v = 1;
  for (int d = 0; d < 3; ++d) {
    lo[d] = P->clo[d] - 3;
    ext[d] = P->chi[d] - P->clo[d] + 7;
    v *= ext[d];
  }
  return v;
}

long long register_faces(const Problem* P) {
  long long n = 0;
  for (int d = 0; d < 3; ++d) {
    long long a = 1;
    for (int e = 0; e < 3; ++e)
      if (e != d) a *= P->chi[e] - P->clo[e] + 1;
    n += 2 * a;
  }
  return n;
}

// Workspace after the stage scratch of both levels: the region at t^n and at
// t^{n+1} (nv = 5 + nspec doubles per cell each), then 2 nv doubles per
// register face.
size_t two_level_extra_bytes(const Problem* P) {
  if (P->nlevels != 2) return 0;
  int ext[3], lo[3];
  const long long rc = region_cells(P, ext, lo);
  const size_t nv = size_t(kNV + P->prm.nspec);
  return 2 * align256(size_t(rc) * nv * sizeof(double)) +
         align256(size_t(register_faces(P)) * 2 * nv * sizeof(double));
}

// Forget the cached work lists (and graphs) that involve problem pid.
void drop_sets(ctuppm_ctx* c, int pid) {
  c->two.erase(pid);
  for (auto it = c->sets.begin(); it != c->sets.end();) {
    const auto& v = std::get<0>(it->first);
    if (std::find(v.begin(), v.end(), pid) != v.end()) it = c->sets.erase(it);
    else ++it;
  }
}

// Build the work lists of level `level` for a set of problems in one form.
int build_set(ctuppm_ctx* c, const std::vector<int>& pids, int form, StepSet** out, int level = 0) {
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
  std::vector<BoxRec> boxes;
  std::vector<March> ch[kNumRegions];
  std::vector<FillTag> ftags;
  std::vector<Chunk> fch;
  std::vector<BcTag> btags[3];
  std::vector<Chunk> bch[3];
  std::vector<ProbDev*> probs;
  for (size_t ip = 0; ip < pids.size(); ++ip) {
    const int pid = pids[ip];
    Problem* P = get_problem(c, pid);
    if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
    if (ip == 0) {
      S->scheme = P->prm.scheme;
      S->riemann = P->prm.riemann;
      S->limiter = P->prm.limiter == CTUPPM_LIMITER_CS ? 1 : (P->prm.steepen ? 2 : 0);
    }
    const int var = P->prm.limiter == CTUPPM_LIMITER_CS ? 1 : (P->prm.steepen ? 2 : 0);
    if (P->prm.scheme != S->scheme || P->prm.riemann != S->riemann || var != S->limiter)
      return fail(c, CTUPPM_EINVAL,
                  "problems stepped together must use the same scheme, Riemann solver and limiter");
    if (level >= P->nlevels) return fail(c, CTUPPM_EINVAL, "problem %d has no level %d", pid, level);
    const Level& L = P->lev[level];
    if (!L.bound || !P->ws) return fail(c, CTUPPM_ESTATE, "problem %d: state or workspace not bound", pid);
    size_t need = 0;
    if (ctuppm_workspace_bytes(c, pid, S->form, &need) != CTUPPM_OK) return CTUPPM_EINVAL;
    if (P->ws_bytes < need)
      return fail(c, CTUPPM_ENOMEM, "problem %d: workspace %zu < %zu bytes", pid, P->ws_bytes, need);
    ProbDev* dPl = level == 0 ? P->dP : P->dPf;
    probs.push_back(dPl);
    const int base = int(boxes.size());
    // stage fabs of a MOL problem first, then the stage scratch
    const size_t wbytes = stage_fab_bytes(L.boxes, P->prm);
    size_t woff = 0;
    size_t off = wbytes;
    size_t slot = 0;  // waves form: every box fits any of the shared scratch slots
    for (const auto& b : L.boxes) slot = std::max(slot, box_scratch_bytes(b, P->prm.nspec));
    if (level == 1)  // level-1 scratch follows all level-0 scratch
      for (const auto& b : P->lev[0].boxes) off += box_scratch_bytes(b, P->prm.nspec);
    int dlo[3], dhi[3];
    level_domain(P->prm, level, dlo, dhi);
    for (size_t b = 0; b < L.boxes.size(); ++b) {
      const ctuppm_box& bx = L.boxes[b];
      BoxRec r{};
      r.U[0] = L.Ua[b];
      r.U[1] = L.Ub[b];
      r.scr = (double*)((char*)P->ws + (S->form == CTUPPM_FORM_PER_BOX ? wbytes
                                         : S->form == CTUPPM_FORM_WAVES ? wbytes + (b % size_t(c->wave_boxes)) * slot
                                                                        : off));
      off += box_scratch_bytes(bx, P->prm.nspec);
      r.P = dPl;
      r.level = level;
      r.ns = P->prm.nspec;
      for (int w = 0; w < stage_fabs(P->prm); ++w)
        r.W[w] = (double*)((char*)P->ws + woff + size_t(w) * (wbytes / size_t(stage_fabs(P->prm))));
      woff += box_fab_bytes(bx, P->prm.nspec);
      for (int d = 0; d < 3; ++d) {
        r.n[d] = box_n(bx, d);
        r.lo[d] = bx.lo[d];
        // reflecting domain walls on the box's faces (a fine level lies inside the domain)
        r.wall[d] = level == 0 ? ((bx.lo[d] == dlo[d] && P->prm.bc_lo[d] == CTUPPM_BC_REFLECT ? 1 : 0) |
                                  (bx.hi[d] == dhi[d] && P->prm.bc_hi[d] == CTUPPM_BC_REFLECT ? 2 : 0))
                               : 0;
      }
      boxes.push_back(r);
    }
    const int nb = int(L.boxes.size());
    // same-level ghost copies, periodic images included
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
    for (int db = 0; db < nb; ++db) {
      const ctuppm_box& D = L.boxes[db];
      int glo[3], ghi[3];
      for (int d = 0; d < 3; ++d) {
        glo[d] = D.lo[d] - kNG;
        ghi[d] = D.hi[d] + kNG;
      }
      for (int sb = 0; sb < nb; ++sb) {
        const ctuppm_box& Sx = L.boxes[sb];
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
              t.dst = base + db;
              t.src = base + sb;
              long long vol = 1;
              for (int d = 0; d < 3; ++d) {
                t.lo[d] = lo[d] - D.lo[d];
                t.ext[d] = hi[d] - lo[d] + 1;
                t.off[d] = D.lo[d] + sh[d] - Sx.lo[d];
                vol *= t.ext[d];
              }
              ftags.push_back(t);
              (void)vol;
            }
      }
    }
    // physical boundaries, one list per direction
    const double rgm1 = 1.0 / (P->prm.gamma - 1.0);
    const double* s = P->prm.inflow;
    double inflow_cons[kMaxV];
    inflow_cons[0] = s[0];
    inflow_cons[1] = s[0] * s[1];
    inflow_cons[2] = s[0] * s[2];
    inflow_cons[3] = s[0] * s[3];
    inflow_cons[4] = s[4] * rgm1 + 0.5 * s[0] * ((s[1] * s[1] + s[2] * s[2]) + s[3] * s[3]);
    for (int sp = 0; sp < P->prm.nspec; ++sp) inflow_cons[kNV + sp] = s[0] * P->prm.inflow_X[sp];
    for (int d = 0; d < 3; ++d) {
      if (P->prm.bc_lo[d] == CTUPPM_BC_PERIODIC) continue;
      for (int b = 0; b < nb; ++b) {
        const ctuppm_box& B = L.boxes[b];
        for (int side = 0; side < 2; ++side) {
          BcTag t{};
          t.box = base + b;
          t.dir = d;
          t.side = side;
          t.bc = side == 0 ? P->prm.bc_lo[d] : P->prm.bc_hi[d];
          t.dom_lo = dlo[d];
          t.dom_hi = dhi[d];
          for (int m = 0; m < kNV + P->prm.nspec; ++m) t.inflow[m] = inflow_cons[m];
          bool any = true;
          for (int e = 0; e < 3; ++e) {
            int lo = -kNG, hi = box_n(B, e) + kNG - 1;  // box-local grown range
            if (e == d) {
              if (side == 0) hi = std::min(hi, dlo[d] - 1 - B.lo[d]);
              else lo = std::max(lo, dhi[d] + 1 - B.lo[d]);
            }
            if (lo > hi) any = false;
            t.lo[e] = lo;
            t.ext[e] = hi - lo + 1;
          }
          if (any) btags[d].push_back(t);
        }
      }
    }
  }
  S->nboxes = int(boxes.size());
  S->nprobs = int(probs.size());
  // march units per region, per box in order; per-box launches use short z
  // segments so one box still fills the GPU
  const int zseg = S->form == CTUPPM_FORM_PER_BOX ? c->zseg_per_box : c->zseg_batched;  // waves: as batched
  for (int k = 0; k < kNumRegions; ++k) {
    S->box_beg[k].resize(S->nboxes);
    S->box_cnt[k].resize(S->nboxes);
    for (int b = 0; b < S->nboxes; ++b) {
      int org[3], ext[3];
      region_of(k, boxes[b].n, org, ext);
      S->box_beg[k][b] = int(ch[k].size());
      march_region(ch[k], b, org, ext, zseg, c->ytile);
      S->box_cnt[k][b] = int(ch[k].size()) - S->box_beg[k][b];
    }
    S->nch[k] = int(ch[k].size());
  }
  // fill tags sorted by destination box so a box's tags are contiguous
  std::stable_sort(ftags.begin(), ftags.end(), [](const FillTag& a, const FillTag& b) { return a.dst < b.dst; });
  S->fbox_beg.assign(S->nboxes, 0);
  S->fbox_cnt.assign(S->nboxes, 0);
  for (size_t t = 0; t < ftags.size(); ++t) {
    const FillTag& T = ftags[t];
    const int before = int(fch.size());
    chunk_region(fch, int(t), (long long)T.ext[0] * T.ext[1] * T.ext[2]);
    if (S->fbox_cnt[T.dst] == 0) S->fbox_beg[T.dst] = before;
    S->fbox_cnt[T.dst] += int(fch.size()) - before;
  }
  S->nfch = int(fch.size());
  for (int d = 0; d < 3; ++d) {
    S->bbox_beg[d].assign(S->nboxes, 0);
    S->bbox_cnt[d].assign(S->nboxes, 0);
    for (size_t t = 0; t < btags[d].size(); ++t) {
      const BcTag& T = btags[d][t];
      const int before = int(bch[d].size());
      chunk_region(bch[d], int(t), (long long)T.ext[0] * T.ext[1] * T.ext[2]);
      if (S->bbox_cnt[d][T.box] == 0) S->bbox_beg[d][T.box] = before;
      S->bbox_cnt[d][T.box] += int(bch[d].size()) - before;
    }
    S->nbch[d] = int(bch[d].size());
  }
  void* p = nullptr;
  HIPCHK(c, S->mem.upload(boxes.data(), boxes.size() * sizeof(BoxRec), &p));
  S->boxes = (BoxRec*)p;
  for (int k = 0; k < kNumRegions; ++k) {
    HIPCHK(c, S->mem.upload(ch[k].data(), ch[k].size() * sizeof(March), &p));
    S->units[k] = (March*)p;
  }
  HIPCHK(c, S->mem.upload(ftags.data(), ftags.size() * sizeof(FillTag), &p));
  S->ftags = (FillTag*)p;
  HIPCHK(c, S->mem.upload(fch.data(), fch.size() * sizeof(Chunk), &p));
  S->fchunks = (Chunk*)p;
  for (int d = 0; d < 3; ++d) {
    HIPCHK(c, S->mem.upload(btags[d].data(), btags[d].size() * sizeof(BcTag), &p));
    S->btags[d] = (BcTag*)p;
    HIPCHK(c, S->mem.upload(bch[d].data(), bch[d].size() * sizeof(Chunk), &p));
    S->bchunks[d] = (Chunk*)p;
  }
  HIPCHK(c, S->mem.upload(probs.data(), probs.size() * sizeof(ProbDev*), &p));
  S->probs = (ProbDev**)p;
  *out = S.get();
  c->sets[key] = std::move(S);
  return CTUPPM_OK;
}

const int kCellStages[] = {kStFlatten, kStTraceX, kStTraceY, kStTraceZ, kStRiemX, kStRiemY, kStRiemZ,
                           kStT1X, kStT1Y, kStT1Z, kStT2X, kStT2Y, kStT2Z, kStUpdate};

int run_cells(ctuppm_ctx* c, StepSet* S, hipStream_t s, int stage, int box, bool timed,
              const StageArgs& A0 = StageArgs()) {
  StageArgs A = A0;
  A.rs = S->riemann;
  A.lim = S->limiter;
  const int k = stage_region(stage);
  if (box < 0) return run_stage(c, s, stage, S->boxes, nullptr, S->units[k], S->nch[k], true, timed, A);
  return run_stage(c, s, stage, S->boxes, nullptr, S->units[k] + S->box_beg[k][box], S->box_cnt[k][box], false,
                   timed, A);
}

// A stage over the boxes b0..b1-1 of a set (their units are contiguous).
int run_range(ctuppm_ctx* c, StepSet* S, hipStream_t s, int stage, int b0, int b1, bool timed,
              const StageArgs& A0 = StageArgs()) {
  StageArgs A = A0;
  A.rs = S->riemann;
  A.lim = S->limiter;
  const int k = stage_region(stage);
  const int beg = S->box_beg[k][b0];
  const int end = S->box_beg[k][b1 - 1] + S->box_cnt[k][b1 - 1];
  return run_stage(c, s, stage, S->boxes, nullptr, S->units[k] + beg, end - beg, true, timed, A);
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
// copies, then the physical boundaries x, y, z.
int fill_arr(ctuppm_ctx* c, StepSet* S, hipStream_t s, bool timed, int arr) {
  StageArgs A;
  A.arr = arr;
  int rc;
  if (S->form == CTUPPM_FORM_PER_BOX) {
    for (int b = 0; b < S->nboxes; ++b)
      if ((rc = run_stage(c, s, kStFill, S->boxes, S->ftags, S->fchunks + S->fbox_beg[b], S->fbox_cnt[b], false,
                          timed, A)))
        return rc;
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < S->nboxes; ++b)
        if ((rc = run_stage(c, s, kStBcX + d, S->boxes, S->btags[d], S->bchunks[d] + S->bbox_beg[d][b],
                            S->bbox_cnt[d][b], false, timed, A)))
          return rc;
    return CTUPPM_OK;
  }
  if ((rc = run_stage(c, s, kStFill, S->boxes, S->ftags, S->fchunks, S->nfch, true, timed, A))) return rc;
  for (int d = 0; d < 3; ++d)
    if ((rc = run_stage(c, s, kStBcX + d, S->boxes, S->btags[d], S->bchunks[d], S->nbch[d], true, timed, A)))
      return rc;
  return CTUPPM_OK;
}

// One method-of-lines step (SSP-RK2 or RK3): per stage a ghost fill of the
// stage's input, cons->prim (with the CFL reduction and dt in the first
// stage), flattening, edge-value face states and normal fluxes along x, y, z,
// and the stage update; the last stage writes the other fab.
int enqueue_mol(ctuppm_ctx* c, StepSet* S, hipStream_t s, bool timed) {
  const bool per_box = S->form == CTUPPM_FORM_PER_BOX;
  const bool waves = S->form == CTUPPM_FORM_WAVES;
  const int nst = S->scheme == 1 ? 2 : 3;
  const int cells[] = {kStFlatten, kStReconX, kStReconY, kStReconZ, kStRiemX, kStRiemY, kStRiemZ};
  int rc;
  for (int r = 0; r < nst; ++r) {
    const int arr = r == 0 ? kArrCur : (r == 1 ? kArrW0 : kArrW1);
    if ((rc = fill_arr(c, S, s, timed, arr))) return rc;
    StageArgs A;
    A.arr = arr;
    if (r == 0) {
      if (per_box) {
        for (int b = 0; b < S->nboxes; ++b)
          if ((rc = run_cells(c, S, s, kStCfl, b, timed, A))) return rc;
      } else if ((rc = run_cells(c, S, s, waves ? kStCfl : kStC2P, -1, timed, A))) {
        return rc;
      }
      hipError_t e = launch_dt(S->probs, S->nprobs, s);
      if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "dt launch: %s", hipGetErrorString(e));
    }
    StageArgs U;
    U.arr = arr;
    U.out = r == nst - 1 ? kArrNext : (r == 0 ? kArrW0 : kArrW1);
    U.comb = r > 0;
    U.c = nst == 2 ? 0.5 : (r == 1 ? 0.25 : 2.0 / 3.0);
    U.last = r == nst - 1;
    if (waves) {
      for (const auto& w : box_groups(c, S)) {
        if ((rc = run_range(c, S, s, kStC2POnly, w.first, w.second, timed, A))) return rc;
        for (int st : cells)
          if ((rc = run_range(c, S, s, st, w.first, w.second, timed))) return rc;
        if ((rc = run_range(c, S, s, kStMolUpdate, w.first, w.second, timed, U))) return rc;
      }
      continue;
    }
    const int nb = per_box ? S->nboxes : 1;
    for (int b = 0; b < nb; ++b) {
      const int box = per_box ? b : -1;
      if ((per_box || r > 0) && (rc = run_cells(c, S, s, kStC2POnly, box, timed, A))) return rc;
      for (int st : cells)
        if ((rc = run_cells(c, S, s, st, box, timed))) return rc;
      if ((rc = run_cells(c, S, s, kStMolUpdate, box, timed, U))) return rc;
    }
  }
  hipError_t e = launch_flip(S->probs, S->nprobs, s);
  if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "flip launch: %s", hipGetErrorString(e));
  return CTUPPM_OK;
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
int enqueue_step_branched(ctuppm_ctx* c, StepSet* S, hipStream_t s) {
  int rc;
  if ((rc = run_stage(c, s, kStFill, S->boxes, S->ftags, S->fchunks, S->nfch, true, false))) return rc;
  for (int d = 0; d < 3; ++d)
    if ((rc = run_stage(c, s, kStBcX + d, S->boxes, S->btags[d], S->bchunks[d], S->nbch[d], true, false))) return rc;
  if ((rc = run_cells(c, S, s, kStC2P, -1, false))) return rc;
  hipError_t e = launch_dt(S->probs, S->nprobs, s);
  if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "dt launch: %s", hipGetErrorString(e));
  if ((rc = run_cells(c, S, s, kStFlatten, -1, false))) return rc;
  const hipStream_t str[3] = {s, c->side[0], c->side[1]};
  const int phases[3][2] = {{kStTraceX, kStRiemX}, {kStT1X, -1}, {kStT2X, -1}};
  for (int ph = 0; ph < 3; ++ph) {
    if ((rc = fork_side(c, s, 3 * ph))) return rc;
    for (int d = 0; d < 3; ++d)
      for (int q = 0; q < 2; ++q)
        if (phases[ph][q] >= 0 && (rc = run_cells(c, S, str[d], phases[ph][q] + d, -1, false))) return rc;
    if ((rc = join_side(c, s, 3 * ph + 1))) return rc;
  }
  if ((rc = run_cells(c, S, s, kStUpdate, -1, false))) return rc;
  e = launch_flip(S->probs, S->nprobs, s);
  if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "flip launch: %s", hipGetErrorString(e));
  return CTUPPM_OK;
}

// Enqueue one step of a set on stream s.
int enqueue_step(ctuppm_ctx* c, StepSet* S, hipStream_t s, bool timed) {
  if (S->scheme != 0) return enqueue_mol(c, S, s, timed);
  const bool per_box = S->form == CTUPPM_FORM_PER_BOX;
  const bool waves = S->form == CTUPPM_FORM_WAVES;
  int rc;
  if (per_box) {
    for (int b = 0; b < S->nboxes; ++b)
      if ((rc = run_stage(c, s, kStFill, S->boxes, S->ftags, S->fchunks + S->fbox_beg[b], S->fbox_cnt[b], false, timed)))
        return rc;
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < S->nboxes; ++b)
        if ((rc = run_stage(c, s, kStBcX + d, S->boxes, S->btags[d], S->bchunks[d] + S->bbox_beg[d][b],
                            S->bbox_cnt[d][b], false, timed)))
          return rc;
    for (int b = 0; b < S->nboxes; ++b)
      if ((rc = run_cells(c, S, s, kStCfl, b, timed))) return rc;
  } else {
    if ((rc = run_stage(c, s, kStFill, S->boxes, S->ftags, S->fchunks, S->nfch, true, timed))) return rc;
    for (int d = 0; d < 3; ++d)
      if ((rc = run_stage(c, s, kStBcX + d, S->boxes, S->btags[d], S->bchunks[d], S->nbch[d], true, timed))) return rc;
    // the waves form converts each wave into its shared scratch right before
    // the wave's stages, so only the CFL pass runs over all boxes here
    if ((rc = run_cells(c, S, s, waves ? kStCfl : kStC2P, -1, timed))) return rc;
  }
  {
    hipError_t e = launch_dt(S->probs, S->nprobs, s);
    if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "dt launch: %s", hipGetErrorString(e));
  }
  const int nst = int(sizeof(kCellStages) / sizeof(int));
  if (per_box) {
    for (int b = 0; b < S->nboxes; ++b) {
      if ((rc = run_cells(c, S, s, kStC2POnly, b, timed))) return rc;
      for (int q = 0; q < nst; ++q)
        if ((rc = run_cells(c, S, s, kCellStages[q], b, timed))) return rc;
    }
  } else if (waves) {
    for (const auto& w : box_groups(c, S)) {
      if ((rc = run_range(c, S, s, kStC2POnly, w.first, w.second, timed))) return rc;
      for (int q = 0; q < nst; ++q)
        if ((rc = run_range(c, S, s, kCellStages[q], w.first, w.second, timed))) return rc;
    }
  } else {
    for (int q = 0; q < nst; ++q)
      if ((rc = run_cells(c, S, s, kCellStages[q], -1, timed))) return rc;
  }
  hipError_t e = launch_flip(S->probs, S->nprobs, s);
  if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "flip launch: %s", hipGetErrorString(e));
  return CTUPPM_OK;
}

int find_box(const std::vector<ctuppm_box>& boxes, const int x[3]) {
  for (size_t b = 0; b < boxes.size(); ++b) {
    const ctuppm_box& B = boxes[b];
    if (x[0] >= B.lo[0] && x[0] <= B.hi[0] && x[1] >= B.lo[1] && x[1] <= B.hi[1] && x[2] >= B.lo[2] &&
        x[2] <= B.hi[2])
      return int(b);
  }
  return -1;
}

template <class T>
int upload_vec(ctuppm_ctx* c, DevAlloc& mem, const std::vector<T>& v, T** out) {
  void* p = nullptr;
  HIPCHK(c, mem.upload(v.data(), v.size() * sizeof(T), &p));
  *out = (T*)p;
  return CTUPPM_OK;
}

// Device tables of a two-level problem (built once, batched forms).
int build_two_level(ctuppm_ctx* c, int pid, TwoLevel** out) {
  auto it = c->two.find(pid);
  if (it != c->two.end()) {
    *out = it->second.get();
    return CTUPPM_OK;
  }
  Problem* P = get_problem(c, pid);
  std::unique_ptr<TwoLevel> T(new TwoLevel);
  const std::vector<int> v{pid};
  int rc = build_set(c, v, CTUPPM_FORM_BATCHED, &T->cset, 0);
  if (rc) return rc;
  rc = build_set(c, v, CTUPPM_FORM_BATCHED, &T->fset, 1);
  if (rc) return rc;
  size_t off = 0;
  for (int l = 0; l < 2; ++l)
    for (const auto& b : P->lev[l].boxes) off += box_scratch_bytes(b, P->prm.nspec);
  int rext[3], rlo[3];
  const long long rcells = region_cells(P, rext, rlo);
  char* base = (char*)P->ws;
  TwoLevelArgs& A = T->args;
  const size_t nv = size_t(kNV + P->prm.nspec);
  A.ct0 = (double*)(base + off);
  off += align256(size_t(rcells) * nv * sizeof(double));
  A.ct1 = (double*)(base + off);
  off += align256(size_t(rcells) * nv * sizeof(double));
  A.reg = (double*)(base + off);
  A.cboxes = T->cset->boxes;
  A.fboxes = T->fset->boxes;
  A.Pc = P->dP;
  A.Pf = P->dPf;
  for (int d = 0; d < 3; ++d) {
    A.rlo[d] = rlo[d];
    A.rext[d] = rext[d];
  }
  const auto& CB = P->lev[0].boxes;
  const auto& FB = P->lev[1].boxes;
  // gather: coarse valid cells inside the region
  std::vector<GatherTag> gt;
  std::vector<Chunk> gch;
  gather_tags(CB, rlo, rext, gt, gch);
  // coarse-to-fine: the ghost cells of each fine box outside the fine rectangle
  std::vector<CfTag> ct;
  std::vector<Chunk> cch;
  for (size_t b = 0; b < FB.size(); ++b) {
    int seg[3][3][2];
    for (int d = 0; d < 3; ++d) {
      const int glo = FB[b].lo[d] - kNG, ghi = FB[b].hi[d] + kNG;
      seg[d][0][0] = glo; seg[d][0][1] = std::min(ghi, P->flo[d] - 1);
      seg[d][1][0] = std::max(glo, P->flo[d]); seg[d][1][1] = std::min(ghi, P->fhi[d]);
      seg[d][2][0] = std::max(glo, P->fhi[d] + 1); seg[d][2][1] = ghi;
    }
    for (int a = 0; a < 3; ++a)
      for (int bb = 0; bb < 3; ++bb)
        for (int cc = 0; cc < 3; ++cc) {
          if (a == 1 && bb == 1 && cc == 1) continue;
          const int q[3] = {a, bb, cc};
          CfTag t{};
          t.box = int(b);
          long long vol = 1;
          bool empty = false;
          for (int d = 0; d < 3; ++d) {
            const int lo = seg[d][q[d]][0], hi = seg[d][q[d]][1];
            if (lo > hi) empty = true;
            t.lo[d] = lo - FB[b].lo[d];
            t.ext[d] = hi - lo + 1;
            vol *= std::max(0, t.ext[d]);
          }
          if (empty) continue;
          chunk_region(cch, int(ct.size()), vol);
          ct.push_back(t);
        }
  }
  // register faces on the six sides of the fine rectangle
  std::vector<RegFace> rf;
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    for (int side = 0; side < 2; ++side) {
      const int cf = side == 0 ? P->clo[d] : P->chi[d] + 1;
      const int uc = side == 0 ? P->clo[d] - 1 : P->chi[d] + 1;
      const int fcell = side == 0 ? P->flo[d] : P->fhi[d];
      const int fface = side == 0 ? P->flo[d] : P->fhi[d] + 1;
      for (int b2 = P->clo[t2]; b2 <= P->chi[t2]; ++b2)
        for (int b1 = P->clo[t1]; b1 <= P->chi[t1]; ++b1) {
          RegFace F{};
          F.d = d;
          F.side = side;
          int u[3];
          u[d] = uc; u[t1] = b1; u[t2] = b2;
          F.cbox = find_box(CB, u);
          int fc[3];
          fc[d] = fcell; fc[t1] = 2 * b1; fc[t2] = 2 * b2;
          F.fbox = find_box(FB, fc);
          if (F.cbox < 0 || F.fbox < 0) return fail(c, CTUPPM_EINVAL, "coarse-fine face without boxes");
          const ctuppm_box& C = CB[F.cbox];
          const ctuppm_box& Fb = FB[F.fbox];
          for (int e = 0; e < 3; ++e) {
            F.ucell[e] = u[e] - C.lo[e];
            F.cface[e] = (e == d ? cf : u[e]) - C.lo[e];
            F.fface[e] = (e == d ? fface : fc[e]) - Fb.lo[e];
          }
          rf.push_back(F);
        }
    }
  }
  // average down: coarse cells covered by each fine box
  std::vector<AvgTag> at;
  std::vector<Chunk> ach;
  for (size_t cb = 0; cb < CB.size(); ++cb)
    for (size_t fb = 0; fb < FB.size(); ++fb) {
      int flo[3], fhi[3], lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        flo[d] = FB[fb].lo[d] / 2;
        fhi[d] = (FB[fb].hi[d] + 1) / 2 - 1;
      }
      if (!intersect(CB[cb].lo, CB[cb].hi, flo, fhi, lo, hi)) continue;
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
      chunk_region(ach, int(at.size()), vol);
      at.push_back(t);
    }
  if ((rc = upload_vec(c, T->mem, gt, &T->gtags)) || (rc = upload_vec(c, T->mem, gch, &T->gchunks)) ||
      (rc = upload_vec(c, T->mem, ct, &T->ctags)) || (rc = upload_vec(c, T->mem, cch, &T->cchunks)) ||
      (rc = upload_vec(c, T->mem, rf, &T->faces)) || (rc = upload_vec(c, T->mem, at, &T->atags)) ||
      (rc = upload_vec(c, T->mem, ach, &T->achunks)))
    return rc;
  T->ngch = int(gch.size());
  T->ncch = int(cch.size());
  T->nfaces = int(rf.size());
  T->nach = int(ach.size());
  *out = T.get();
  c->two[pid] = std::move(T);
  return CTUPPM_OK;
}

#define TLCHK(expr)                                                                                \
  do {                                                                                             \
    hipError_t _e = (expr);                                                                        \
    if (_e != hipSuccess) return fail(c, CTUPPM_EHIP, "two-level launch %s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

int level_fill(ctuppm_ctx* c, StepSet* S, hipStream_t s, bool timed) {
  int rc = run_stage(c, s, kStFill, S->boxes, S->ftags, S->fchunks, S->nfch, true, timed);
  for (int d = 0; d < 3 && !rc; ++d)
    rc = run_stage(c, s, kStBcX + d, S->boxes, S->btags[d], S->bchunks[d], S->nbch[d], true, timed);
  return rc;
}

// One coarse step of a two-level problem: coarse advance, two fine substeps
// with coarse-to-fine ghost cells at theta = 0 and 1/2, average down, reflux.
int enqueue_two_level(ctuppm_ctx* c, Problem* P, TwoLevel* T, hipStream_t s, bool timed) {
  StepSet* C = T->cset;
  StepSet* F = T->fset;
  const TwoLevelArgs& A = T->args;
  const int nst = int(sizeof(kCellStages) / sizeof(int));
  int rc;
  if ((rc = level_fill(c, C, s, timed))) return rc;
  if ((rc = run_cells(c, C, s, kStC2P, -1, timed))) return rc;
  if ((rc = run_cells(c, F, s, kStCfl, -1, timed))) return rc;
  TLCHK(launch_dt2(P->dP, P->dPf, s));
  TLCHK(launch_gather(A, T->gtags, T->gchunks, T->ngch, 0, s));
  for (int q = 0; q < nst; ++q)
    if ((rc = run_cells(c, C, s, kCellStages[q], -1, timed))) return rc;
  TLCHK(launch_reg_coarse(A, T->faces, T->nfaces, s));
  TLCHK(launch_gather(A, T->gtags, T->gchunks, T->ngch, 1, s));
  for (int sub = 0; sub < 2; ++sub) {
    if ((rc = level_fill(c, F, s, timed))) return rc;
    TLCHK(launch_cfinterp(A, T->ctags, T->cchunks, T->ncch, sub == 0 ? 0.0 : 0.5, s));
    if ((rc = run_cells(c, F, s, kStC2POnly, -1, timed))) return rc;
    for (int q = 0; q < nst; ++q)
      if ((rc = run_cells(c, F, s, kCellStages[q], -1, timed))) return rc;
    TLCHK(launch_reg_fine(A, T->faces, T->nfaces, s));
    TLCHK(launch_flip(F->probs, F->nprobs, s));
  }
  TLCHK(launch_avgdown(A, T->atags, T->achunks, T->nach, s));
  TLCHK(launch_reflux(A, T->faces, T->nfaces, s));
  TLCHK(launch_flip(C->probs, C->nprobs, s));
  return CTUPPM_OK;
}

int step_two_level(ctuppm_ctx* c, int pid, int form) {
  Problem* P = get_problem(c, pid);
  if (form == CTUPPM_FORM_PER_BOX || form == CTUPPM_FORM_WAVES)
    return fail(c, CTUPPM_EINVAL, "two-level problems step in the batched forms only");
  if (!P->lev[0].bound || !P->lev[1].bound || !P->ws)
    return fail(c, CTUPPM_ESTATE, "problem %d: state or workspace not bound", pid);
  size_t need = 0;
  if (ctuppm_workspace_bytes(c, pid, CTUPPM_FORM_BATCHED, &need) != CTUPPM_OK) return CTUPPM_EINVAL;
  if (P->ws_bytes < need) return fail(c, CTUPPM_ENOMEM, "problem %d: workspace %zu < %zu bytes", pid, P->ws_bytes, need);
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
  if (S->form != CTUPPM_FORM_PER_BOX) return run_cells(c, S, s, kStCfl, -1, c->timing);
  for (int b = 0; b < S->nboxes; ++b) {
    const int rc = run_cells(c, S, s, kStCfl, b, c->timing);
    if (rc) return rc;
  }
  return CTUPPM_OK;
}

// cons->prim and the cell stages of a level, box by box in the per-box form.
int advance_cells(ctuppm_ctx* c, StepSet* S, hipStream_t s) {
  const int nst = int(sizeof(kCellStages) / sizeof(int));
  const bool per_box = S->form == CTUPPM_FORM_PER_BOX;
  for (const auto& g : box_groups(c, S)) {
    int rc = per_box ? run_cells(c, S, s, kStC2POnly, g.first, c->timing)
                     : run_range(c, S, s, kStC2POnly, g.first, g.second, c->timing);
    for (int q = 0; q < nst && !rc; ++q)
      rc = per_box ? run_cells(c, S, s, kCellStages[q], g.first, c->timing)
                   : run_range(c, S, s, kCellStages[q], g.first, g.second, c->timing);
    if (rc) return rc;
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
  *out = c.release();
  return CTUPPM_OK;
}

int ctuppm_ctx_destroy(ctuppm_ctx* c) {
  if (!c) return CTUPPM_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  c->two.clear();
  c->sets.clear();
  for (auto& kv : c->probs) {
    if (kv.second->dP) (void)hipFree(kv.second->dP);
    if (kv.second->dPf) (void)hipFree(kv.second->dPf);
  }
  c->probs.clear();
  for (auto& t : c->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
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
  ProbDev h{};
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
  HIPCHK(c, hipMalloc((void**)&P->dP, sizeof(ProbDev)));
  HIPCHK(c, hipMemcpy(P->dP, &h, sizeof(ProbDev), hipMemcpyHostToDevice));
  if (nlevels == 2) {
    for (int d = 0; d < 3; ++d) {
      h.dx[d] = prm->dx[d] / 2.0;
      h.rdx[d] = 1.0 / h.dx[d];
    }
    HIPCHK(c, hipMalloc((void**)&P->dPf, sizeof(ProbDev)));
    HIPCHK(c, hipMemcpy(P->dPf, &h, sizeof(ProbDev), hipMemcpyHostToDevice));
  }
  P->id = c->next_id++;
  *pid_out = P->id;
  c->probs[P->id] = std::move(P);
  return CTUPPM_OK;
}

int ctuppm_problem_destroy(ctuppm_ctx* c, int pid) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  (void)hipStreamSynchronize(c->stream);
  drop_sets(c, pid);
  if (P->dP) (void)hipFree(P->dP);
  if (P->dPf) (void)hipFree(P->dPf);
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
  const size_t wb = stage_fab_bytes(P->lev[0].boxes, P->prm);
  if (form == CTUPPM_FORM_PER_BOX) {
    if (P->nlevels == 2) return fail(c, CTUPPM_EINVAL, "two-level problems step in the batched forms only");
    *bytes = wb + mx;
  } else if (form == CTUPPM_FORM_BATCHED || form == CTUPPM_FORM_GRAPH) {
    *bytes = wb + total + two_level_extra_bytes(P);
  } else if (form == CTUPPM_FORM_WAVES) {
    if (P->nlevels == 2) return fail(c, CTUPPM_EINVAL, "two-level problems step in the batched forms only");
    *bytes = wb + std::min(size_t(c->wave_boxes), P->lev[0].boxes.size()) * mx;
  } else {
    return fail(c, CTUPPM_EINVAL, "unknown form %d", form);
  }
  return CTUPPM_OK;
}

int ctuppm_bind_state(ctuppm_ctx* c, int pid, int level, double* const* Ua, double* const* Ub) {
  if (!c || !Ua || !Ub) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (level < 0 || level >= P->nlevels) return fail(c, CTUPPM_EINVAL, "bad level %d", level);
  Level& L = P->lev[level];
  L.Ua.assign(Ua, Ua + L.boxes.size());
  L.Ub.assign(Ub, Ub + L.boxes.size());
  for (size_t b = 0; b < L.boxes.size(); ++b)
    if (!L.Ua[b] || !L.Ub[b] || ((uintptr_t)L.Ua[b] & 7) || ((uintptr_t)L.Ub[b] & 7))
      return fail(c, CTUPPM_EINVAL, "box %zu: null or misaligned fab pointer", b);
  L.bound = true;
  P->cur = 0;
  drop_sets(c, pid);
  // parity back to A
  int zero = 0;
  HIPCHK(c, hipMemcpyAsync(&(level == 0 ? P->dP : P->dPf)->cur, &zero, sizeof(int), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CTUPPM_OK;
}

int ctuppm_bind_workspace(ctuppm_ctx* c, int pid, void* ws, size_t bytes) {
  if (!c || !ws) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if ((uintptr_t)ws & 255) return fail(c, CTUPPM_EINVAL, "workspace must be 256-byte aligned");
  P->ws = ws;
  P->ws_bytes = bytes;
  drop_sets(c, pid);
  return CTUPPM_OK;
}

int ctuppm_set_fixed_dt(ctuppm_ctx* c, int pid, double dt) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  const double v = dt > 0.0 ? dt : 0.0;
  HIPCHK(c, hipMemcpyAsync(&P->dP->fixed_dt, &v, sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CTUPPM_OK;
}

int ctuppm_step(ctuppm_ctx* c, const int* pids, int npids, int form) {
  if (!c || !pids || npids < 1) return CTUPPM_EINVAL;
  if (form < CTUPPM_FORM_PER_BOX || form > CTUPPM_FORM_WAVES) return fail(c, CTUPPM_EINVAL, "unknown form %d", form);
  std::vector<int> v(pids, pids + npids);
  for (size_t i = 0; i < v.size(); ++i) {
    for (size_t j = 0; j < i; ++j)
      if (v[i] == v[j]) return fail(c, CTUPPM_EINVAL, "problem %d listed twice", v[i]);
    Problem* P = get_problem(c, v[i]);
    if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", v[i]);
    if (P->phase != 0)
      return fail(c, CTUPPM_ESTATE, "problem %d is in the middle of a step taken in pieces", v[i]);
    if (P->nlevels == 2) {
      if (npids != 1) return fail(c, CTUPPM_EINVAL, "a two-level problem steps on its own");
      return step_two_level(c, v[i], form);
    }
  }
  StepSet* S = nullptr;
  int rc = build_set(c, v, form, &S);
  if (rc) return rc;
  if (form == CTUPPM_FORM_GRAPH) {
    if (!S->exec) {
      HIPCHK(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
      rc = (c->concurrent && S->scheme == 0) ? enqueue_step_branched(c, S, c->capture)
                                             : enqueue_step(c, S, c->capture, false);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->capture, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "graph capture: %s", hipGetErrorString(e));
      S->graph = g;
      HIPCHK(c, hipGraphInstantiate(&S->exec, g, nullptr, nullptr, 0));
    }
    HIPCHK(c, hipGraphLaunch(S->exec, c->stream));
  } else {
    rc = enqueue_step(c, S, c->stream, c->timing);
    if (rc) return rc;
  }
  for (int pid : v) {
    Problem* P = get_problem(c, pid);
    P->cur ^= 1;
    P->steps += 1;
    P->state_changed();
  }
  return CTUPPM_OK;
}

int ctuppm_fill_ghosts(ctuppm_ctx* c, int pid, int level, int form) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = nullptr;
  int rc = piece_problem(c, pid, form, &P);
  if (rc) return rc;
  if (level < 0 || level >= P->nlevels) return fail(c, CTUPPM_EINVAL, "problem %d has no level %d", pid, level);
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
      if ((rc = level_fill(c, T->cset, c->stream, c->timing))) return rc;
    } else {
      if (P->phase != 1 || P->fine_done >= 2)
        return fail(c, CTUPPM_ESTATE, "problem %d: fine ghost cells are filled after the coarse advance, before "
                    "each of the two fine substeps", pid);
      if ((rc = level_fill(c, T->fset, c->stream, c->timing))) return rc;
      LCHK(launch_cfinterp(T->args, T->ctags, T->cchunks, T->ncch, 0.5 * P->fine_done, c->stream));
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
    LCHK(launch_dt(S->probs, S->nprobs, c->stream));
  } else {
    TwoLevel* T = nullptr;
    if ((rc = build_two_level(c, pid, &T))) return rc;
    if ((rc = run_cells(c, T->cset, c->stream, kStCfl, -1, c->timing)) ||
        (rc = run_cells(c, T->fset, c->stream, kStCfl, -1, c->timing)))
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
    LCHK(launch_flip(S->probs, S->nprobs, s));
    P->cur ^= 1;
    P->steps += 1;
    P->state_changed();
    return CTUPPM_OK;
  }
  TwoLevel* T = nullptr;
  if ((rc = build_two_level(c, pid, &T))) return rc;
  const TwoLevelArgs& A = T->args;
  if (level == 0) {
    if (dt_dev) LCHK(launch_set_dt(P->dP, P->dPf, dt_dev, s));
    LCHK(launch_gather(A, T->gtags, T->gchunks, T->ngch, 0, s));
    if ((rc = advance_cells(c, T->cset, s))) return rc;
    LCHK(launch_reg_coarse(A, T->faces, T->nfaces, s));
    LCHK(launch_gather(A, T->gtags, T->gchunks, T->ngch, 1, s));
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
  LCHK(launch_reg_fine(A, T->faces, T->nfaces, s));
  LCHK(launch_flip(T->fset->probs, T->fset->nprobs, s));
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
  LCHK(launch_avgdown(T->args, T->atags, T->achunks, T->nach, c->stream));
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
  LCHK(launch_reflux(T->args, T->faces, T->nfaces, c->stream));
  LCHK(launch_flip(T->cset->probs, T->cset->nprobs, c->stream));
  P->phase = 0;
  P->fine_done = 0;
  P->averaged = false;
  P->cur ^= 1;
  P->steps += 1;
  P->state_changed();
  return CTUPPM_OK;
}

int ctuppm_step_checked(ctuppm_ctx* c, int pid, int form, int* retried) {
  if (!c || !retried) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  if (P->nlevels != 1) return fail(c, CTUPPM_EINVAL, "checked steps are for single-level problems");
  *retried = 0;
  long long before[6], after[6];
  int rc = ctuppm_status(c, pid, before);
  if (rc) return rc;
  if ((rc = ctuppm_step(c, &pid, 1, form))) return rc;
  if ((rc = ctuppm_status(c, pid, after))) return rc;
  if (after[4] == before[4]) return CTUPPM_OK;
  // rejected: U^n is intact in the other fab; undo the flip and the step count
  ProbDev h;
  HIPCHK(c, hipMemcpy(&h, P->dP, sizeof(ProbDev), hipMemcpyDeviceToHost));
  const double dt = h.dt, keep_fixed = h.fixed_dt;
  h.cur ^= 1;
  h.nsteps -= 1;
  h.fail_step = -1;
  h.fixed_dt = 0.5 * dt;
  HIPCHK(c, hipMemcpy(P->dP, &h, sizeof(ProbDev), hipMemcpyHostToDevice));
  P->cur ^= 1;
  P->steps -= 1;
  for (int half = 0; half < 2; ++half)
    if ((rc = ctuppm_step(c, &pid, 1, form))) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(&P->dP->fixed_dt, &keep_fixed, sizeof(double), hipMemcpyHostToDevice));
  *retried = 1;
  return CTUPPM_OK;
}

int ctuppm_set_fail_hook(ctuppm_ctx* c, int pid, int step_index) {
  if (!c) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(&P->dP->fail_step, &step_index, sizeof(int), hipMemcpyHostToDevice));
  return CTUPPM_OK;
}

int ctuppm_current_state(ctuppm_ctx* c, int pid, int* which) {
  if (!c || !which) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  *which = P->cur;
  return CTUPPM_OK;
}

int ctuppm_get_dt(ctuppm_ctx* c, int pid, double* dt) {
  if (!c || !dt) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(dt, &P->dP->dt, sizeof(double), hipMemcpyDeviceToHost));
  return CTUPPM_OK;
}

int ctuppm_status(ctuppm_ctx* c, int pid, long long counters[6]) {
  if (!c || !counters) return CTUPPM_EINVAL;
  Problem* P = get_problem(c, pid);
  if (!P) return fail(c, CTUPPM_EINVAL, "unknown problem %d", pid);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  ProbDev h;
  HIPCHK(c, hipMemcpy(&h, P->dP, sizeof(ProbDev), hipMemcpyDeviceToHost));
  for (int i = 0; i < 5; ++i) counters[i] = (long long)h.cnt[i];
  counters[5] = h.nsteps;
  if (P->dPf) {
    HIPCHK(c, hipMemcpy(&h, P->dPf, sizeof(ProbDev), hipMemcpyDeviceToHost));
    for (int i = 0; i < 5; ++i) counters[i] += (long long)h.cnt[i];
  }
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
  StepSet* S = nullptr;
  const std::vector<int> v{pid};
  int rc = build_set(c, v, CTUPPM_FORM_BATCHED, &S, 0);
  if (rc) return rc;
  if ((rc = fill_arr(c, S, c->stream, false, kArrCur))) return rc;
  int dn[3];
  for (int d = 0; d < 3; ++d) dn[d] = P->prm.domain_hi[d] - P->prm.domain_lo[d] + 1;
  hipError_t e =
      launch_tag(S->boxes, S->units[kValid], S->nch[kValid], threshold, tags, dn, P->prm.domain_lo, c->stream);
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
    if (!Ua[b] || !Ub[b]) return fail(c, CTUPPM_EINVAL, "null fab for fine box %d", b);
  int rc = check_level(c, P->prm, 1, fine_boxes, nfine);
  if (rc) return rc;
  const std::vector<ctuppm_box> NB(fine_boxes, fine_boxes + nfine);
  int flo[3], fhi[3], clo[3], chi[3];
  if ((rc = fine_geometry(c, P->prm, NB, flo, fhi, clo, chi))) return rc;
  // the coarse cells the interpolation reads: parents and their neighbours
  StepSet* S0 = nullptr;
  StepSet* S1 = nullptr;
  const std::vector<int> v{pid};
  if ((rc = build_set(c, v, CTUPPM_FORM_BATCHED, &S0, 0)) || (rc = build_set(c, v, CTUPPM_FORM_BATCHED, &S1, 1)))
    return rc;
  TwoLevelArgs A{};
  int rlo[3], rext[3];
  long long rcells = 1;
  for (int d = 0; d < 3; ++d) {
    rlo[d] = clo[d] - 1;
    rext[d] = chi[d] - clo[d] + 3;
    rcells *= rext[d];
    A.rlo[d] = rlo[d];
    A.rext[d] = rext[d];
  }
  std::vector<GatherTag> gt;
  std::vector<Chunk> gch;
  gather_tags(P->lev[0].boxes, rlo, rext, gt, gch);
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
    // pieces of the box below, inside and above the old fine rectangle, per direction
    int seg[3][3][2];
    for (int d = 0; d < 3; ++d) {
      const int lo = NB[b].lo[d], hi = NB[b].hi[d];
      seg[d][0][0] = lo; seg[d][0][1] = std::min(hi, P->flo[d] - 1);
      seg[d][1][0] = std::max(lo, P->flo[d]); seg[d][1][1] = std::min(hi, P->fhi[d]);
      seg[d][2][0] = std::max(lo, P->fhi[d] + 1); seg[d][2][1] = hi;
    }
    for (int qa = 0; qa < 3; ++qa)
      for (int qb = 0; qb < 3; ++qb)
        for (int qc = 0; qc < 3; ++qc) {
          const int q[3] = {qa, qb, qc};
          int lo[3], hi[3];
          bool empty = false;
          for (int d = 0; d < 3; ++d) {
            lo[d] = seg[d][q[d]][0];
            hi[d] = seg[d][q[d]][1];
            empty = empty || lo[d] > hi[d];
          }
          if (empty) continue;
          if (qa == 1 && qb == 1 && qc == 1) {  // inside the old rectangle: copy, box by box
            for (size_t o = 0; o < OB.size(); ++o) {
              int ilo[3], ihi[3];
              if (intersect(lo, hi, OB[o].lo, OB[o].hi, ilo, ihi)) add(b, int(o), ilo, ihi);
            }
          } else {
            add(b, -1, lo, hi);
          }
        }
  }
  DevAlloc tmp;
  double* region = nullptr;
  const size_t rbytes = size_t(rcells) * size_t(kNV + ns) * sizeof(double);
  HIPCHK(c, hipMalloc((void**)&region, rbytes));
  tmp.ptrs.push_back(region);
  GatherTag* dgt = nullptr;
  Chunk* dgch = nullptr;
  ProlongTag* dpt = nullptr;
  Chunk* dpch = nullptr;
  BoxRec* dnrec = nullptr;
  if ((rc = upload_vec(c, tmp, gt, &dgt)) || (rc = upload_vec(c, tmp, gch, &dgch)) ||
      (rc = upload_vec(c, tmp, pt, &dpt)) || (rc = upload_vec(c, tmp, pch, &dpch)) ||
      (rc = upload_vec(c, tmp, nrec, &dnrec))) {
    (void)hipStreamSynchronize(c->stream);
    tmp.release();
    return rc;
  }
  A.cboxes = S0->boxes;
  A.fboxes = S1->boxes;
  A.Pc = P->dP;
  A.Pf = P->dPf;
  A.ct0 = region;
  hipError_t e = launch_gather(A, dgt, dgch, int(gch.size()), 0, c->stream);
  if (e == hipSuccess) e = launch_prolong(A, dnrec, S1->boxes, dpt, dpch, int(pch.size()), c->stream);
  hipError_t e2 = hipStreamSynchronize(c->stream);
  tmp.release();
  if (e != hipSuccess) return fail(c, CTUPPM_EHIP, "regrid launch: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(c, CTUPPM_EHIP, "regrid: %s", hipGetErrorString(e2));
  // the fine level's parity: the new state is in the A fabs
  ProbDev h;
  HIPCHK(c, hipMemcpy(&h, P->dPf, sizeof(ProbDev), hipMemcpyDeviceToHost));
  h.cur = 0;
  HIPCHK(c, hipMemcpy(P->dPf, &h, sizeof(ProbDev), hipMemcpyHostToDevice));
  drop_sets(c, pid);
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
  if (!P->ws) return fail(c, CTUPPM_ESTATE, "problem %d: no workspace bound", pid);
  // the box's scratch, laid out as the step of that form laid it out
  const int ns = P->prm.nspec;
  size_t off = stage_fab_bytes(P->lev[0].boxes, P->prm);
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
  long long first, count;  // in doubles from the scratch start
  if (array == 0) {
    first = 0;
    count = nq * grown;
  } else if (array == 1) {
    first = nq * grown;
    count = h1;
  } else {
    first = nq * grown + (1 + nv * (array - 2)) * h1;
    count = nv * h1;
  }
  *elems = count;
  if (!out) return CTUPPM_OK;
  const double* src = (const double*)((const char*)P->ws + off) + first;
  HIPCHK(c, hipMemcpyAsync(out, src, size_t(count) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return CTUPPM_OK;
}

int ctuppm_set_wave_boxes(ctuppm_ctx* c, int boxes) {
  if (!c || boxes < 1) return CTUPPM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->wave_boxes = boxes;
  for (auto it = c->sets.begin(); it != c->sets.end();) {  // slot assignment changes
    if (std::get<1>(it->first) == CTUPPM_FORM_WAVES) it = c->sets.erase(it);
    else ++it;
  }
  return CTUPPM_OK;
}

int ctuppm_set_concurrency(ctuppm_ctx* c, int on) {
  if (!c) return CTUPPM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->concurrent = on ? 1 : 0;
  for (auto& kv : c->sets)  // graphs are re-captured
    if (kv.second->exec) {
      (void)hipGraphExecDestroy(kv.second->exec);
      (void)hipGraphDestroy(kv.second->graph);
      kv.second->exec = nullptr;
      kv.second->graph = nullptr;
    }
  return CTUPPM_OK;
}

int ctuppm_set_tuning(ctuppm_ctx* c, int bpc, int zb, int zp) {
  return ctuppm_set_tuning2(c, bpc, zb, zp, c ? c->ytile : 0);
}

int ctuppm_set_tuning2(ctuppm_ctx* c, int bpc, int zb, int zp, int ytile) {
  if (!c || bpc < 0 || zb < 1 || zp < 1 || ytile < 0) return CTUPPM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->ytile = ytile;
  c->blocks_per_cu = bpc;
  c->zseg_batched = zb;
  c->zseg_per_box = zp;
  c->two.clear();
  c->sets.clear();  // work lists and graphs depend on the tuning
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
      default: break;
    }
  }
  *bytes = tot;
  return CTUPPM_OK;
}

}  // extern "C"
