// Internal host/device structures of the CTU/PPM library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ctu {

constexpr int kNV = 5;     // rho, rho u, rho v, rho w, rho E (species rho X_s follow)
constexpr int kMaxSpec = 16;
constexpr int kMaxV = kNV + kMaxSpec;
constexpr int kNG = 4;     // ghost layers
constexpr int kBlock = 256;  // threads per block = items per chunk
constexpr int kSlots = 64;   // signal-speed max accumulators per problem (spread atomics)

// Work regions of a box (n valid cells per direction), as (origin, extent):
//   kValid  cells [0, n)            kGrown cells [-4, n+4)   kCells1 cells [-1, n]
//   kFaceD  faces [0, n] along D, cells [-1, n] across
//   kFinD   faces [0, n] along D, cells [0, n) across, with x over [-1, n]
//           (whole rows of the halo-1 arrays: the threads off the faces
//           store zeros, so a row is written in whole lines)
//   kCells1T  cells [-1, n] like kCells1: the merged tracing's own region, so
//   its work units can march through more planes than stage 1's (a block
//   marching through consecutive planes finds the z stencils of the next
//   plane in its caches)
enum Region : int { kValid = 0, kGrown, kCells1, kFace0, kFace1, kFace2, kFin0, kFin1, kFin2, kCells1T, kNumRegions };

__host__ __device__ inline void region_of(int kind, const int n[3], int org[3], int ext[3]) {
  for (int d = 0; d < 3; ++d) {
    switch (kind) {
      case kValid: org[d] = 0; ext[d] = n[d]; break;
      case kGrown: org[d] = -kNG; ext[d] = n[d] + 2 * kNG; break;
      case kCells1: case kCells1T: org[d] = -1; ext[d] = n[d] + 2; break;
      case kFace0: case kFace1: case kFace2:
        if (d == kind - kFace0) { org[d] = 0; ext[d] = n[d] + 1; } else { org[d] = -1; ext[d] = n[d] + 2; }
        break;
      default:
        if (d == 0) { org[d] = -1; ext[d] = n[d] + 2; }
        else if (d == kind - kFin0) { org[d] = 0; ext[d] = n[d] + 1; }
        else { org[d] = 0; ext[d] = n[d]; }
        break;
    }
  }
}

// Per-problem device record: constants, then the state the kernels update.
struct ProbDev {
  double gamma, gm1, rgm1, cfl, small_dens, small_pres, grav_z;
  double dx[3], rdx[3];
  double fixed_dt;                 // > 0: use this dt instead of the CFL one
  double dt;                       // dt of the current/last step
  // per-direction factors of that dt, set with it once per step so no thread
  // divides: dt/dx_d, (dt/dx_d)/3 (transverse stage 1), (dt/dx_d)/2 (stage 2)
  double dtdx[3], dt3dx[3], dt2dx[3];
  unsigned long long cnt[5];       // dens floor, pres floor, traced floors, transverse fall-backs, failures
  int cur;                         // which of U[0], U[1] holds the current state
  int nsteps;
  int nlevels;
  int fail_step;                   // test hook: the update flags a failure at this step (-1: off)
  int nspec;                       // passive species after rho E
  int scheme;                      // 0 CTU, 1 MOL + SSP-RK2, 2 MOL + SSP-RK3
  int riemann;                     // 0 HLLC, 1 two-shock
  int limiter;                     // 0 CW84, 1 Colella & Sekora
  int steepen;                     // CW84 contact steepening of the density
  int rejected;                    // guarded steps rejected (their new state failed)
  unsigned long long fail_mark;    // failure count [4] when the last step was committed or rejected
  int* hflag;                      // host-mapped copy of `rejected` (read by the host without a sync)
  int pad5[2];
  // running max of the signal speed as bit patterns (>= 0), one 128-byte
  // line per slot so blocks of one launch do not contend on one address
  unsigned long long smax[kSlots][16];
};

// One box of a step set.
struct BoxRec {
  double* U[2];     // grown fabs [5 + ns][nz+8][ny+8][nx+8], caller-owned
  double* W[2];     // Runge-Kutta stage fabs (same layout, in the workspace; MOL only)
  double* scr;      // stage scratch of this box
  ProbDev* P;       // problem the box belongs to
  int n[3];         // valid cells
  int lo[3];        // level index of valid cell (0,0,0)
  int level;
  int ns;           // passive species of the problem
  int wall[3];      // bit 0: the box's low face along d is a reflecting domain wall; bit 1: its high face
};

struct Chunk { int box; int start; };  // tag index, first item (ghost-fill work lists)

// Column-march work unit: items [start, min(start+256, end)) of the (x, y)
// plane of a box region (i fastest), for the box-local planes z in [z0, z1),
// visited in order.
struct March { int box; int start; int end; int z0; int z1; int pad; };  // 32-bit fields: shorts cost VGPRs

// One launch covers the work of up to kMaxSeg problems: segment s holds the
// problem's box records, its work list (march units or tag chunks, with box
// and tag indices local to the problem), its tags and its record; items
// beg[s] .. beg[s+1]-1 of the launch are items 0.. of segment s.  Passed by
// value as a kernel argument, so a launch needs no device table of its own.
constexpr int kMaxSeg = 16;
struct Seg {
  const BoxRec* boxes;
  const void* work;
  const void* tags;
  ProbDev* P;
};
struct Segs {
  int n;
  int beg[kMaxSeg + 1];
  Seg s[kMaxSeg];
};

// Same-level ghost copy: dst-local cells [lo, lo+ext) <- src-local (cell + off).
struct FillTag { int dst, src; int lo[3]; int ext[3]; int off[3]; int pad; };
// Physical boundary along dir on one side of the domain, over a box's grown cells.
struct BcTag { int box; int dir; int side; int bc; int lo[3]; int ext[3]; int dom_lo, dom_hi; double inflow[kMaxV]; };

// Two-level problems (ratio 2).  The fine level is one rectangle of fine
// boxes covering coarse cells clo..chi; the coarse cells clo-3..chi+3 (the
// "region") are gathered from the coarse boxes at t^n and t^{n+1} for the
// coarse-to-fine ghost interpolation.
struct GatherTag { int box; int lo[3]; int ext[3]; int roff[3]; };   // box-local valid cells -> region offset
struct CfTag { int box; int lo[3]; int ext[3]; int pad; };           // fine box-local ghost cells to interpolate
// A coarse face on the patch boundary: the coarse box holding the uncovered
// neighbour cell, the face and that cell in its box-local index, the fine box
// holding the four fine sub-faces and the first sub-face in its box-local
// index; register slot = index of the face in the list.
struct RegFace { int d, side, cbox, fbox; int cface[3]; int ucell[3]; int fface[3]; int pad; };
// Coarse cells covered by one fine box: coarse box-local range and the fine
// box-local index of the first child.
struct AvgTag { int cbox, fbox; int clo[3]; int ext[3]; int flo[3]; int pad; };

// Regrid of a fine level: cells [lo, lo+ext) of new fine box `box` (box-local)
// are copied from old fine box `src` (>= 0) or interpolated from the gathered
// coarse region (src = -1).
struct ProlongTag { int box, src; int lo[3]; int ext[3]; };

struct TwoLevelArgs {
  const BoxRec* cboxes;
  const BoxRec* fboxes;
  ProbDev* Pc;
  ProbDev* Pf;
  double* ct0;      // region state at t^n
  double* ct1;      // region state at t^{n+1}
  double* reg;      // per face: dt_c F_c (nv), fine sum S (nv)
  int rlo[3];       // region origin (coarse index)
  int rext[3];      // region extent
};

// Scratch layout per box, in doubles, with nv = 5 + nspec components:
// q ((6 + nspec) x grown: rho, u, v, w, p, c, X_s), phi (1 x halo-1),
// ql[3], qr[3], fn[3], f1[6], ff[3] (nv x halo-1 each).  A halo-1 plane
// (cells -1..n in x and y) is padded to a multiple of 16 doubles, so every
// plane and every component starts on a 128-byte line: a wave storing 64
// consecutive cells of a plane then writes whole lines (partial-line stores
// cost HBM write bandwidth).
__host__ __device__ inline long long grown_cells(const int n[3]) {
  return (long long)(n[0] + 2 * kNG) * (n[1] + 2 * kNG) * (n[2] + 2 * kNG);
}
__host__ __device__ inline int h1_plane(const int n[3]) { return ((n[0] + 2) * (n[1] + 2) + 15) & ~15; }
__host__ __device__ inline long long h1_cells(const int n[3]) { return (long long)h1_plane(n) * (n[2] + 2); }
__host__ __device__ inline long long scratch_doubles(const int n[3], int nspec) {
  return (6 + nspec) * grown_cells(n) + (1 + 18 * (kNV + nspec)) * h1_cells(n);
}

// ---------------------------------------------------------------- launchers
enum Stage : int {
  kStFill = 0, kStBcX, kStBcY, kStBcZ, kStC2P, kStCfl, kStC2POnly, kStDt, kStFlatten,
  kStTraceX, kStTraceY, kStTraceZ, kStRiemX, kStRiemY, kStRiemZ, kStT1X, kStT1Y, kStT1Z,
  kStT2X, kStT2Y, kStT2Z, kStUpdate, kStFlip,
  kStReconX, kStReconY, kStReconZ, kStMolUpdate, kStTrace3, kStT1All, kStRecon3, kStSpec3, kNumStages
};

// State array a stage reads (fill, boundaries, cons->prim, MOL stages) or
// the MOL update writes: the current fab, a Runge-Kutta stage fab, or the
// other fab (which receives the new state).
enum Arr : int { kArrCur = 0, kArrW0 = 1, kArrW1 = 2, kArrNext = 3 };

// Region each march stage runs over.
__host__ __device__ inline int stage_region(int stage) {
  switch (stage) {
    case kStC2P: case kStC2POnly: return kGrown;
    case kStCfl: return kValid;
    case kStFlatten: return kCells1;
    case kStT1All: return kCells1;
    case kStTrace3: case kStRecon3: case kStSpec3: return kCells1T;
    case kStTraceX: case kStTraceY: case kStTraceZ: return kCells1;
    case kStReconX: case kStReconY: case kStReconZ: return kCells1;
    case kStMolUpdate: return kValid;
    case kStRiemX: case kStRiemY: return kCells1;  // whole rows / planes of stores
    case kStT1X: return kFace0;
    case kStT1Y: return kFace1;
    case kStRiemZ: case kStT1Z: return kFace2;
    case kStT2X: return kFin0;
    case kStT2Y: return kFin1;
    case kStT2Z: return kFin2;
    case kStUpdate: return kValid;
    default: return -1;
  }
}

struct Launch {
  Segs segs;           // problems, their work lists and tags
  int grid;            // blocks (multiple of 8)
  hipStream_t stream;
  int arr = kArrCur;   // array read by fill / boundaries / cons->prim / MOL update
  int out = kArrNext;  // array the MOL update writes
  int comb = 0;        // MOL update: combine with the current fab (U0 + c (T - U0))
  double c = 0.0;      // its weight
  int last = 1;        // MOL update: the step's last stage (test hook applies)
  int rs = 0;          // Riemann solver of the flux stages: 0 HLLC, 1 two-shock
  int lim = 0;         // reconstruction variant: 0 CW84, 1 Colella & Sekora, 2 CW84 + contact steepening
  int sp = 0;          // a problem of the launch carries passive species (merged tracing and stage 1)
  int mol = 0;         // method-of-lines scheme (the species stage stores edge values)
  int spstage = 0;     // the species stage traces the species (the merged kernels leave them)
};

hipError_t launch_stage(int stage, const Launch& L);
// Two-level kernels: gather (which: 0 = state at t^n into ct0, 1 = new state
// into ct1), coarse-to-fine interpolation at theta, register init from the
// coarse fluxes, register accumulation of the fine fluxes, average down,
// reflux, and the two-level dt.
hipError_t launch_gather(const TwoLevelArgs& A, const GatherTag* tags, const Chunk* chunks, int n, int which,
                         hipStream_t s);
hipError_t launch_cfinterp(const TwoLevelArgs& A, const CfTag* tags, const Chunk* chunks, int n, double theta,
                           hipStream_t s);
hipError_t launch_reg_coarse(const TwoLevelArgs& A, const RegFace* faces, int n, hipStream_t s);
hipError_t launch_reg_fine(const TwoLevelArgs& A, const RegFace* faces, int n, hipStream_t s);
hipError_t launch_avgdown(const TwoLevelArgs& A, const AvgTag* tags, const Chunk* chunks, int n, hipStream_t s);
hipError_t launch_reflux(const TwoLevelArgs& A, const RegFace* faces, int n, hipStream_t s);
hipError_t launch_dt2(ProbDev* Pc, ProbDev* Pf, hipStream_t s);
// Regridding: density-jump tags of level-0 valid cells into a dense domain
// array (dn = domain extent, dlo = its first index), and the new fine state
// of a regrid.
hipError_t launch_tag(const Segs& L, int grid, double threshold, unsigned char* tags, const int dn[3],
                      const int dlo[3], hipStream_t s);
hipError_t launch_prolong(const TwoLevelArgs& A, const BoxRec* newf, const BoxRec* oldf, const ProlongTag* tags,
                          const Chunk* chunks, int n, hipStream_t s);
// dt of every problem of the segments from its signal-speed slots (or its fixed dt).
hipError_t launch_dt(const Segs& L, hipStream_t s);
hipError_t launch_set_dt(ProbDev* Pc, ProbDev* Pf, const double* dt, hipStream_t s);
// Commit the new state of every problem of the segments (flip the current
// fab, count the step).  guard = 1: a problem whose failure count grew during
// the step keeps its old state and counts a rejection instead.
hipError_t launch_flip(const Segs& L, int guard, hipStream_t s);
const char* stage_name(int stage);
// Streaming probe over `bytes` (a multiple of 16): kind 0 copies src to dst,
// 1 reads src, 2 writes dst; `blocks` blocks of 256 threads, grid-stride.
hipError_t launch_probe(int kind, const void* src, void* dst, size_t bytes, int blocks, hipStream_t s);
// Stage scratch of the allocation-free step (a file-scope device array of
// kStaticScratchBytes): its address on device `dev`, which must be the
// current device (taken once per device with hipGetSymbolAddress).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(int dev, void** ptr);

}  // namespace ctu
