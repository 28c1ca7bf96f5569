// Internal declarations shared by the host side (ec_capi.hip) and the
// kernels (ec_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ec {

// Mixed-radix plan of one x transform of length n (radices in pass order).
constexpr int kMaxRadices = 32;
struct FftPlan {
  int n;
  int nr;
  int r[kMaxRadices];
};

// The x transforms run in place in one LDS buffer (each pass reads its inputs
// into registers, the block synchronises, the outputs overwrite the buffer)
// when every radix has a register butterfly and a pass gives each thread at
// most kFftPerThread elements; otherwise they ping-pong between two buffers.
// (Kernels built for fewer elements per thread need fewer registers.)
constexpr int kFftPerThread = 16;
__host__ __device__ inline bool fft_in_place(const FftPlan& pl, int threads, int per_thread = kFftPerThread) {
  for (int p = 0; p < pl.nr; ++p) {
    const int r = pl.r[p];
    if (r != 2 && r != 3 && r != 4 && r != 5 && r != 8) return false;
  }
  return pl.n <= per_thread * threads;
}

// Rows per collide tile, a function of the grid alone: the tile edges fix
// the summation order of the next step's charge density, so the launch
// shape must not move them.  One row below 512 rows; ny / 256 rows up to
// 4095 rows (256 tiles, one round of one tile per CU); eight rows from 4096
// rows on (two or more rounds: at 4096 x 4096 the 512 tiles of 8 rows run
// the collide in 496 us against 502 with 256 tiles of 16, and the whole
// step 4-5 us faster in every precision; heights that leave a round partly
// empty are slower: 12 rows, 625 us).
__host__ __device__ inline int tile_rows(int ny) { return ny < 512 ? 1 : (ny < 4096 ? ny / 256 : 8); }

// Bands of rows reduced by separate blocks in the diagnostics.
constexpr int kStatsBands = 1024;

// Doubles per row of a batch slot's diagnostics history: step, rms u_y,
// max |u|, sum of rho_c, amplitude of the first x mode of u_y (lattice
// units), number of unhealthy nodes (non-finite moments or rho <= 0), the
// collector current (charge the next streaming takes out through the upper
// electrode, lattice units).
constexpr int kHistCols = 7;

// LDS of one workgroup on gfx950.
constexpr size_t kMaxLds = 160 * 1024;

// Rows per chunk of the partitioned per-wavenumber solves.
constexpr int kChunk = 32;
// Chunk types: the whole column (one chunk), the first one (lower electrode
// ghost row), an interior one, the last one (upper electrode ghost row).
enum ChunkType { CH_SINGLE = 0, CH_FIRST = 1, CH_INTERIOR = 2, CH_LAST = 3 };

// Scalar constants of one instance, in lattice units (see the public header
// for the unit conventions).  Kernels convert to their storage type.
struct Consts {
  int nx, ny;  // grid
  int P;       // row pitch of node arrays, elements
  int M;       // number of non-negative x wavenumbers, nx/2 + 1
  int MP;      // row pitch of spectral arrays, elements
  int NC;      // number of y chunks, ceil(ny / kChunk)
  int KP;      // row pitch of the interface factor table (NC - 1 rounded up to 8)
  int TH;      // rows per collide tile (tile_rows(ny))
  int TW;      // columns per collide tile (nx: whole rows; set per launch from the tuning, results do not depend on it)
  double wp, wm, wgp, wgm;  // TRT rates: fluid +/-, charge +/-
  double K;                 // ion mobility
  double eps;               // permittivity
  double bx;                // body force density along x
  double H;                 // electrode gap (= ny)
  double u0;                // velocity unit K / H
  // slope s of the reference density rho_ref(y) = 1 + s (y - H/2); the
  // reference force s/3 balances it.  The fluid populations are stored as
  // deviations from f_ref,i = w_i (rho_ref - (s/2) c_iy) before collision and
  // from w_i (rho_ref + (s/2) c_iy) after it, the exact fixed point of the
  // forced TRT step with halfway bounce-back for that density and force.
  double s_ref;
  // slope of the initial density profile, 1 + s_init (y - H/2); the same in
  // every precision (s_ref is rounded coarser for FP32 storage)
  double s_init;
  // injector anti-bounce-back constants 2 (w_i rho0 - R_i(0)) on deviations
  double g_abb_axis, g_abb_diag;
  // initial state
  int init_mode;
  double noise_amp;
  uint64_t seed;
};

// The interface system of the y solves is solved by recursive doubling (one
// wave per wavenumber, kScanPerLane interfaces per lane) when it has at most
// kScanMax interfaces (8224 rows), and by a serial block elimination
// otherwise.  Four per lane rather than eight: shorter serial parts per lane
// and fewer registers (2 us faster at 4096 rows).
constexpr int kScanPerLane = 4;
constexpr int kScanMax = 64 * kScanPerLane;

// Factors of the interface system per (m, k), in this order (table rf).
enum ReducedFactor { RF_INV = 0, RF_IB, RF_A, RF_P, RF_Q, RF_C, RF_G, RF_COUNT };

// Row bands of collide tiles (one edge row each way per band).
__host__ __device__ inline int collide_tiles(const Consts& c) { return (c.ny + c.TH - 1) / c.TH; }
// Column tiles per band, and blocks of one collide launch (band-major: the
// column tiles of a band are consecutive blocks).
__host__ __device__ inline int collide_xtiles(const Consts& c) { return (c.nx + c.TW - 1) / c.TW; }
__host__ __device__ inline int collide_blocks(const Consts& c) { return collide_tiles(c) * collide_xtiles(c); }

// Columns per collide tile: by default whole rows while their ten LDS rows
// fit one workgroup (nx <= 4096 in FP32 storage, 2048 in FP64: measured
// faster than narrower tiles, which collide two halo columns per row in a
// second round), tiles of kTileW columns (with recomputed halo columns)
// beyond; `req` > 0 asks for a width.
constexpr int kTileW = 1024;
__host__ __device__ inline int tile_width(int nx, int req, int tsize) {
  if (req > 0) return nx <= req ? nx : req;
  return 10 * (long long)nx * tsize <= 160 * 1024 ? nx : (nx <= kTileW ? nx : kTileW);
}

// Per-row tables in the storage type (index k * ny + j).
enum RowTable {
  ROW_RHO_REF = 0,   // hydrostatic reference density rho_ref(j)
  ROW_R = 1,         // reference charge row r(j)
  ROW_DG_UP_AXIS,    // R_axis(j-1) - R_axis(j): g arriving from below
  ROW_DG_UP_DIAG,
  ROW_DG_DN_AXIS,    // R_axis(j+1) - R_axis(j): g arriving from above
  ROW_DG_DN_DIAG,
  ROW_KQ,            // sum of the constants the pull adds to the charge populations of row j
  ROW_COUNT
};

// Per-row tables in FP64 (index k * ny + j).
enum RowTableD {
  ROWD_RHO_REF = 0,  // rho_ref(j)
  ROWD_R = 1,        // r(j)
  ROWD_RC_CLOSED,    // closed-form charge profile (initial state)
  ROWD_DCSUM,        // sum over x of the charge deviation (written each step)
  ROWD_EYM,          // x-mean field E_y(j) (written each step)
  ROWD_PHIM,         // x-mean potential (written each step)
  ROWD_DFY,          // r(j) E_y mean(j) - s/3: x-mean force less the reference force
  ROWD_RNEXT,        // r(j) of a new T while the state is re-referenced to it
  ROWD_COUNT
};

// Device pointers of one instance inside the caller's workspace.
struct Bufs {
  void* f[2];    // [9][ny][P] populations (deviations), ping-pong
  void* g[2];
  void* phi;     // [ny][P] potential fluctuation (m >= 1 modes)
  void* spec;    // [ny][MP] complex spectrum (forward, then chunk solutions in place)
  void* tt;      // [4 types][3: cp, v, w][kChunk][MP] chunk tables of the y solves
  void* ends;    // [P][2][MP] complex: first / last row of each chunk's local solution
  void* gh;      // [P][6][MP]: block-elimination scratch of the interface system
  void* rf;      // [MP][7][KP]: data-independent factors of the interface system
  void* rq;      // [ny][P] charge density deviation of the next step, summed by the collide tiles
  void* eu;      // [tiles][P] contribution of each tile's last row to the row above it
  void* ed;      // [tiles][P] contribution of each tile's first row to the row below it
  void* iface;   // [P][2][MP] complex: interface values a_k (last row of chunk k),
                 //                      b_k (first row of chunk k+1)
  void* tw;      // [nx] complex twiddles exp(-2 pi i k / nx), then [<= nx] pass-major ones
  void* twy;     // the same for the length 2 ny of the spectral y solve
  void* rows;    // ROW_COUNT x [ny]
  double* rowsd; // ROWD_COUNT x [ny]
  double* dmean; // [ny + 1] x-mean row differences D(-1) .. D(ny-1)
  double* mom;   // [4][ny][nx] emitted moments: rho - rho_ref, ux, uy, rho_c - r
  double* stats; // [16]
  double* spart; // [kStatsBands][8] partial diagnostics of bands of rows
};

// One slot of a batch: an instance's constants, buffers and transform plan,
// and its step state, which the device advances so that a captured
// multi-step graph needs no host updates between steps.
struct SlotDesc {
  Consts c;
  Bufs b;
  FftPlan plan;
  int cur;             // buffer holding the latest post-collision populations
  int active;          // 1 while steps_done < steps_target
  int emit_every;      // moments and diagnostics every emit_every steps and at the end
  int hist_cap;        // rows of the diagnostics history
  long long steps_done, steps_target;
  double* hist;        // [hist_cap][kHistCols], see kb_stats_advance
};

// Launch shapes that do not change results: threads per x-transform block
// and per collide tile (cbx * cby threads, a multiple of 64 up to 1024).
struct Tuning {
  int fft_threads = 256;
  int cbx = 256, cby = 1;
  int ctw = 0;  // columns per collide tile (0: tile_width's default)
};

// Batched kernels; slot s owns the blocks [off[k][s], off[k][s+1]) of launch k.
enum BatchKernel { BK_FORWARD = 0, BK_TRI_LOCAL, BK_TRI_REDUCED, BK_INVERSE, BK_COLLIDE, BK_STATS, BK_COUNT };

// Blocks that kernel k uses for one instance (independent of the launch
// shapes, so that a block-to-slot table never depends on the tuning).
int batch_blocks(const Consts& c, int k);

// Enqueues one batched step (all kernels, then the device-side advance) for
// ns slots.  d_off holds BK_COUNT rows of ns + 1 offsets; totals[k] is the
// block count of launch k; lds the dynamic LDS of the transforms.
// fft8: every slot's transform fits eight elements per thread (the lighter
// kernel build).
template <typename T, typename C>
hipError_t launch_batch_step(const SlotDesc* d_desc, const int* d_off, const int* totals, int ns, size_t lds,
                             size_t collide_lds, bool fft8, const Tuning& tu, hipStream_t s);

// Kernel launchers (ec_kernels.hip).  All enqueue on `s` and return the
// launch status.
template <typename T>
hipError_t launch_init_charge(const Consts& c, const Bufs& b, hipStream_t s);
template <typename T>
hipError_t launch_init_populations(const Consts& c, const Bufs& b, int dst, hipStream_t s);
// mode 0: pull-gather from post-collision g[src]; 1: local sum of g[src];
// 2: read the charge deviation field held in b.mom (plane 3)
template <typename T>
hipError_t launch_forward(const Consts& c, const Bufs& b, const FftPlan& pl, int mode, int src,
                          const Tuning& tu, hipStream_t s);
// chunk-local solves of the m >= 1 y systems, then the interface system
// (the chunk corrections, and the x-mean mode, are done by launch_inverse)
template <typename T>
hipError_t launch_tridiag(const Consts& c, const Bufs& b, hipStream_t s);
template <typename T>
hipError_t launch_inverse(const Consts& c, const Bufs& b, const FftPlan& pl, const Tuning& tu, hipStream_t s);
// T: storage type of the populations, C: arithmetic type of the collision
template <typename T, typename C>
hipError_t launch_collide(const Consts& c, const Bufs& b, bool pull, bool emit, int src, int dst,
                          const Tuning& tu, hipStream_t s);
template <typename T>
hipError_t launch_fields(const Consts& c, const Bufs& b, double* rho, double* ux, double* uy,
                         double* rho_c, double* phi, double* rho_m1, hipStream_t s);
template <typename T>
hipError_t launch_charge_in(const Consts& c, const Bufs& b, const double* rho_c_nd, hipStream_t s);
// cur: the buffer holding the post-collision populations (boundary charge)
template <typename T>
hipError_t launch_stats(const Consts& c, const Bufs& b, int cur, hipStream_t s);

// Continuation at another T: the post-collision charge populations g[cur]
// and the charge moment become scale (their reference + themselves) less the
// new reference, with the old reference row in ROWD_R and the new one in
// ROWD_RNEXT; the fluid deviations f[cur] and the density moment follow the
// change ddelta of the storage rounding of the reference force slope.
template <typename T>
hipError_t launch_continue(const Consts& c, const Bufs& b, int cur, double scale, double ddelta, hipStream_t s);
// The charge density rows the next step reads (what the collide tiles form
// from the populations they write), formed from the stored g[cur].
template <typename T>
hipError_t launch_density(const Consts& c, const Bufs& b, int cur, const Tuning& tu, hipStream_t s);

// Spectral y solve of the m >= 1 modes (Eq. 21-25), in place of the chunked
// tridiagonal one: py is the plan of length 2 ny, b.twy its twiddles.
template <typename T>
hipError_t launch_yspec(const Consts& c, const Bufs& b, const FftPlan& py, hipStream_t s);
// Its LDS bytes (two buffers of 2 ny complex values).
template <typename T>
size_t yspec_lds_bytes(int ny);

// LDS bytes of a collide tile (ten rows of nx values of T).
template <typename T>
size_t collide_lds_bytes(int tw, int nx);

// LDS bytes of the x-transform kernels for plan pl on blocks of `threads`.
template <typename T>
size_t fft_lds_bytes(const FftPlan& pl, int threads);

}  // namespace ec
