// Private declarations of libconvreal: the plan and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/convreal.h"

namespace convreal {

// Per-thread message for conv_real_last_error().
void set_error(const std::string& msg);
// Records the message of a failed HIP call, clears the runtime's sticky error and returns the
// matching error code (ENOMEM for out-of-memory, EHIP otherwise).
int hip_fail(hipError_t e, const char* what);
// The current device if it is a gfx950 (ENODEV otherwise).
int check_device(int* dev_out);
// Grid, precision and device of a valid plan (EINVAL otherwise).
int plan_info(const conv_real_plan* p, int* nside, int* precision, int* device);

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  hipError_t enter(int dev) {
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != dev) {
      e = hipSetDevice(dev);
      if (e != hipSuccess) return e;
      changed = true;
    }
    return hipSuccess;
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};


// Device buffer owned by a plan.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Ring grid of the ring-ordered pixelization, host side, FP64 plus exact integers.
// z_i = Z_i / (3 N^2) with Z_i an integer; sin(theta_i) = sqrt((3N^2 - Z_i)(3N^2 + Z_i)) / (3N^2);
// pixel a of ring i sits at phi = pi (2a + c_i) / n_i with c_i in {0, 1}.
struct RingGrid {
  int nside = 0;
  int nrings = 0;
  long long npix = 0;
  std::vector<long long> Z;     // numerator of z
  std::vector<double> z;        // z_i
  std::vector<double> s;        // sin(theta_i)
  std::vector<int> n;           // pixels in ring
  std::vector<int> c;           // azimuth offset numerator
  std::vector<long long> start; // first pixel index
};

RingGrid make_ring_grid(int nside);

// Neighbour ring ranges: ring r sees rings jlo[r]..jhi[r] (0-based, contiguous).
void neighbour_rings(const RingGrid& g, double dcut2, std::vector<int>& jlo, std::vector<int>& jhi);

constexpr int kMaxSlots = 64;  // maps per persistent mixed-path launch
constexpr int kXcds = 8;        // accelerator complex dies of the MI355X, each with its own L2
constexpr int kMaxChunks = 16; // work-queue chunks
// K-chunks (32 window offsets) of one belt weight block: the LDS stage holds one block's window;
// wider windows of one input ring are split into several blocks
constexpr int kBeltBlockChunks = 4;
// 16-row blocks per cap tile when the plan holds a weight store: the blocks of a tile share every
// step's inputs and every ring pair's set-up (the cap items are bound by vector instruction issue),
// and each block adds its weight registers to every pipeline slot
constexpr int kStoreBlocks = 2;
// per cap store tile: first group (low bits) and a flag for tiles where some ring pair's inputs
// wrap around the input ring for some lane (the apply takes them one step at a time)
constexpr long long kTileWraps = 1LL << 62;
constexpr long long kTileOffsetMask = kTileWraps - 1;
// the per-pair kernel stages the table as cubic coefficients (4 doubles per segment, 64 KB of LDS)
// up to this many segments, as nodes beyond
constexpr int kCoefMaxSegs = 2048;

// One cap-touching ring pair (output ring i, input ring j) as the mixed path's cap tiles read it:
// one 64-byte record, fetched with a single scalar load per pair and tile.
struct CapPair {
  double A;          // (z_i - z_j)^2 + (s_i - s_j)^2
  double B;          // 4 s_i s_j
  double hw;         // window half-width in pixels of ring j
  double scale;      // half azimuth difference per unit of the integer numerator: pi / (2 n_i n_j)
  long long xoff;    // first pixel of ring j
  long long xoff_m;  // first pixel of the north/south mirror of ring j
  int nj;            // pixels of ring j
  int cj;            // azimuth offset numerator of ring j
  int whole;         // 1 if the window is the whole ring (2 hw >= n_j)
  int pad;
};
static_assert(sizeof(CapPair) == 64, "CapPair is one 64-byte record");

// One cap-touching ring pair as the ring-FFT method's FP64 cap kernel reads it: one 64-byte record,
// fetched with a single scalar load per pair and tile (pixel offsets fit 32 bits: Nside <= 2048).
struct CapPair64 {
  double A;          // (z_i - z_j)^2 + (s_i - s_j)^2
  double B;          // 4 s_i s_j
  double hw;         // window half-width in pixels of ring j
  double sd;         // sin(pi / n_j)
  double cd;         // cos(pi / n_j)
  int nj;            // pixels of ring j
  int cj;            // azimuth offset numerator of ring j
  int xoff;          // first pixel of ring j
  int xoff_m;        // first pixel of the north/south mirror of ring j
  int pad[2];
};
static_assert(sizeof(CapPair64) == 64, "CapPair64 is one 64-byte record");

// Everything the mixed path's device routines read about one plan (lives in device memory).
struct MixedDesc {
  // geometry
  const int* rn;
  const int* rc;
  const long long* rstart;
  int nrings;
  int ring_n;                 // 4N
  long long npix;
  // belt ring pairs
  const _Float16* wt;
  const int* blk_j;           // per weight block: input ring
  const int* band_nj;         // per band: weight blocks
  const int* band_woff;
  const int* blk_koff;
  const int* blk_nk;
  const int* blk_mlo;
  int belt_lo;
  int belt_hi;
  const int* ring_add;        // per ring: receives a belt and a cap-pair contribution
  long long zero_lo[2];       // pixel ranges of such rows (zeroed before the launch)
  long long zero_hi[2];
  // cap-touching ring pairs
  const float* coef;          // per segment: 4 FP32 cubic coefficients x Omega x s_w
  int nseg;
  int n_citems;
  const int* citem_ring;
  const int* citem_a0;
  const long long* rest_off;  // per ring: first record in cpair
  const CapPair* cpair;       // cap-touching ring pairs, grouped by output ring
  const void* wstore;         // cap weight store, 16-byte groups (nullptr: weights evaluated on the fly)
  const long long* wtile_off; // per cap tile: first group of the tile in wstore
  double inv_h;
  double dcut2;
  float inv_sw;
};

// Per-launch map slots of the persistent kernel (passed by value).
struct Slots {
  const MixedDesc* desc[kMaxSlots];
  const float* x[kMaxSlots];
  float* y[kMaxSlots];
};

// Launch configuration of the persistent kernel (see conv_real_tuning).
struct Tuning {
  int seg = 256;       // belt output pixels per work item: 256 or 512
  int wg_per_cu = 3;   // resident workgroups per compute unit
  int order = 3;       // 0: all items by decreasing cost; 1: belt and cap items alternating;
                       // 2: one chunk per XCD of neighbouring rings, each by decreasing cost;
                       // 3: roles (a belt chunk, two cap chunks); 4: roles with the cap items in one
                       // chunk of neighbouring rings per XCD
};

// Events recorded between kernels by conv_real_profile.
struct Recorder {
  static constexpr int kMax = 32;
  hipEvent_t ev[kMax + 1];
  const char* name[kMax];
  long long work[kMax];
  int n = 0;
};

}  // namespace convreal

// The opaque plan of the C ABI.
struct conv_real_plan {
  int magic = 0;
  int device = 0;
  int nside = 0;
  int precision = 0;
  int n_tab = 0;
  int nrings = 0;
  long long npix = 0;
  double theta_cut = 0.0;
  double dcut = 0.0;
  double dcut2 = 0.0;
  double h = 0.0;
  double inv_h = 0.0;
  double omega = 0.0;
  long long pairs = 0;
  long long npairs_ring = 0;   // number of (output ring, neighbour ring) pairs
  int ntiles = 0;              // output tiles of the plain kernel

  // device arrays (plain path)
  double* d_table = nullptr;   // n_tab
  double* d_coef64 = nullptr;  // (n_tab - 2) x 4: cubic coefficients per segment (null: n_tab > 2050)
  int* d_rn = nullptr;         // per ring
  int* d_rc = nullptr;
  long long* d_rstart = nullptr;
  double* d_rcd = nullptr;     // cos(pi / n)
  double* d_rsd = nullptr;     // sin(pi / n)
  long long* d_Z = nullptr;
  double* d_s = nullptr;
  long long* d_poff = nullptr; // nrings + 1, CSR offsets into ring-pair arrays
  int* d_jlo = nullptr;        // per ring
  int* d_pi = nullptr;         // per ring pair: output ring
  int* d_pj = nullptr;         // per ring pair: neighbour ring
  double* d_pA = nullptr;      // per ring pair: (dz)^2 + (ds)^2
  double* d_pB = nullptr;      // per ring pair: 4 s_i s_j
  double* d_phw = nullptr;     // per ring pair: window half-width in pixels of ring j
  int* d_tile_ring = nullptr;  // per tile
  int* d_tile_a0 = nullptr;    // per tile
  unsigned long long* d_count = nullptr;

  // mixed path: belt ring pairs on the matrix cores, the rest (cap-touching pairs) per pair
  int belt_enabled = 0;
  int belt_lo = 1;             // belt output rings [belt_lo, belt_hi] (0-based); empty if disabled
  int belt_hi = 0;
  int belt_nk = 0;             // largest number of K-chunks (32 window offsets) of any block
  int belt_nbands = 0;         // bands of 16 output rings
  int belt_nsegs = 0;          // 256-pixel segments per ring
  long long n_wblk = 0;        // weight blocks (band, input ring)
  long long n_chunks = 0;      // K-chunks over all weight blocks
  double belt_sw = 1.0;        // power-of-two weight scale
  int* d_blk_j = nullptr;      // per weight block: input ring
  int* d_band_nj = nullptr;    // per band: number of weight blocks (input rings, wide windows split)
  int* d_band_woff = nullptr;  // per band: first weight block
  int* d_blk_koff = nullptr;   // per weight block: first K-chunk
  int* d_blk_nk = nullptr;     // per weight block: K-chunks
  int* d_blk_mlo = nullptr;    // per weight block: first window offset m = b - a
  int* d_chunk_band = nullptr; // per K-chunk
  int* d_chunk_j = nullptr;
  int* d_chunk_m0 = nullptr;
  _Float16* d_wt = nullptr;    // n_chunks * 1024 FP16
  unsigned* d_amax = nullptr;  // per map (up to kMaxMixedMaps): max |x| bits
  long long* d_rest_off = nullptr;   // per ring: CSR offsets into d_rest_idx
  long long* d_rest_idx = nullptr;   // ring-pair indices handled per pair
  int* d_rtile_ring = nullptr;
  int* d_rtile_a0 = nullptr;
  int n_rtiles = 0;
  long long pairs_rest = 0;    // pixel pairs per map that touch a polar cap
  // cap-touching ring pairs on the matrix cores (on-the-fly FP32 weights, 16 symmetric images)
  int cap_mode = 0;            // 1: cap_mfma_kernel; 0: FP64 per-pair remainder kernel
  float* d_coef = nullptr;     // (n_tab - 2) x 4: per-segment cubic coefficients x Omega x s_w
  int* d_citem_ring = nullptr; // per cap tile: output ring (north half)
  int* d_citem_a0 = nullptr;   // per cap tile: first pixel (tiles of cap_rows pixels)
  int n_citems = 0;
  int cap_rows = 16;           // 16, or 16 kStoreBlocks while the plan holds a weight store
  std::vector<int> cap_F;      // per ring: fundamental-domain pixels if it has cap-touching pairs, else 0
  std::vector<double> cap_ring_cost;   // per ring: estimated cycles of one 16-row tile
  convreal::CapPair* d_cpair = nullptr;  // per cap-touching ring pair, in d_rest_idx order
  // cap weight store: per cap tile, ring pair and row inside the fundamental domain, the row's
  // weights in 16-byte groups of 4 inputs (FP16 hi x 4, FP16 lo x 4) that meet the row's window
  uint4* d_wstore = nullptr;
  long long* d_wtile_off = nullptr;  // per cap tile: first group
  long long wstore_groups = 0;
  int wstore_mode = 2;               // CONV_REAL_STORE_OFF / ON / AUTO as last requested
  convreal::MixedDesc h_desc{};      // host copy of d_desc
  int* d_ring_add = nullptr;   // per ring: 1 if it gets a belt and a cap-pair contribution
  int cap_nseg = 0;            // coefficient segments (n_tab - 2) if cap_mode
  convreal::MixedDesc* d_desc = nullptr;  // device copy of the plan's descriptor
  convreal::Tuning tune;
  int tune_user = 0;           // 1 once the caller set the launch configuration (or autotuned it)
  int2* d_items = nullptr;     // work queue of one map (slot 0), chunk after chunk
  int n_items = 0;
  int* d_qchunk_off = nullptr; // n_qchunks + 1 offsets into d_items
  int n_qchunks = 1;
  unsigned* d_counter = nullptr;   // kMaxChunks counters
  std::vector<double> cost_belt;   // per belt band: estimated cycles per 16-pixel column block
  std::vector<double> cost_cap;    // per cap work item (4 tiles): estimated cycles

  // ring-FFT method (FP64 plans): belt ring pairs through per-ring FFTs, the rest per pair
  int method = 0;              // CONV_REAL_METHOD_DIRECT or CONV_REAL_METHOD_RING_FFT
  int fft_n = 0;               // belt ring length 4 Nside (a power of two)
  int fft_logn = 0;
  long long fft_npairs = 0;    // belt ring pairs (north output ring, input ring), output-ring major
  double2* d_fft_tw = nullptr; // n / 2 twiddles exp(-2 pi i m / n)
  int* d_fft_pi = nullptr;     // per belt pair: output ring, input ring, chord constants
  int* d_fft_pj = nullptr;
  double* d_fft_pA = nullptr;
  double* d_fft_pB = nullptr;
  long long* d_fft_boff = nullptr;  // per north belt output ring: first belt pair, first pair whose input ring
                                    // has the other azimuth offset (+ 1 entry)
  double* d_fft_K = nullptr;   // per belt pair: n / 2 + 1 real spectrum amplitudes of k_ij (phase removed)
  double2* d_fft_X = nullptr;  // per belt ring: n / 2 + 1 frequencies of one map's ring (workspace)
  double2* d_fft_Y = nullptr;  // per belt ring: n / 2 + 1 frequencies of its output (workspace)
  long long fft_work_bytes = 0; // bytes of the two workspaces above
  convreal::CapPair64* d_fft_cpair = nullptr;  // per listed cap-touching pair (d_rest_idx order)
  int* d_mtile_ring = nullptr; // cap-touching pairs by symmetry: tiles of 16 fundamental-domain pixels
  int* d_mtile_a0 = nullptr;   // (one wave each) of the north-half rings that have such pairs
  int n_mtiles = 0;

  convreal::Recorder* rec = nullptr;  // set only inside conv_real_profile
  std::vector<void*> owned;    // every device allocation, freed by destroy
};

namespace convreal {
// Record a profiling event after a kernel launch (no-op unless conv_real_profile is running).
inline void mark(const conv_real_plan* p, hipStream_t st, const char* name, long long work) {
  Recorder* r = p->rec;
  if (!r || r->n >= Recorder::kMax) return;
  if (hipEventRecord(r->ev[r->n + 1], st) != hipSuccess) return;
  r->name[r->n] = name;
  r->work[r->n] = work;
  r->n += 1;
}
}  // namespace convreal

namespace convreal {

constexpr int kMaxMixedMaps = 64;  // maps per mixed-path launch (larger batches are chunked)

// Launchers (each in the translation unit that defines its kernel).
hipError_t launch_ring_window(const conv_real_plan* p, hipStream_t st);
hipError_t launch_pair_count(const conv_real_plan* p, bool remainder, hipStream_t st);
hipError_t launch_pair_accumulate(const conv_real_plan* p, const void* x, void* y, int nmaps,
                                  hipStream_t st);
hipError_t launch_remainder(const conv_real_plan* p, const float* x, float* y, int nmaps,
                            hipStream_t st);
hipError_t launch_remainder_f64(const conv_real_plan* p, const double* x, double* y, int nmaps, hipStream_t st);
hipError_t launch_cap_mfma64(const conv_real_plan* p, const double* x, double* y, int nmaps, hipStream_t st);
// ring-FFT method: spectra of the belt pairs' kernels (set-up), and an apply of FP64 maps
hipError_t ring_fft_spectra(const conv_real_plan* p);
hipError_t launch_ring_fft(const conv_real_plan* p, const void* x, void* y, int nmaps, hipStream_t st);
// the belt ring pairs of one FP32 map through the ring FFTs (a mixed plan on the ring-FFT method):
// writes the belt rings of y
hipError_t ring_fft_belt_f32(const conv_real_plan* p, const float* x, float* y, hipStream_t st);
hipError_t build_belt_weights(conv_real_plan* p);
size_t belt_stage_bytes(int seg);
size_t shared_lds_bytes(int nseg);
hipError_t set_lds_limits(int nseg);
hipError_t launch_mixed_queue(const conv_real_plan* mark_plan, const Slots& S, int nslots, const int2* items,
                              int n_items, int nrep, const int* chunk_off, int n_chunks, unsigned* amax,
                              unsigned* counter, const Tuning& tune, int max_nseg, long long npix_max,
                              long long pairs, bool fly, hipStream_t st, bool zero_rows = true);
hipError_t launch_mixed(const conv_real_plan* p, const float* x, float* y, int nmaps, hipStream_t st);
// the same apply with its per-launch scratch (max |x| per map slot, then the work-queue counters)
// at `amax` (kMaxSlots words) and `counter` (kMaxChunks words) instead of the plan's own
hipError_t launch_mixed(const conv_real_plan* p, const float* x, float* y, int nmaps, hipStream_t st,
                        unsigned* amax, unsigned* counter);
// Fixed device scratch of conv_real_apply_noalloc: a file-scope array in device memory (each device
// holds its own copy), resolved to its device address once per device with that device current.
constexpr int kNoallocScratchWords = 256;   // 1 KiB: kMaxSlots + kMaxChunks words used
constexpr int kNoallocMaxDevices = 64;
hipError_t noalloc_scratch_resolve(int device);
unsigned* noalloc_scratch(int device);      // nullptr until resolved on that device
// number of weights of each cap tile in the store (counts[n_citems]), and the store's fill
hipError_t cap_store_count(const conv_real_plan* p, long long* counts_dev);
hipError_t cap_store_fill(const conv_real_plan* p);
hipError_t tabulate_device(const double* k_ell, int lmax, double h, int n_tab, double* table_host);

}  // namespace convreal
