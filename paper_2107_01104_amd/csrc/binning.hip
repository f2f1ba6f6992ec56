// Particle binning: cell keys, a stable LSD radix sort of (key, index) pairs,
// the bin offset array, and permutation gathers/scatters.
//
// This is the GPU form of the paper's local particle ordering (Sec. 3.3.1,
// "Ordering the particles locally"): particles of one group are stored
// contiguously, groups in increasing order, with an offset array of size
// groups+1 whose last entry is the particle count.  The paper partitions by
// x3 slice with an incomplete Quicksort; here a group is a window of W cell
// layers of a T x T tile column (x3 fastest within a column, as the paper's
// slices), and the partition is a stable radix sort, so that ties keep their
// input order and the result is reproducible bit for bit.
#include "device_common.h"
#include "launch.h"

namespace ptk {

// ---------------------------------------------------------------------------
// keys and locate
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_keys(const double* __restrict__ X, int64_t n, int N,
                                              double invd, BinGeom g, uint32_t* __restrict__ keys,
                                              int* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double x1 = X[3 * i], x2 = X[3 * i + 1], x3 = X[3 * i + 2];
  if (!in_domain3(x1, x2, x3)) {
    atomicOr(flag, kFlagDomain);
    keys[i] = 0;
    return;
  }
  int c1, c2, c3;
  double t;
  locate(x1, N, invd, &c1, &t);
  locate(x2, N, invd, &c2, &t);
  locate(x3, N, invd, &c3, &t);
  keys[i] = bin_key(c1, c2, c3, g);
}

__global__ __launch_bounds__(256) void k_locate(const double* __restrict__ X, int64_t n3, int N,
                                                double invd, int32_t* __restrict__ cell,
                                                double* __restrict__ off, int* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n3) return;
  double x = X[i];
  if (!in_domain(x)) {
    atomicOr(flag, kFlagDomain);
    cell[i] = 0;
    if (off) off[i] = 0.0;
    return;
  }
  int c;
  double t;
  locate(x, N, invd, &c, &t);
  cell[i] = c;
  if (off) off[i] = t;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, one pass per digit
//   tile = 256 threads x 8 items; each wave owns 512 consecutive items and
//   ranks them in 8 rounds of 64 with a ballot-built "same digit" lane mask.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  uint32_t wpre = 0, tot = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) wpre += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  *total = tot;
  return wpre + x - v;
}

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kTile = kSortThreads * kSortItems;  // 2048

// n_dev (optional): the element count held on the device; n is then an upper
// bound that sized the grid, and tiles past the count contribute nothing.
// tiles of a sort of n elements, or of min(n, *n_dev) when the count lives on
// the device; the digit histograms are laid out [digit][tiles]
__device__ __forceinline__ int64_t sort_tiles(int64_t n, const uint32_t* n_dev) {
  if (n_dev) n = min(n, (int64_t)*n_dev);
  return (n + kTile - 1) / kTile;
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                    const uint32_t* __restrict__ n_dev, int shift, uint32_t mask,
                                                    uint32_t* __restrict__ hist, int64_t n_tiles) {
  if (n_dev) {
    n_tiles = sort_tiles(n, n_dev);
    if ((int64_t)blockIdx.x >= n_tiles) return;
    n = min(n, (int64_t)*n_dev);
  }
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int k = 0; k < kSortItems; ++k) {
    int64_t i = base + k * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, int64_t n,
    const uint32_t* __restrict__ n_dev, int shift, uint32_t mask, int bits, const uint32_t* __restrict__ prefix,
    int64_t n_tiles, uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  if (n_dev) {
    n_tiles = sort_tiles(n, n_dev);
    n = min(n, (int64_t)*n_dev);
  }
  if ((int64_t)blockIdx.x * kTile >= n) return;
  __shared__ uint32_t wcount[4][256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t scan_sh[4];
  __shared__ uint32_t skey[kTile], sval[kTile];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < 4 * 256; d += 256) (&wcount[0][0])[d] = 0;
  __syncthreads();
  const int64_t wbase = (int64_t)blockIdx.x * kTile + wave * (64 * kSortItems);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = wbase + r * 64 + lane;
    bool valid = i < n;
    uint32_t k = valid ? keys_in[i] : 0u;
    uint32_t v = valid ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
    uint32_t d = (k >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    uint32_t before = (uint32_t)__popcll(peers & lt_mask);
    uint32_t base = valid ? wcount[wave][d] : 0u;
    // every lane of this wave has read the running count before the leader of
    // each digit group adds the group's size
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wcount[wave][d] = base + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    key[r] = k;
    val[r] = v;
    rank[r] = valid ? base + before : 0xFFFFFFFFu;
  }
  __syncthreads();
  // exclusive prefix of the per-wave counts over waves, per digit, and the
  // start of each digit's run inside the tile
  uint32_t tile_count = 0;
  {
    for (int w = 0; w < 4; ++w) {
      uint32_t c = wcount[w][threadIdx.x];
      wcount[w][threadIdx.x] = tile_count;
      tile_count += c;
    }
  }
  uint32_t ntile;
  const uint32_t my_start = block_excl_scan_256(tile_count, scan_sh, &ntile);
  dstart[threadIdx.x] = my_start;
  __syncthreads();
  // the tile in digit order in LDS, then written out run by run: consecutive
  // threads write consecutive addresses of a digit's run
  for (int r = 0; r < kSortItems; ++r) {
    if (rank[r] == 0xFFFFFFFFu) continue;
    const uint32_t d = (key[r] >> shift) & mask;
    const uint32_t lp = dstart[d] + wcount[wave][d] + rank[r];
    skey[lp] = key[r];
    sval[lp] = val[r];
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < ntile; j += kSortThreads) {
    const uint32_t k = skey[j];
    const uint32_t d = (k >> shift) & mask;
    const uint64_t pos = (uint64_t)prefix[(int64_t)d * n_tiles + blockIdx.x] + (j - dstart[d]);
    keys_out[pos] = k;
    vals_out[pos] = sval[j];
  }
}

// exclusive scan of n uint32 (in place): block sums, scan of sums, apply
constexpr int kScanBlock = 1024;  // elements per block (256 threads x 4)


// length of a scan over sort histograms whose tile count lives on the device
// (cnt != NULL: 256 digits x sort_tiles(cap, cnt)), else n
__device__ __forceinline__ int64_t scan_len(int64_t n, const uint32_t* cnt, int64_t cap) {
  return cnt ? 256 * sort_tiles(cap, cnt) : n;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ a, int64_t n,
                                                     uint32_t* __restrict__ sums, const uint32_t* __restrict__ cnt,
                                                     int64_t cap) {
  n = scan_len(n, cnt, cap);
  if ((int64_t)blockIdx.x * kScanBlock >= n) return;
  __shared__ uint32_t sh[4];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  uint32_t s = 0;
  for (int k = 0; k < 4; ++k)
    if (base + k < n) s += a[base + k];
  uint32_t tot;
  block_excl_scan_256(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_top(uint32_t* __restrict__ sums, int64_t nb,
                                                  const uint32_t* __restrict__ cnt, int64_t cap) {
  if (cnt) nb = (scan_len(0, cnt, cap) + kScanBlock - 1) / kScanBlock;
  __shared__ uint32_t sh[4];
  uint32_t carry = 0;
  for (int64_t base = 0; base < nb; base += 256) {
    int64_t i = base + threadIdx.x;
    uint32_t v = i < nb ? sums[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_excl_scan_256(v, sh, &tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(256) void k_scan_apply(uint32_t* __restrict__ a, int64_t n,
                                                    const uint32_t* __restrict__ sums,
                                                    const uint32_t* __restrict__ cnt, int64_t cap) {
  n = scan_len(n, cnt, cap);
  if ((int64_t)blockIdx.x * kScanBlock >= n) return;
  __shared__ uint32_t sh[4];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  uint32_t v[4], s = 0;
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? a[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_excl_scan_256(s, sh, &tot) + sums[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) a[base + k] = ex;
    ex += v[k];
  }
}

// offsets[b] = first sorted index with key >= b, for b in [0, n_bins]
__global__ __launch_bounds__(256) void k_offsets(const uint32_t* __restrict__ skeys, int64_t n,
                                                 int64_t n_bins, uint32_t* __restrict__ offsets) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i > n) return;
  int64_t lo = (i == 0) ? -1 : (int64_t)skeys[i - 1];
  int64_t hi = (i == n) ? n_bins : (int64_t)skeys[i];
  if (hi > n_bins) hi = n_bins;  // keys are < n_bins by construction; never write past the array
  for (int64_t b = lo + 1; b <= hi; ++b) offsets[b] = (uint32_t)i;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather3(const T* __restrict__ in, const uint32_t* __restrict__ perm,
                                                 int64_t n, T* __restrict__ out) {
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  int64_t s = perm[k];
  out[3 * k] = in[3 * s];
  out[3 * k + 1] = in[3 * s + 1];
  out[3 * k + 2] = in[3 * s + 2];
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatterW(const T* __restrict__ in, const uint32_t* __restrict__ idx,
                                                  int64_t n, int width, T* __restrict__ out) {
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  int64_t d = idx[k];
  for (int e = 0; e < width; ++e) out[d * width + e] = in[k * width + e];
}

__global__ __launch_bounds__(256) void k_gather_u32(const uint32_t* __restrict__ in,
                                                    const uint32_t* __restrict__ perm, int64_t n,
                                                    uint32_t* __restrict__ out) {
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  out[k] = in[perm[k]];
}


// ---------------------------------------------------------------------------
// incremental re-binning (particles move less than a cell per step, so few
// change bins; only those are sorted, the rest keep their relative order)
// ---------------------------------------------------------------------------
// Tile of 2048 items: wave w owns items [512w, 512w + 512) of the tile in 8
// rounds of 64.  For each item: whether its key changed ("mover") and the
// number of movers before it in the tile.
struct TileMovers {
  uint32_t ok[kSortItems], nk[kSortItems], before[kSortItems];
  bool valid[kSortItems], mover[kSortItems];
  uint32_t total;
};

__device__ __forceinline__ void tile_movers(const uint32_t* okeys, const uint32_t* nkeys, int64_t n, TileMovers& t) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wbase = (int64_t)blockIdx.x * kTile + wave * (64 * kSortItems);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t run = 0;
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = wbase + r * 64 + lane;
    t.valid[r] = i < n;
    t.ok[r] = t.valid[r] ? okeys[i] : 0u;
    t.nk[r] = t.valid[r] ? nkeys[i] : 0u;
    t.mover[r] = t.valid[r] && t.ok[r] != t.nk[r];
    const uint64_t bal = __ballot(t.mover[r]);
    t.before[r] = run + (uint32_t)__popcll(bal & lt_mask);
    run += (uint32_t)__popcll(bal);
  }
  if (lane == 0) wsum[wave] = run;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) pre += wsum[w];
    tot += wsum[w];
  }
  for (int r = 0; r < kSortItems; ++r) t.before[r] += pre;
  t.total = tot;
}

__device__ __forceinline__ int64_t tile_item(int r) {
  return (int64_t)blockIdx.x * kTile + (threadIdx.x >> 6) * (64 * kSortItems) + r * 64 + (threadIdx.x & 63);
}

// movers per tile
__global__ __launch_bounds__(256) void k_rebin_count(const uint32_t* __restrict__ okeys,
                                                     const uint32_t* __restrict__ nkeys, int64_t n,
                                                     uint32_t* __restrict__ tile_cnt) {
  TileMovers t;
  tile_movers(okeys, nkeys, n, t);
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = t.total;
}

// movers, in current order, to (mk, mv, mo) = (new key, current index, old key)
__global__ __launch_bounds__(256) void k_rebin_compact(const uint32_t* __restrict__ okeys,
                                                       const uint32_t* __restrict__ nkeys, int64_t n,
                                                       const uint32_t* __restrict__ tile_off,
                                                       uint32_t* __restrict__ mk, uint32_t* __restrict__ mv,
                                                       uint32_t* __restrict__ mo) {
  TileMovers t;
  tile_movers(okeys, nkeys, n, t);
  const uint32_t base = tile_off[blockIdx.x];
  for (int r = 0; r < kSortItems; ++r)
    if (t.mover[r]) {
      mk[base + t.before[r]] = t.nk[r];
      mv[base + t.before[r]] = (uint32_t)tile_item(r);
      mo[base + t.before[r]] = t.ok[r];
    }
}

// first[b] = first index i < m with keys[i] >= b (m if none), for sorted keys
// and b = 0..n_bins, by binary search (one thread per bin, so the cost does
// not depend on how the keys are spread); m is read on the device
__global__ __launch_bounds__(256) void k_first_ge(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ m_dev,
                                                  int64_t n_bins, uint32_t* __restrict__ first) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b > n_bins) return;
  uint32_t lo = 0, hi = *m_dev;
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (keys[mid] < (uint32_t)b)
      lo = mid + 1;
    else
      hi = mid;
  }
  first[b] = lo;
}

// new offsets: elements with new key < b = (old key < b) - (movers whose old
// key < b) + (movers whose new key < b); also clears the per-bin count of
// movers that come from earlier bins
__global__ __launch_bounds__(256) void k_rebin_offsets(const uint32_t* __restrict__ ooff,
                                                       const uint32_t* __restrict__ out_before,
                                                       const uint32_t* __restrict__ in_start, int64_t n_bins,
                                                       uint32_t* __restrict__ noff, uint32_t* __restrict__ inc_before) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b > n_bins) return;
  noff[b] = ooff[b] - out_before[b] + in_start[b];
  inc_before[b] = 0u;
}

// Place the movers, sorted by (new key, current index): in bin b they follow
// the movers from earlier bins and, if they come from a later bin, the
// particles that stay in b.  Also counts, per bin, the movers from earlier bins.
__global__ __launch_bounds__(256) void k_rebin_movers(const uint32_t* __restrict__ sk, const uint32_t* __restrict__ sv,
                                                      const uint32_t* __restrict__ m_dev,
                                                      const uint32_t* __restrict__ ooff,
                                                      const uint32_t* __restrict__ noff,
                                                      const uint32_t* __restrict__ in_start,
                                                      const uint32_t* __restrict__ out_before,
                                                      uint32_t* __restrict__ inc_before, uint32_t* __restrict__ perm,
                                                      uint32_t* __restrict__ skeys) {
  const int64_t m = *m_dev;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < m; r += (int64_t)gridDim.x * 256) {
    const uint32_t b = sk[r], i = sv[r];
    const bool from_before = i < ooff[b];
    if (from_before) atomicAdd(&inc_before[b], 1u);
    const uint32_t stay = (ooff[b + 1] - ooff[b]) - (out_before[b + 1] - out_before[b]);
    const uint32_t pos = noff[b] + (uint32_t)(r - in_start[b]) + (from_before ? 0u : stay);
    perm[pos] = i;
    skeys[pos] = b;
  }
}

// Place the particles that stay in their bin b: after the movers from earlier
// bins, in their current order.
__global__ __launch_bounds__(256) void k_rebin_stayers(const uint32_t* __restrict__ okeys,
                                                       const uint32_t* __restrict__ nkeys, int64_t n,
                                                       const uint32_t* __restrict__ tile_off,
                                                       const uint32_t* __restrict__ ooff,
                                                       const uint32_t* __restrict__ noff,
                                                       const uint32_t* __restrict__ out_before,
                                                       const uint32_t* __restrict__ inc_before,
                                                       uint32_t* __restrict__ perm, uint32_t* __restrict__ skeys) {
  TileMovers t;
  tile_movers(okeys, nkeys, n, t);
  const uint32_t base = tile_off[blockIdx.x];
  for (int r = 0; r < kSortItems; ++r) {
    if (!t.valid[r] || t.mover[r]) continue;
    const uint32_t b = t.nk[r];
    const uint32_t i = (uint32_t)tile_item(r);
    const uint32_t movers_before = base + t.before[r];         // movers at positions < i
    const uint32_t out_in_seg = movers_before - out_before[b];  // of them, inside bin b's segment
    const uint32_t pos = noff[b] + inc_before[b] + (i - ooff[b]) - out_in_seg;
    perm[pos] = i;
    skeys[pos] = b;
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_keys(const double* X, int64_t n, int N, double invd, const BinGeom& g, uint32_t* keys,
                       int* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_keys<<<blocks_for(n, 256), 256, 0, s>>>(X, n, N, invd, g, keys, flag);
  return hipGetLastError();
}

hipError_t launch_locate(const double* X, int64_t n3, int N, double invd, int32_t* cell, double* off,
                         int* flag, hipStream_t s) {
  if (n3 == 0) return hipSuccess;
  k_locate<<<blocks_for(n3, 256), 256, 0, s>>>(X, n3, N, invd, cell, off, flag);
  return hipGetLastError();
}

size_t sort_hist_words(int64_t n) {
  int64_t n_tiles = (n + kTile - 1) / kTile;
  return (size_t)256 * (size_t)(n_tiles > 0 ? n_tiles : 1);
}

size_t scan_tmp_words(int64_t m) { return (size_t)((m + kScanBlock - 1) / kScanBlock + 1); }

// exclusive scan of a[0, m); with cnt != NULL the length is the histogram
// size of a sort of min(cap, *cnt) elements (m is then its upper bound)
static hipError_t scan_u32(uint32_t* a, int64_t m, uint32_t* tmp, const uint32_t* cnt, int64_t cap,
                           hipStream_t s) {
  if (m == 0) return hipSuccess;
  int64_t nb = (m + kScanBlock - 1) / kScanBlock;
  k_scan_reduce<<<(unsigned)nb, 256, 0, s>>>(a, m, tmp, cnt, cap);
  k_scan_top<<<1, 256, 0, s>>>(tmp, nb, cnt, cap);
  k_scan_apply<<<(unsigned)nb, 256, 0, s>>>(a, m, tmp, cnt, cap);
  return hipGetLastError();
}

hipError_t exclusive_scan_u32(uint32_t* a, int64_t m, uint32_t* tmp, hipStream_t s) {
  return scan_u32(a, m, tmp, nullptr, 0, s);
}

// Stable sort of keys.  Values: those in va if vals_in_va, else the input
// positions.  n_dev (optional) holds the element count on the device, n an
// upper bound.  On return *keys_sorted and *perm point into {ka, kb} / {va, vb}.
hipError_t radix_sort_keys(uint32_t* ka, uint32_t* kb, uint32_t* va, uint32_t* vb, int64_t n,
                           const uint32_t* n_dev, bool vals_in_va, int key_bits, uint32_t* hist,
                           uint32_t* tmp, uint32_t** keys_sorted, uint32_t** perm, hipStream_t s) {
  if (n == 0) {
    *keys_sorted = ka;
    *perm = va;
    return hipSuccess;
  }
  const int64_t n_tiles = (n + kTile - 1) / kTile;
  const int passes = key_bits <= 0 ? 1 : (key_bits + 7) / 8;
  const int bits = key_bits <= 0 ? 1 : (key_bits + passes - 1) / passes;
  const uint32_t mask = (1u << bits) - 1u;
  // pass p reads (kin, vin) and writes (kout, vout); the first pass takes the
  // input positions as values
  uint32_t *kin = ka, *kout = kb, *vin = vals_in_va ? va : nullptr, *vout = vals_in_va ? vb : va,
           *vspare = vb;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * bits;
    k_radix_hist<<<(unsigned)n_tiles, 256, 0, s>>>(kin, n, n_dev, shift, mask, hist, n_tiles);
    // with the count on the device, every kernel sizes the histogram from it
    hipError_t e = scan_u32(hist, 256 * n_tiles, tmp, n_dev, n, s);
    if (e != hipSuccess) return e;
    k_radix_scatter<<<(unsigned)n_tiles, 256, 0, s>>>(kin, vin, n, n_dev, shift, mask, bits, hist, n_tiles,
                                                      kout, vout);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* t = kin;
    kin = kout;
    kout = t;
    uint32_t* old_vin = vin;
    vin = vout;
    vout = old_vin ? old_vin : vspare;
  }
  *keys_sorted = kin;
  *perm = vin;
  return hipSuccess;
}

size_t rebin_block_words(int64_t n) { return (size_t)((n + kTile - 1) / kTile + 2); }

hipError_t rebin_incremental(const uint32_t* okeys, const uint32_t* ooff, const uint32_t* nkeys, int64_t n,
                             int64_t n_bins, int key_bits, const RebinScratch& w, uint32_t* perm, uint32_t* skeys,
                             uint32_t* noff, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t n_tiles = (n + kTile - 1) / kTile;
  hipError_t e;
  // movers per tile, exclusive scan: the last entry becomes the mover count m
  if ((e = launch_fill_i32((int*)(w.blockoff + n_tiles), 1, 0, s)) != hipSuccess) return e;
  k_rebin_count<<<(unsigned)n_tiles, 256, 0, s>>>(okeys, nkeys, n, w.blockoff);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = exclusive_scan_u32(w.blockoff, n_tiles + 1, w.scan_tmp, s)) != hipSuccess) return e;
  const uint32_t* m_dev = w.blockoff + n_tiles;
  // movers in current order (their old keys are then sorted), then sorted by new key
  k_rebin_compact<<<(unsigned)n_tiles, 256, 0, s>>>(okeys, nkeys, n, w.blockoff, w.mk_a, w.mv_a, w.mo);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_first_ge<<<blocks_for(n_bins + 1, 256), 256, 0, s>>>(w.mo, m_dev, n_bins, w.out_before);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint32_t *sk = nullptr, *sv = nullptr;
  if ((e = radix_sort_keys(w.mk_a, w.mk_b, w.mv_a, w.mv_b, n, m_dev, true, key_bits, w.hist, w.scan_tmp, &sk, &sv,
                           s)) != hipSuccess)
    return e;
  k_first_ge<<<blocks_for(n_bins + 1, 256), 256, 0, s>>>(sk, m_dev, n_bins, w.in_start);
  k_rebin_offsets<<<blocks_for(n_bins + 1, 256), 256, 0, s>>>(ooff, w.out_before, w.in_start, n_bins, noff,
                                                             w.inc_before);
  const int64_t mgrid = min((int64_t)4096, (n + 255) / 256);
  k_rebin_movers<<<(unsigned)mgrid, 256, 0, s>>>(sk, sv, m_dev, ooff, noff, w.in_start, w.out_before, w.inc_before,
                                                 perm, skeys);
  k_rebin_stayers<<<(unsigned)n_tiles, 256, 0, s>>>(okeys, nkeys, n, w.blockoff, ooff, noff, w.out_before,
                                                    w.inc_before, perm, skeys);
  return hipGetLastError();
}

// a fill of n ints (a kernel, so that a captured graph records no memset node)
__global__ __launch_bounds__(256) void k_fill_i32(int* __restrict__ p, int64_t n, int value) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = value;
}

hipError_t launch_fill_i32(int* p, int64_t n, int value, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_fill_i32<<<blocks_for(n, 256), 256, 0, s>>>(p, n, value);
  return hipGetLastError();
}

hipError_t launch_offsets(const uint32_t* skeys, int64_t n, int64_t n_bins, uint32_t* offsets,
                          hipStream_t s) {
  k_offsets<<<blocks_for(n + 1, 256), 256, 0, s>>>(skeys, n, n_bins, offsets);
  return hipGetLastError();
}

hipError_t gather3_f64(const double* in, const uint32_t* perm, int64_t n, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_gather3<double><<<blocks_for(n, 256), 256, 0, s>>>(in, perm, n, out);
  return hipGetLastError();
}

hipError_t gather3_f32(const float* in, const uint32_t* perm, int64_t n, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_gather3<float><<<blocks_for(n, 256), 256, 0, s>>>(in, perm, n, out);
  return hipGetLastError();
}

hipError_t gather_u32(const uint32_t* in, const uint32_t* perm, int64_t n, uint32_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_gather_u32<<<blocks_for(n, 256), 256, 0, s>>>(in, perm, n, out);
  return hipGetLastError();
}

hipError_t scatter_f64(const double* in, const uint32_t* idx, int64_t n, int width, double* out,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_scatterW<double><<<blocks_for(n, 256), 256, 0, s>>>(in, idx, n, width, out);
  return hipGetLastError();
}

hipError_t scatter_f32(const float* in, const uint32_t* idx, int64_t n, int width, float* out,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_scatterW<float><<<blocks_for(n, 256), 256, 0, s>>>(in, idx, n, width, out);
  return hipGetLastError();
}

}  // namespace ptk
